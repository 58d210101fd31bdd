"""Pins of the oracle's constant-density matter probability (prob_3nu_matter)
against what fixes it independently of its own algebra:
  * the Schroedinger propagation of the full three-flavour state
    (scipy.linalg.expm of the flavour-basis Hamiltonian with an arbitrary
    theta23 and CP phase, neither of which P_ee may depend on);
  * the vacuum limit (zero density) = the exact vacuum form;
  * the textbook two-flavour MSW formula for electron antineutrinos at
    theta13 = 0;
  * probability bounds, and complex-step derivatives against central
    differences (the complex-safe path the oracle's gradients take)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oscillation as O


def pmns(s2_t12, s2_t13, s2_t23, delta):
    s12, s13, s23 = np.sqrt([s2_t12, s2_t13, s2_t23])
    c12, c13, c23 = np.sqrt([1 - s2_t12, 1 - s2_t13, 1 - s2_t23])
    e = np.exp(1j * delta)
    r23 = np.array([[1, 0, 0], [0, c23, s23], [0, -s23, c23]], dtype=complex)
    u13 = np.array([[c13, 0, s13 / e], [0, 1, 0], [-s13 * e, 0, c13]], dtype=complex)
    r12 = np.array([[c12, s12, 0], [-s12, c12, 0], [0, 0, 1]], dtype=complex)
    return r23 @ u13 @ r12


def propagate(u, L, s2_t12, s2_t13, dm2_21, dm2_31, rho_ye, s2_t23=0.55, delta=1.2):
    """|<e| exp(-i H L) |e>|^2 for electron antineutrinos, H = M / 2E:
    M = U* diag(0, m21, m31) U^T - A e e^T (eV^2); the phase M L / 2E is
    2 PHASE_K M u in the oracle's units."""
    U = pmns(s2_t12, s2_t13, s2_t23, delta)
    m = np.diag([0.0, dm2_21 * O.DM2_21_UNIT, dm2_31 * O.DM2_31_UNIT])
    A = O.MATTER_A * rho_ye * (L / u)
    M = np.conj(U) @ m @ U.T - A * np.diag([1.0, 0.0, 0.0])
    S = expm(-2j * O.PHASE_K * u * M)
    return abs(S[0, 0]) ** 2


def test_matter_constant_from_its_definition():
    # sqrt(2) G_F N_e for rho Y_e = 1 g/cm^3: 7.63e-14 eV (standard figure)
    assert abs(O.MATTER_V_EV - 7.63e-14) < 0.01e-14
    assert abs(O.MATTER_A - 2e6 * O.MATTER_V_EV) < 1e-20


@pytest.mark.parametrize("dm2_31", [2.53, -2.45])
def test_zero_density_is_the_vacuum_form(dm2_31):
    rng = np.random.default_rng(1)
    u = rng.uniform(300.0, 40000.0, 2000)
    for s12, s13, m21 in ((0.307, 0.0218, 7.53), (0.28, 0.03, 6.9)):
        pm = O.prob_3nu_matter(u, 52500.0, s12, s13, m21, dm2_31, 0.0)
        pv = O.prob_3nu(u, s12, s13, m21, dm2_31)
        assert np.max(np.abs(pm - pv)) < 1e-13


@pytest.mark.parametrize("dm2_31", [2.53, -2.45])
@pytest.mark.parametrize("L,rho_ye", [(52500.0, 1.3), (1050.0, 1.3), (295e3, 1.4), (1.3e6, 1.7), (52500.0, 60.0)])
def test_matches_schroedinger_propagation(dm2_31, L, rho_ye):
    rng = np.random.default_rng(int(L) % 1000 + int(rho_ye * 10))
    for _ in range(12):
        e = rng.uniform(1.8, 12.0)
        u = L / e
        s12, s13, m21 = rng.uniform(0.25, 0.35), rng.uniform(0.015, 0.03), rng.uniform(6.5, 8.5)
        p = O.prob_3nu_matter(u, L, s12, s13, m21, dm2_31, rho_ye)
        q = propagate(u, L, s12, s13, m21, dm2_31, rho_ye)
        assert abs(p - q) < 2e-11, (u, L, p, q)
        # theta23 and the CP phase do not enter P_ee
        q2 = propagate(u, L, s12, s13, m21, dm2_31, rho_ye, s2_t23=0.41, delta=-2.0)
        assert abs(q2 - q) < 2e-11


def test_two_flavour_msw_limit():
    """theta13 = 0: P = 1 - sin^2(2 th_m) sin^2(PHASE_K dm2_m u) with, for
    antineutrinos, dm2_m = sqrt((m21 cos 2th + A)^2 + (m21 sin 2th)^2) and
    sin 2th_m = m21 sin 2th / dm2_m."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        L = rng.uniform(1e3, 3e5)
        e = rng.uniform(1.8, 12.0)
        rho = rng.uniform(0.5, 80.0)
        s12, m21 = rng.uniform(0.2, 0.4), rng.uniform(6.0, 9.0)
        u = L / e
        m = m21 * O.DM2_21_UNIT
        A = O.MATTER_A * rho * e
        c2, s2 = 1.0 - 2.0 * s12, 2.0 * np.sqrt(s12 * (1.0 - s12))
        dm = np.sqrt((m * c2 + A) ** 2 + (m * s2) ** 2)
        expect = 1.0 - (m * s2 / dm) ** 2 * np.sin(O.PHASE_K * dm * u) ** 2
        got = O.prob_3nu_matter(u, L, s12, 0.0, m21, 2.5, rho)
        assert abs(got - expect) < 1e-12


def test_bounds_and_complex_step_derivative():
    rng = np.random.default_rng(4)
    u = rng.uniform(300.0, 40000.0, 500)
    p = O.prob_3nu_matter(u, 52500.0, 0.307, 0.0218, 7.53, 2.53, 1.3)
    assert np.all(p >= -1e-15) and np.all(p <= 1 + 1e-15)
    args = [0.307, 0.0218, 7.53, 2.53]
    for j in range(4):
        h = 1e-30
        a = [complex(x) for x in args]
        a[j] += 1j * h
        cs = np.imag(O.prob_3nu_matter(u, 52500.0, *a, 1.3)) / h
        # five-point central difference (truncation error of order step^4)
        e = 1e-4 * abs(args[j])

        def f(k):
            a2 = list(args)
            a2[j] += k * e
            return O.prob_3nu_matter(u, 52500.0, *a2, 1.3)
        fd = (-f(2) + 8.0 * f(1) - 8.0 * f(-1) + f(-2)) / (12.0 * e)
        assert np.max(np.abs(cs - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))
