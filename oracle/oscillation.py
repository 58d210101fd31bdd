"""Survival probabilities of reactor antineutrinos (oracle; test infrastructure).

Units: u = L/E in m/MeV; dm2_ee and dm2_31 in 1e-3 eV^2; dm2_21 in 1e-5 eV^2.
The oscillation phase Delta m^2 L / 4E (Eq. 1, natural units) is
PHASE_K * dm2[eV^2] * u with PHASE_K = 1 / (4 hbar c) expressed in
MeV / (eV^2 m), hbar c = 1.973269804593025e-7 eV m (exact SI-2019 constants).

All functions accept complex arguments so that complex-step derivatives pass
through them.
"""
import numpy as np

PHASE_K = 1.266932679039099
DM2_EE_UNIT = 1e-3
DM2_31_UNIT = 1e-3
DM2_21_UNIT = 1e-5
DM2_41_UNIT = 1e-3


def sin2_t13_from_sin2_2t13(s2_2t13):
    """sin^2(theta13) from sin^2(2 theta13), branch theta13 <= pi/4."""
    return 0.5 * (1.0 - np.sqrt(1.0 - s2_2t13))


def prob_eq1(u, s2_2t13, dm2_ee, s2_t12, dm2_21):
    """Short-baseline survival probability exactly as Eq. 1 prints it.

    P = 1 - sin^2(2 th13) sin^2(dm2_ee L/4E) - cos^4(th13) sin^2(2 th12) sin^2(dm2_21 L/4E).
    """
    s2_t13 = sin2_t13_from_sin2_2t13(s2_2t13)
    c4_t13 = (1.0 - s2_t13) ** 2
    s2_2t12 = 4.0 * s2_t12 * (1.0 - s2_t12)
    ph_ee = PHASE_K * (dm2_ee * DM2_EE_UNIT) * u
    ph_21 = PHASE_K * (dm2_21 * DM2_21_UNIT) * u
    return 1.0 - s2_2t13 * np.sin(ph_ee) ** 2 - c4_t13 * s2_2t12 * np.sin(ph_21) ** 2


def prob_3nu(u, s2_t12, s2_t13, dm2_21, dm2_31):
    """Exact vacuum three-flavour electron-antineutrino survival probability.

    P = 1 - 4|Ue1|^2|Ue2|^2 sin^2 D21 - 4|Ue1|^2|Ue3|^2 sin^2 D31 - 4|Ue2|^2|Ue3|^2 sin^2 D32,
    |Ue1|^2 = c12^2 c13^2, |Ue2|^2 = s12^2 c13^2, |Ue3|^2 = s13^2, dm2_32 = dm2_31 - dm2_21.
    This is the formula Eq. 10 rewrites for medium baselines (see prob_eq10).
    The sign of dm2_31 selects the ordering (positive: normal, negative: inverted).
    """
    c2_12 = 1.0 - s2_t12
    c2_13 = 1.0 - s2_t13
    ue1 = c2_12 * c2_13
    ue2 = s2_t12 * c2_13
    ue3 = s2_t13
    m21 = dm2_21 * DM2_21_UNIT
    m31 = dm2_31 * DM2_31_UNIT
    m32 = m31 - m21
    d21 = PHASE_K * m21 * u
    d31 = PHASE_K * m31 * u
    d32 = PHASE_K * m32 * u
    return (1.0 - 4.0 * ue1 * ue2 * np.sin(d21) ** 2
            - 4.0 * ue1 * ue3 * np.sin(d31) ** 2
            - 4.0 * ue2 * ue3 * np.sin(d32) ** 2)


def dm2_ee_from_3nu(s2_t12, dm2_21, dm2_31):
    """Eq. 2: dm2_ee = cos^2(th12)|dm2_31| + sin^2(th12)|dm2_32|, in units of 1e-3 eV^2."""
    m31 = dm2_31 * DM2_31_UNIT
    m32 = m31 - dm2_21 * DM2_21_UNIT
    return ((1.0 - s2_t12) * abs(m31) + s2_t12 * abs(m32)) / DM2_EE_UNIT


def prob_eq10(u, s2_t12, s2_t13, dm2_21, dm2_31):
    """Eq. 10, medium-baseline form, under the reading used throughout this project.

    The printed equation is garbled by text extraction; it is read as
      P = 1 - 1/2 sin^2(2th13) [1 - sqrt(1 - sin^2(2th12) sin^2 D21) cos(2 D_ee +- phi)]
            - sin^2(2th12) cos^4(th13) sin^2 D21,
      D_ab = dm2_ab L / 4E, dm2_ee from Eq. 2,
      phi = atan2(cos(2th12) sin D21, cos D21) - D21 cos(2th12)  (quadrant-correct arctan),
      + for normal ordering (dm2_31 > 0), - for inverted.
    Real arguments only (identity check against prob_3nu).
    """
    s2_2t12 = 4.0 * s2_t12 * (1.0 - s2_t12)
    c2t12 = 1.0 - 2.0 * s2_t12
    s2_2t13 = 4.0 * s2_t13 * (1.0 - s2_t13)
    c4_t13 = (1.0 - s2_t13) ** 2
    dee = dm2_ee_from_3nu(s2_t12, dm2_21, dm2_31)
    d21 = PHASE_K * dm2_21 * DM2_21_UNIT * u
    dee_ph = PHASE_K * dee * DM2_EE_UNIT * u
    phi = np.arctan2(c2t12 * np.sin(d21), np.cos(d21)) - d21 * c2t12
    sign = 1.0 if dm2_31 > 0 else -1.0
    amp = np.sqrt(1.0 - s2_2t12 * np.sin(d21) ** 2)
    return (1.0 - 0.5 * s2_2t13 * (1.0 - amp * np.cos(2 * dee_ph + sign * phi))
            - s2_2t12 * c4_t13 * np.sin(d21) ** 2)


def prob_two_flavour(u, s2_2t, dm2_ev2):
    """Textbook two-flavour survival probability 1 - sin^2(2th) sin^2(dm2 L/4E), dm2 in eV^2."""
    return 1.0 - s2_2t * np.sin(PHASE_K * dm2_ev2 * u) ** 2


def sin2_t14_from_sin2_2t14(s2_2t14):
    """sin^2(theta14) from sin^2(2 theta14), branch theta14 <= pi/4."""
    return 0.5 * (1.0 - np.sqrt(1.0 - s2_2t14))


def prob_4nu(u, s2_t12, s2_t13, dm2_21, dm2_31, s2_2t14, dm2_41):
    """Vacuum 3+1 electron-antineutrino survival probability (the model of the
    paper's sterile-neutrino searches, "Extensions of the framework"; the
    paper does not print it).

    P = 1 - 4 sum_{i<j} |Ue_i|^2 |Ue_j|^2 sin^2(dm2_ji L / 4E), i, j = 1..4, with
    the first row of U = R34 R24 R14 R23 R13 R12 (no CP phases):
    |Ue1|^2 = c12^2 c13^2 c14^2, |Ue2|^2 = s12^2 c13^2 c14^2, |Ue3|^2 = s13^2 c14^2,
    |Ue4|^2 = s14^2; dm2_41 in 1e-3 eV^2 (fit units), dm2_4j = dm2_41 - dm2_j1.
    """
    s2_t14 = sin2_t14_from_sin2_2t14(s2_2t14)
    c2_12, c2_13, c2_14 = 1.0 - s2_t12, 1.0 - s2_t13, 1.0 - s2_t14
    ue = [c2_12 * c2_13 * c2_14, s2_t12 * c2_13 * c2_14, s2_t13 * c2_14, s2_t14]
    m2 = [0.0, dm2_21 * DM2_21_UNIT, dm2_31 * DM2_31_UNIT, dm2_41 * DM2_41_UNIT]
    p = 1.0
    for i in range(4):
        for j in range(i + 1, 4):
            d = PHASE_K * (m2[j] - m2[i]) * u
            p = p - 4.0 * ue[i] * ue[j] * np.sin(d) ** 2
    return p


# Constant-density matter (next step of the medium-baseline analysis: the
# paper's JUNO-like fit takes matter effects from GLoBES, "Description of the
# input model"). The electron-antineutrino Hamiltonian, in units of 1/(2E) and
# eV^2, is M = U* diag(0, dm2_21, dm2_31) U^T - A e e^T with A = 2 sqrt(2) G_F
# N_e E. With N_e = rho Y_e N_A per cm^3 (rho in g/cm^3, one gram per mole of
# nucleons), G_F = 1.1663787e-5 GeV^-2, hbar c = 1.973269804593025e-14 GeV cm
# and N_A = 6.02214076e23 / mol:  sqrt(2) G_F N_e = V * rho Y_e with V in eV,
# and A = 2 V rho Y_e E = MATTER_A * rho Y_e * E[MeV] in eV^2.
GF_GEV2 = 1.1663787e-5
HBARC_GEV_CM = 1.973269804593025e-14
AVOGADRO = 6.02214076e23
MATTER_V_EV = np.sqrt(2.0) * GF_GEV2 * HBARC_GEV_CM ** 3 * AVOGADRO * 1e9  # eV per (g/cm^3)
MATTER_A = 2.0 * MATTER_V_EV * 1e6  # eV^2 per (g/cm^3 MeV)


def cubic_real_roots(a, b, c):
    """The three real roots of x^3 + a x^2 + b x + c (trigonometric form of
    Cardano's solution; requires three real roots). Works on complex inputs
    (complex-step derivatives) through numpy's analytic sqrt/arccos/cos."""
    p = b - a * a / 3.0
    q = 2.0 * a ** 3 / 27.0 - a * b / 3.0 + c
    r = 2.0 * np.sqrt(-p / 3.0)
    phi = np.arccos((3.0 * q / (2.0 * p)) * np.sqrt(-3.0 / p)) / 3.0
    return [r * np.cos(phi - 2.0 * np.pi * k / 3.0) - a / 3.0 for k in range(3)]


def prob_3nu_matter(u, L, s2_t12, s2_t13, dm2_21, dm2_31, rho_ye):
    """Exact three-flavour electron-antineutrino survival probability in matter
    of constant electron density rho_ye (g/cm^3 times electrons per nucleon).

    The eigenvalues l_i of M (eV^2) are the roots of its characteristic
    polynomial. M differs from the vacuum matrix M0 only in its ee entry, so
      det(l - M) = l (l - dm2_21)(l - dm2_31) + A Q(l),
    Q(l) = det(l - N) for the (mu, tau) block N of M0, which matter does not
    touch: Q(l) = l^2 + q1 l + q0, q1 = -(tr M0 - (M0)_ee), q0 = det N
    = |Ue1|^2 dm2_21 dm2_31 (vacuum eigenvector-eigenvalue identity at l = 0),
    (M0)_ee = |Ue2|^2 dm2_21 + |Ue3|^2 dm2_31. The mixing in matter follows from
    the same identity: |Ue_i^m|^2 = Q(l_i) / prod_{j != i} (l_i - l_j). Then
      P = 1 - 4 sum_{i<j} |Ue_i^m|^2 |Ue_j^m|^2 sin^2((l_i - l_j) L / 4E).
    theta23 and the CP phase drop out of P_ee (the rotations they belong to
    leave the electron row alone). u = L/E in m/MeV, L in m; units of the
    mass splittings as in prob_3nu.
    """
    c2_12 = 1.0 - s2_t12
    c2_13 = 1.0 - s2_t13
    m21 = dm2_21 * DM2_21_UNIT
    m31 = dm2_31 * DM2_31_UNIT
    A = MATTER_A * rho_ye * (L / u)
    ee = s2_t12 * c2_13 * m21 + s2_t13 * m31
    q1 = -(m21 + m31 - ee)
    q0 = c2_12 * c2_13 * m21 * m31
    lam = cubic_real_roots(-(m21 + m31) + A, m21 * m31 + A * q1, A * q0)
    x = []
    for i in range(3):
        den = 1.0
        for j in range(3):
            if j != i:
                den = den * (lam[i] - lam[j])
        x.append((lam[i] * lam[i] + q1 * lam[i] + q0) / den)
    p = 1.0
    for i in range(3):
        for j in range(i + 1, 3):
            p = p - 4.0 * x[i] * x[j] * np.sin(PHASE_K * (lam[i] - lam[j]) * u) ** 2
    return p
