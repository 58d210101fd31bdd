// Exact three-flavour survival probability of electron antineutrinos in matter
// of constant electron density, and its derivatives by the four oscillation
// slots, per event (the matter step of the medium-baseline analysis, which the
// paper takes from GLoBES: "Description of the input model"; vacuum form:
// Eq. 10 and the exact three-flavour sum).
//
// In units of eV^2 (the Hamiltonian times 2E) the flavour-basis matrix is
//   M = U* diag(0, m21, m31) U^T - A e e^T,  A = 2 sqrt(2) G_F N_e E.
// M differs from its vacuum part M0 only in the ee entry, so its
// characteristic polynomial is the vacuum one plus A times that of the
// (mu, tau) block N of M0, which matter leaves alone:
//   det(l - M) = l (l - m21)(l - m31) + A Q(l),  Q(l) = det(l - N) = l^2 + q1 l + q0,
//   q1 = (M0)_ee - (m21 + m31),  (M0)_ee = s12 c13 m21 + s13 m31,
//   q0 = det N = c12 c13 m21 m31  (the vacuum eigenvector-eigenvalue identity at l = 0),
// with s_ij, c_ij the squared sines and cosines. Its roots l_i (three real
// ones: M is Hermitian) give the mixing in matter by the same identity,
// |U_ei|^2 = Q(l_i) / P'(l_i), and
//   P_ee = 1 - 4 sum_{i<j} |U_ei|^2 |U_ej|^2 sin^2(PHASE_K (l_i - l_j) u),  u = L/E.
// theta23 and the CP phase do not enter P_ee.
//
// Roots: the trigonometric form of Cardano's solution, then one Newton step
// each. Derivatives: by implicit differentiation at the roots,
//   dl = -(da l^2 + db l + dc) / P'(l),
//   d|U_ei|^2 = (dQ(l_i) - |U_ei|^2 dP'(l_i)) / P'(l_i)  (total derivatives,
//   through dl as well), with a, b, c the cubic's coefficients.
#pragma once

#include "fastmath.hpp"
#include "plan.hpp"

namespace nufold {

// P and dP/dslot for slots (sin^2 th12, sin^2 th13, dm2_21 [1e-5 eV^2],
// dm2_31 [1e-3 eV^2]); m21, m31 in eV^2; aL = MATTER_A_PER_MEV rho_ye L, so
// that A = aL / u.
__device__ __forceinline__ void matter_event(double u, double aL, double s12, double s13, double m21, double m31,
                                             double& P, double* dP) {
  constexpr double THIRD = 1.0 / 3.0;
  constexpr double HALF_SQRT3 = 0.86602540378443864676;
  constexpr double PK = 0.5 * TWO_PHASE_K;
  const double A = aL / u;
  const double c12 = 1.0 - s12, c13 = 1.0 - s13;
  const double sm = m21 + m31, pm = m21 * m31;
  const double ee = fma(s12 * c13, m21, s13 * m31);
  const double q1 = ee - sm;
  const double q0 = c12 * c13 * pm;
  const double a = A - sm, b = fma(A, q1, pm), c = A * q0;
  // depressed cubic t^3 + p t + q (l = t - a/3): p < 0 for distinct roots
  const double a3 = a * THIRD;
  const double p = fma(-a, a3, b);
  const double q = fma(a3 * a3, 2.0 * a3, fma(-a3, b, c));
  const double rr = 2.0 * sqrt(-p * THIRD);
  double x = 3.0 * q / (p * rr);  // (3q / 2p) sqrt(-3/p), as sqrt(-3/p) = 2 / rr
  x = fmin(1.0, fmax(-1.0, x));
  double sp, cp;
  sincos_fold(acos(x) * THIRD, sp, cp);
  double l[3] = {fma(rr, cp, -a3), fma(rr, fma(-0.5, cp, HALF_SQRT3 * sp), -a3),
                 fma(rr, fma(-0.5, cp, -HALF_SQRT3 * sp), -a3)};
  double rp[3], X[3];
  // Newton step; 1/P' is taken before the step (the root moves by far less
  // than the roots' separation, so 1/P' changes in its last bits only)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double y = l[k];
    const double f = fma(fma(y + a, y, b), y, c);
    rp[k] = 1.0 / fma(fma(3.0, y, 2.0 * a), y, b);
    y = fma(-f, rp[k], y);
    l[k] = y;
    X[k] = fma(y + q1, y, q0) * rp[k];
  }
  // pairs 01, 02, 12: sin^2 of the phase and sin of twice the phase
  constexpr int PI_[3] = {0, 0, 1}, PJ_[3] = {1, 2, 2};
  double s2[3], sn2[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double s, co;
    sincos_fold(PK * (l[PI_[r]] - l[PJ_[r]]) * u, s, co);
    s2[r] = s * s;
    sn2[r] = 2.0 * s * co;
  }
  P = 1.0 - 4.0 * (X[0] * X[1] * s2[0] + X[0] * X[2] * s2[1] + X[1] * X[2] * s2[2]);
  const double pku = PK * u;
#pragma unroll
  for (int j = 0; j < NSLOT; ++j) {
    const double d12 = j == 0 ? 1.0 : 0.0, d13 = j == 1 ? 1.0 : 0.0;
    const double d21 = j == 2 ? UNIT_1EM5 : 0.0, d31 = j == 3 ? UNIT_1EM3 : 0.0;
    const double dee = (d12 * c13 - s12 * d13) * m21 + s12 * c13 * d21 + d13 * m31 + s13 * d31;
    const double dsm = d21 + d31, dpm = d21 * m31 + m21 * d31;
    const double dq1 = dee - dsm;
    const double dq0 = -(d12 * c13 + c12 * d13) * pm + c12 * c13 * dpm;
    const double da = -dsm, db = fma(A, dq1, dpm), dc = A * dq0;
    double dl[3], dX[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double y = l[k];
      dl[k] = -fma(fma(da, y, db), y, dc) * rp[k];
      const double dQ = fma(dq1, y, dq0) + (2.0 * y + q1) * dl[k];
      const double dPp = fma(2.0 * da, y, db) + fma(6.0, y, 2.0 * a) * dl[k];
      dX[k] = (dQ - X[k] * dPp) * rp[k];
    }
    double g = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int i = PI_[r], k = PJ_[r];
      g += (dX[i] * X[k] + X[i] * dX[k]) * s2[r] + X[i] * X[k] * sn2[r] * pku * (dl[i] - dl[k]);
    }
    dP[j] = -4.0 * g;
  }
}

}  // namespace nufold
