// FP64 sin/cos pairs for the oscillation phases, and bit helpers.
//
// sincos_fold: polynomial pair after reduction by pi (the matter form's
// phases and any other scattered use); sincos_tab: table-driven pair, fewer
// instructions per phase and more accurate, for the FP64 event folds, which
// hold the table in LDS.
//
// sincos_fold: reduction by pi (Cody & Waite 1980 style, two-constant split of pi with
// fused multiply-adds): q = nearest integer to x/pi, r = x - q*pi in
// [-pi/2, pi/2], sin x = (-1)^q sin r, cos x = (-1)^q cos r. The sign is a
// single XOR on the high words, so no quadrant swap is needed. The integer q
// is produced by the 1.5*2^52 rounding trick, which leaves q's parity in the
// lowest mantissa bit. Polynomials: see sincos_coeffs.hpp (|error| < 1e-12
// on [-pi/2, pi/2], far inside the 1e-9 agreement of the FP64 mode). Valid for
// |x| < 2^40 or so; phases in this engine stay below 1e4.
//
// The header compiles as host code too (plain C++), so the CPU test suite can
// check the routine against the C library.
#pragma once

#include <cstdint>
#include <cmath>

#include "sincos_coeffs.hpp"

#if defined(__HIPCC__)
#define NF_HD __host__ __device__ __forceinline__
#else
#define NF_HD inline
#endif

namespace nufold {

constexpr double INV_PI = 0.31830988618379067154;
constexpr double PI_HI = 3.141592653589793116;        // fl(pi)
constexpr double PI_LO = 1.2246467991473532072e-16;   // fl(pi - fl(pi))
constexpr double ROUND_MAGIC = 6755399441055744.0;    // 1.5 * 2^52

NF_HD uint64_t bits_of(double v) { return __builtin_bit_cast(uint64_t, v); }
NF_HD double from_bits(uint64_t b) { return __builtin_bit_cast(double, b); }

// sin(x), cos(x) for moderate |x|.
NF_HD void sincos_fold(double x, double& s, double& c) {
  const double qm = std::fma(x, INV_PI, ROUND_MAGIC);
  const double q = qm - ROUND_MAGIC;
  double r = std::fma(-q, PI_HI, x);
  r = std::fma(-q, PI_LO, r);
  const double r2 = r * r;
  constexpr int NS = sizeof(SIN_C) / sizeof(double), NC = sizeof(COS_C) / sizeof(double);
  double ps = SIN_C[NS - 1];
#pragma unroll
  for (int j = NS - 2; j >= 0; --j) ps = std::fma(ps, r2, SIN_C[j]);
  double pc = COS_C[NC - 1];
#pragma unroll
  for (int j = NC - 2; j >= 0; --j) pc = std::fma(pc, r2, COS_C[j]);
  const double sv = std::fma(r * r2, ps, r);
  const double cv = std::fma(r2, pc, 1.0);
  // (-1)^q: parity of q is the lowest mantissa bit of qm
  const uint64_t flip = bits_of(qm) << 63;
  s = from_bits(bits_of(sv) ^ flip);
  c = from_bits(bits_of(cv) ^ flip);
}

// sin and cos of 2 pi y / TAB_N from a table (the FP64 fold's form: y is the
// phase in table units, y = x TAB_PER_RAD). y = n + t with n the nearest
// integer (the 1.5*2^52 rounding trick leaves n mod 2^32 in the low word of
// the sum) and |t| <= 1/2, exact; sin and cos of A = 2 pi n / TAB_N come from
// tab (TAB_N correctly rounded (sin, cos) pairs, SINCOS_TAB), those of
// b = 2 pi t / TAB_N from short polynomials in t (sincos_coeffs.hpp, error
// below 2e-16), and the angle-sum formulas are taken with cos b - 1 so that
// the small terms are added last:
//   sin(A + b) = sin A + (sin A (cos b - 1) + cos A sin b),
//   cos(A + b) = cos A + (cos A (cos b - 1) - sin A sin b).
// |error| below 1e-15 for |y| < 2^40 given y; the rounding of y itself adds
// about 1.1e-16 |x| for a phase x in radians.
NF_HD void sincos_tab(double y, const double* tab, double& s, double& c) {
  const double qm = y + ROUND_MAGIC;
  const double n = qm - ROUND_MAGIC;
  const double t = y - n;
  const double t2 = t * t;
  const double sb = t * std::fma(t2, std::fma(t2, TAB_SIN_C[2], TAB_SIN_C[1]), TAB_SIN_C[0]);
  const double cm = t2 * std::fma(t2, TAB_COS_C[1], TAB_COS_C[0]);
  const unsigned i = (unsigned)bits_of(qm) & (unsigned)(TAB_N - 1);
  const double sa = tab[2 * i], ca = tab[2 * i + 1];
  s = std::fma(ca, sb, std::fma(sa, cm, sa));
  c = std::fma(-sa, sb, std::fma(ca, cm, ca));
}

}  // namespace nufold
