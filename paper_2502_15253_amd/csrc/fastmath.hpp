// FP64 sin/cos pair for the fold's oscillation phases, and bit helpers.
//
// Reduction by pi (Cody & Waite 1980 style, two-constant split of pi with
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

}  // namespace nufold
