// Oscillation coefficients and agent-scope memory helpers shared by the fold
// and bin-stage kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace nufold {

// Write-through store and coherent load at device (agent) scope: a value
// stored this way by one workgroup and followed by s_waitcnt(0) is visible to
// a load_agent of any other workgroup, on any XCD, that observes a later
// counter update; no cache write-back is needed.
__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of a double over the 64 lanes of a wavefront in a fixed order, returned
// to every lane: pairs, quads, half-rows and rows by DPP lane swaps (every lane
// of a group ends with the same group total), then the four row totals by two
// row broadcasts, read from lane 63. Needs all lanes active; uses no address
// registers.
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
__device__ __forceinline__ double wave_sum_fixed(double x) {
  x += dpp_swap<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_swap<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_swap<0x141>(x);  // row_half_mirror
  x += dpp_swap<0x140>(x);  // row_mirror: every lane holds its row total r_q
  // rows 1 and 3 add the total of the row below (r0 + r1, r2 + r3), then row
  // 3 adds row 1: lane 63 holds (r2 + r3) + (r0 + r1)
  {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x142, 0xa, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x142, 0xa, 0xf, false);
    x += __hiloint2double(hi, lo);
  }
  {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x143, 0xc, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x143, 0xc, 0xf, false);
    x += __hiloint2double(hi, lo);
  }
  return lane_value(x, 63);
}

// Inclusive prefix sum of a double over the 64 lanes of a wavefront in a
// fixed order: Hillis-Steele steps within each 16-lane row (row_shr 1, 2, 4,
// 8), then the row totals carried across rows (row_bcast 15 and 31).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_shift0(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_scan_incl(double x) {
  x += dpp_shift0<0x111, 0xf>(x);  // row_shr:1
  x += dpp_shift0<0x112, 0xf>(x);  // row_shr:2
  x += dpp_shift0<0x114, 0xf>(x);  // row_shr:4
  x += dpp_shift0<0x118, 0xf>(x);  // row_shr:8
  x += dpp_shift0<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_shift0<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Value of lane l ^ (1 << S) within each 16-lane row (S = 0..3): quad
// permutations for 1 and 2; for 4 and 8, a row shift left for the lanes whose
// bit S is clear and a row shift right for the others (DPP bank masks select
// the groups of four lanes each shift writes).
template <int S>
__device__ __forceinline__ int xor_lane_b32(int v) {
  static_assert(S >= 0 && S < 4, "row-local partners only");
  if constexpr (S == 0) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
  } else if constexpr (S == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
  } else if constexpr (S == 2) {
    const int t = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xf, 0x5, false);  // row_shl:4, lanes 0-3, 8-11
    return __builtin_amdgcn_update_dpp(t, v, 0x114, 0xf, 0xA, false);         // row_shr:4, lanes 4-7, 12-15
  } else {
    const int t = __builtin_amdgcn_update_dpp(0, v, 0x108, 0xf, 0x3, false);  // row_shl:8, lanes 0-7
    return __builtin_amdgcn_update_dpp(t, v, 0x118, 0xf, 0xC, false);         // row_shr:8, lanes 8-15
  }
}
template <int S>
__device__ __forceinline__ double xor_lane(double x) {
  const int lo = xor_lane_b32<S>(__double2loint(x));
  const int hi = xor_lane_b32<S>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// One step of a row-local reduce-scatter of NV values (NV a power of two):
// lane pairs l, l ^ (1 << S) exchange halves, the lane whose bit S is clear
// keeps the lower half, the other the upper half, and each adds its partner's
// copy of the half it keeps. With NV = 1 the pair simply adds.
template <int S, int NV>
__device__ __forceinline__ void rs_step(double* c, int lane) {
  if constexpr (NV == 1) {
    c[0] += xor_lane<S>(c[0]);
  } else {
    constexpr int H = NV / 2;
    const bool up = (lane >> S) & 1;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = up ? c[i + H] : c[i];
      const double send = up ? c[i] : c[i + H];
      c[i] = keep + xor_lane<S>(send);
    }
  }
}

// Reduce-scatter of NP values (1, 2, 4, 8 or 16) over each 16-lane row in a
// fixed order: log2(NP) halving steps, then plain pairwise steps. Returns, in
// lane l, the row total of value j = bit-reverse of the low log2(NP) bits of
// l (every lane with the same low bits holds the same total). 15 exchanges
// for 16 values instead of 16 separate reductions.
template <int NP>
__device__ __forceinline__ double row_reduce_scatter(double* c, int lane) {
  static_assert(NP == 1 || NP == 2 || NP == 4 || NP == 8 || NP == 16, "power of two up to 16");
  rs_step<0, NP>(c, lane);
  rs_step<1, (NP >= 2 ? NP / 2 : 1)>(c, lane);
  rs_step<2, (NP >= 4 ? NP / 4 : 1)>(c, lane);
  rs_step<3, (NP >= 8 ? NP / 8 : 1)>(c, lane);
  return c[0];
}

// Oscillation coefficient rows: row 0 gives S, rows 1..4 dS/d(slot j), each a
// linear combination of (W, M_1..M_NM), CF_STRIDE doubles per row.
// The parameter domain of the oscillation formula: finite slot values and,
// for Eq. 1 and the 3+1 form, sin^2(2 theta) < 1 (cos^2 theta from its square
// root). Exactly the cases in which osc_coefficients returns false.
__device__ inline bool osc_domain_ok(const OscPlan& o, const double* th) {
  bool ok = true;
  for (int j = 0; j < NSLOT; ++j) {
    const double v = o.slot_param[j] >= 0 ? th[o.slot_param[j]] : o.slot_value[j];
    ok = ok && isfinite(v);
    if (j == 0 && o.formula == FORM_EQ1) ok = ok && v < 1.0;
    if (j == 2 && o.formula == FORM_4NU) ok = ok && v < 1.0;
    if (o.formula == FORM_MATTER) {
      // mixing in [0, 1] (theta13 below pi/2), dm2_21 > 0 and dm2_31 != 0:
      // three distinct eigenvalues in matter
      if (j == 0) ok = ok && v >= 0.0 && v <= 1.0;
      if (j == 1) ok = ok && v >= 0.0 && v < 1.0;
      if (j == 2) ok = ok && v > 0.0;
      if (j == 3) ok = ok && v != 0.0;
    }
  }
  return ok;
}

__host__ __device__ inline int num_phases(int formula) { return formula == FORM_4NU ? 3 : 2; }

// Angular frequencies a (rad per m/MeV) of the computed phases x = a u:
//   eq1: ee, 21;  3nu: 21, 31;  4nu: 21, 31, 41.
// The fold and the coefficient rows both take them from here, so the FP32
// frequencies derived from them are bit-identical on both sides.
template <int FORM>
__device__ __forceinline__ void osc_freqs_form(const OscPlan& o, const double* th, double* a) {
  auto v = [&](int j) { return o.slot_param[j] >= 0 ? th[o.slot_param[j]] : o.slot_value[j]; };
  if constexpr (FORM == FORM_EQ1) {
    a[0] = TWO_PHASE_K * UNIT_1EM3 * v(1);  // dm2_ee
    a[1] = TWO_PHASE_K * UNIT_1EM5 * v(3);  // dm2_21
  } else if constexpr (FORM == FORM_3NU) {
    a[0] = TWO_PHASE_K * UNIT_1EM5 * v(2);  // dm2_21
    a[1] = TWO_PHASE_K * UNIT_1EM3 * v(3);  // dm2_31
  } else {
    a[0] = TWO_PHASE_K * UNIT_1EM5 * o.cst[1];  // dm2_21 (fixed)
    a[1] = TWO_PHASE_K * UNIT_1EM3 * v(1);      // dm2_31
    a[2] = TWO_PHASE_K * UNIT_1EM3 * v(3);      // dm2_41
  }
}
__device__ __forceinline__ void osc_freqs(const OscPlan& o, const double* th, double* a) {
  if (o.formula == FORM_EQ1) osc_freqs_form<FORM_EQ1>(o, th, a);
  else if (o.formula == FORM_3NU) osc_freqs_form<FORM_3NU>(o, th, a);
  else if (o.formula == FORM_4NU) osc_freqs_form<FORM_4NU>(o, th, a);
  // the matter form has no fixed frequencies
}

// FP32 frequency in revolutions per (m/MeV) used by the M32 fold: the phase
// of an event is fract(f u) with f = fp32_rev(a); the fold's moments are then
// those of the angular frequency 2 pi f instead of a.
__device__ __forceinline__ float fp32_rev(double a) {
  constexpr double INV_2PI = 0.15915494309189533577;
  return (float)(a * INV_2PI);
}

// First-order frequency correction of the M32 moments. With frequency a' in
// place of a, C(a) = C(a') - (a - a') Q(a') + O((a - a')^2 u^2) because
// dC/da = -Q, so S = sum_c cf_c M_c(a) becomes cf_Q -= (a - a') cf_C on every
// row. a - a' is at most 2^-24 a, so the neglected term is below 1e-11 of C
// at the phases of reactor baselines. Q itself keeps its first-order error
// (a - a') sum w u^2 cos, which only enters the derivative rows of dm2.
template <int FORM>
__device__ __forceinline__ void fp32_correction_form(const OscPlan& o, const double* th, double* cf) {
  constexpr double TWO_PI = 6.283185307179586477;
  constexpr int NPH = FORM == FORM_4NU ? 3 : 2;
  constexpr int NP = FORM == FORM_EQ1 ? 2 : FORM == FORM_3NU ? 3 : 6;  // (C, Q) pairs
  double a[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
  osc_freqs_form<FORM>(o, th, a);
#pragma unroll
  for (int q = 0; q < NPH; ++q) d[q] = a[q] - TWO_PI * (double)fp32_rev(a[q]);
  // frequency error of each pair (derived pairs by angle subtraction)
  double dp[6] = {d[0], d[1], d[1] - d[0], d[2], d[2] - d[0], d[2] - d[1]};
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    double* row = cf + CF_STRIDE * r;
#pragma unroll
    for (int q = 0; q < NP; ++q) row[1 + NP + q] -= dp[q] * row[1 + q];
  }
}
__device__ inline void fp32_frequency_correction(const OscPlan& o, const double* th, double* cf) {
  if (o.formula == FORM_EQ1) fp32_correction_form<FORM_EQ1>(o, th, cf);
  else if (o.formula == FORM_3NU) fp32_correction_form<FORM_3NU>(o, th, cf);
  else if (o.formula == FORM_4NU) fp32_correction_form<FORM_4NU>(o, th, cf);
}

__device__ inline bool osc_coefficients(const OscPlan& o, const double* th, double* cf) {
  double v[NSLOT];
  for (int j = 0; j < NSLOT; ++j) v[j] = o.slot_param[j] >= 0 ? th[o.slot_param[j]] : o.slot_value[j];
  for (int i = 0; i < CF_SIZE; ++i) cf[i] = 0.0;
  bool ok = true;
  for (int j = 0; j < NSLOT; ++j) ok = ok && isfinite(v[j]);
  double* r0 = cf;
  double* r1 = cf + CF_STRIDE;
  double* r2 = cf + 2 * CF_STRIDE;
  double* r3 = cf + 3 * CF_STRIDE;
  double* r4 = cf + 4 * CF_STRIDE;
  if (o.formula == FORM_EQ1) {
    // moments: 1 C_ee, 2 C_21, 3 Q_ee, 4 Q_21
    const double s = v[0], s12 = v[2];
    if (!(s < 1.0)) return false;
    const double r = sqrt(1.0 - s);
    const double c13sq = 0.5 * (1.0 + r);
    const double c4 = c13sq * c13sq;
    const double s2t12 = 4.0 * s12 * (1.0 - s12);
    const double A = c4 * s2t12;
    const double dA_ds = -s2t12 * c13sq / (2.0 * r);
    const double dA_ds12 = c4 * 4.0 * (1.0 - 2.0 * s12);
    const double aee = TWO_PHASE_K * UNIT_1EM3, a21 = TWO_PHASE_K * UNIT_1EM5;
    r0[0] = 1.0 - 0.5 * s - 0.5 * A; r0[1] = 0.5 * s; r0[2] = 0.5 * A;
    // d/d sin^2(2 th13)
    r1[0] = -0.5 - 0.5 * dA_ds; r1[1] = 0.5; r1[2] = 0.5 * dA_ds;
    // d/d dm2_ee
    r2[3] = -0.5 * s * aee;
    // d/d sin^2 th12
    r3[0] = -0.5 * dA_ds12; r3[2] = 0.5 * dA_ds12;
    // d/d dm2_21
    r4[4] = -0.5 * A * a21;
  } else if (o.formula == FORM_3NU) {
    // moments: 1 C_21, 2 C_31, 3 C_32, 4 Q_21, 5 Q_31, 6 Q_32
    const double s12 = v[0], s13 = v[1];
    const double c12 = 1.0 - s12, c13 = 1.0 - s13;
    const double K21 = 4.0 * c12 * s12 * c13 * c13;
    const double K31 = 4.0 * c12 * c13 * s13;
    const double K32 = 4.0 * s12 * c13 * s13;
    const double a21 = TWO_PHASE_K * UNIT_1EM5, a31 = TWO_PHASE_K * UNIT_1EM3;
    r0[0] = 1.0 - 0.5 * (K21 + K31 + K32);
    r0[1] = 0.5 * K21; r0[2] = 0.5 * K31; r0[3] = 0.5 * K32;
    const double d12[3] = {4.0 * (1.0 - 2.0 * s12) * c13 * c13, -4.0 * c13 * s13, 4.0 * c13 * s13};
    const double d13[3] = {-8.0 * c12 * s12 * c13, 4.0 * c12 * (1.0 - 2.0 * s13),
                           4.0 * s12 * (1.0 - 2.0 * s13)};
    r1[0] = -0.5 * (d12[0] + d12[1] + d12[2]);
    r2[0] = -0.5 * (d13[0] + d13[1] + d13[2]);
    for (int j = 0; j < 3; ++j) {
      r1[1 + j] = 0.5 * d12[j];
      r2[1 + j] = 0.5 * d13[j];
    }
    // d/d dm2_21: x21 grows, x32 = x31 - x21 shrinks
    r3[4] = -0.5 * K21 * a21; r3[6] = 0.5 * K32 * a21;
    // d/d dm2_31
    r4[5] = -0.5 * K31 * a31; r4[6] = -0.5 * K32 * a31;
  } else if (o.formula == FORM_MATTER) {
    // the fold sums S and its slot derivatives per event (moments 1..5)
    for (int r = 0; r < 5; ++r) cf[CF_STRIDE * r + 1 + r] = 1.0;
    return ok && osc_domain_ok(o, th);
  } else {
    // 3+1: |U_e1..4|^2 = c12 c13 c14, s12 c13 c14, s13 c14, s14 (squared sines
    // and cosines), P = 1 - sum_{i<j} K_ij sin^2(x_ji / 2), K_ij = 4 |U_ei|^2 |U_ej|^2.
    // moments: 1..6 C of the pairs 21, 31, 32, 41, 42, 43, then 7..12 their Q
    const double s12 = o.cst[0], s13 = v[0], X = v[2];
    if (!(X < 1.0)) return false;
    const double rt = sqrt(1.0 - X);
    const double s14 = 0.5 * (1.0 - rt), c14 = 0.5 * (1.0 + rt);
    const double c12 = 1.0 - s12, c13 = 1.0 - s13;
    const double U1 = c12 * c13 * c14, U2 = s12 * c13 * c14, U3 = s13 * c14, U4 = s14;
    // derivatives of |U_ei|^2 by sin^2 th13 and by sin^2(2 th14) (through sin^2 th14)
    const double g = 0.25 / rt;
    const double a1 = -c12 * c14, a2 = -s12 * c14, a3 = c14, a4 = 0.0;
    const double b1 = -c12 * c13 * g, b2 = -s12 * c13 * g, b3 = -s13 * g, b4 = g;
    double sK = 0.0, sd13 = 0.0, sd14 = 0.0, Kp[6];
    auto pair = [&](int q, double ui, double uj, double dai, double daj, double dbi, double dbj) {
      Kp[q] = 4.0 * ui * uj;
      const double k13 = 4.0 * (dai * uj + ui * daj);
      const double k14 = 4.0 * (dbi * uj + ui * dbj);
      r0[1 + q] = 0.5 * Kp[q];
      r1[1 + q] = 0.5 * k13;
      r3[1 + q] = 0.5 * k14;
      sK += Kp[q]; sd13 += k13; sd14 += k14;
    };
    pair(0, U1, U2, a1, a2, b1, b2);  // 21
    pair(1, U1, U3, a1, a3, b1, b3);  // 31
    pair(2, U2, U3, a2, a3, b2, b3);  // 32
    pair(3, U1, U4, a1, a4, b1, b4);  // 41
    pair(4, U2, U4, a2, a4, b2, b4);  // 42
    pair(5, U3, U4, a3, a4, b3, b4);  // 43
    r0[0] = 1.0 - 0.5 * sK;
    r1[0] = -0.5 * sd13;
    r3[0] = -0.5 * sd14;
    const double am = TWO_PHASE_K * UNIT_1EM3;
    // d/d dm2_31: x31 and x32 grow, x43 = x41 - x31 shrinks
    r2[7 + 1] = -0.5 * Kp[1] * am; r2[7 + 2] = -0.5 * Kp[2] * am; r2[7 + 5] = 0.5 * Kp[5] * am;
    // d/d dm2_41: x41, x42, x43 grow
    r4[7 + 3] = -0.5 * Kp[3] * am; r4[7 + 4] = -0.5 * Kp[4] * am; r4[7 + 5] = -0.5 * Kp[5] * am;
  }
  if (o.fp32_phase) fp32_frequency_correction(o, th, cf);
  return ok;
}

}  // namespace nufold
