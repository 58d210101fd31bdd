// Bin stages, NLL and adjoint gradient of one model evaluation.
//
// Inputs per fine bin k of a dataset: Hs[k] = sum_s A_s S[s][k] (oscillated
// spectrum with source norms) and its derivatives with respect to the four
// oscillation slots, and S[s][k] per source. For a single evaluation the fold
// kernel has produced them; for a batch of fits each fit's workgroup first
// sums the fold's partial moments itself (phase A, one thread per segment,
// then per fine bin).
//
// Forward (paper, "Structure of the framework", steps 2 and 3; Eq. 3-6, 9):
//   H_k = Hs_k (1 + F_k),  m_k = H_k / w,
//   d_k = harmonic mean of m_{k-1}, m_k (ends: d_0 = m_0, d_K = m_{K-1}),
//   in fine bin k, t in [0, 1]: rho(t) = d_k (1-t) + d_{k+1} t + 6 (m_k - (d_k+d_{k+1})/2) t (1-t),
//   whose integral from the bin's lower edge is
//   P_k(t) = w [d_k (t - t^2/2) + d_{k+1} t^2/2 + 6 (m_k - (d_k+d_{k+1})/2)(t^2/2 - t^3/3)],
//   P_k(1) = H_k (area conserving). The analysis edge x_i maps to y_i = g(x_i),
//   g the inverse of f(E) = c0 + (1+c1) E + c2 E^2, in fine bin k_i at t_i.
//   The signal of analysis bin i is the integral of the spline between its
//   mapped edges, taken locally: with kk = k clamped to [0, K] and the piece
//   p = P_k(t) for an edge inside the fine range (0 outside),
//     s_i = sum_{k = kk_i}^{kk_{i+1} - 1} H_k + p_{i+1} - p_i,
//   which equals C(y_{i+1}) - C(y_i) for the cumulative C of the spline, so
//   no prefix sum over the fine bins is needed.
//   mu_i = s_i + sum_b R_b T_bi (1 + beta_bi),  NLL += mu - n + n ln(n/mu)  (n = 0: mu),
//   then the prior rows.
//
// Reverse pass (exact adjoint; replaces numerical gradients), with
// lambda_i = dNLL/dmu_i = 1 - n_i/mu_i:
//   background rates and shapes from lambda_i directly;
//   energy scale: ds_i/dc = rho(t_{i+1}) dy_{i+1}/dc - rho(t_i) dy_i/dc,
//     dy/dc_j = -(1, y, y^2)_j / f'(y);
//   fine bin k gathers lambda of the one analysis bin that covers it whole
//   (dH direct) and, from the edges inside fine bins k-1, k, k+1 (weights
//   lambda_{j-1} - lambda_j), the adjoints of m_k, d_k and d_{k+1}; d depends
//   on the neighbouring m by the harmonic mean;
//   lambda_H -> flux modes (lambda_F = lambda_H Hs), and lambda_Hs =
//   lambda_H (1 + F) -> source norms (sum_k lambda_Hs S[s][k]) and, through the
//   fold's forward-mode derivative rows, the oscillation parameters.
//
// Work per dataset, one workgroup: a parameter pass (1 + F per fine bin,
// mapped edges and backgrounds, read straight from global memory while the
// fold's rows are being copied into LDS), one pass over the analysis bins, one
// over the fine bins, one block reduction of every summed gradient, one pass
// over the flux modes and source norms: four barriers besides the reduction's.
//
// All arithmetic is FP64. Sums over threads are taken in a fixed order; the
// few gradient entries that several threads of one pass can reach (a norm
// shared by sources, a parameter with two prior rows) use LDS atomic adds,
// which only affects the last bits.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <algorithm>

#include "kernels.hpp"
#include "osc.hpp"
#include "stages.hpp"

namespace nufold {

template <int NT>
struct Lds {
  double* th;     // P     parameters
  double* grad;   // P
  double* coef;   // CF_SIZE
  DsPlan* dsl;    // D dataset plans
  double* red;    // block reduction scratch (red_doubles)
  double* Hk;     // K     H_k = Hs_k (1 + F_k)
  double* mk;     // K     m_k = H_k / w
  double* LF;     // K     lambda_F
  double* LHs;    // K     lambda_Hs (read back only for sources past the first sixteen)
  double* Hs;     // K     the oscillated spectrum with source norms (fold row 0)
  double* Ss;     // S K   per-source spectra
  double* lam;    // Nb    observed counts, then lambda_mu
  double* eP;     // E     spline integral from its fine bin's lower edge to the mapped edge (0 outside)
  double* eR;     // E     spline density at the mapped edge over f'(y) (0 outside)
  double* st;     // the LDS part of the dataset's static blob (flux modes, norm lists, background parameters)
  double* fit;    // minimiser scratch
  // the dataset's block of the parameter pass (pre_layout), in one region:
  double* F1;     // K     1 + F_k
  double* Bv;     // Nb    background expectation
  double* bkr;    // B Nb  dmu_i/dR_b
  double* bks;    // B Nb  dmu_i/dbeta_bi
  double* eT;     // E     t of each mapped edge
  double* eY;     // E     y of each mapped edge
  double* eQ;     // E     1 / f'(y) at the mapped edge
  int* ek;        // E     fine bin of each mapped edge: -1 below y_0, K at or above y_K
  // pointers into st:
  int* bki;       // B Nb  shape parameter of (b, i), or -1
  int* brt;       // B     rate parameter of each background, or -1
  // the prior rows and flags, in one region (the layout of the parameter
  // pass's global block):
  double* prv;    // NR    gradient contribution of each prior row
  int* pri;       // NR    parameter of each prior row
  double* misc;   // 2 + D the parameter pass's prior NLL and domain flags (single evaluation)
  int* first;     // K + 2 first[q] = first edge whose clamped fine bin is >= q (E: none)
  int* flag;      // 2
  // region bases: copies land at their source's alignment modulo 16 bytes
  double *thb, *Ssb, *lamb, *dsb;
};

// Points the per-dataset arrays at the dataset's layout inside their regions.
template <int NT>
__device__ __forceinline__ void point_dataset(Lds<NT>& L, const DsPlan& ds, const BlobLayout& BL) {
  const PreLayout PL = pre_layout(ds.K, ds.Nb, ds.nbkg);
  L.F1 = L.dsb + PL.F1;
  L.Bv = L.dsb + PL.B;
  L.bkr = L.dsb + PL.bkr;
  L.bks = L.dsb + PL.bks;
  L.eT = L.dsb + PL.et;
  L.eY = L.dsb + PL.ey;
  L.eQ = L.dsb + PL.eq;
  L.ek = reinterpret_cast<int*>(L.dsb + PL.ek);
  L.bki = reinterpret_cast<int*>(L.st + BL.shp);
  L.brt = reinterpret_cast<int*>(L.st + BL.brt);
}

template <int NT>
__device__ Lds<NT> carve(double* base, const DevPlan& p) {
  Lds<NT> L;
  const int K = p.max_K, E = p.max_Nb + 1, Nb = p.max_Nb;
  // regions filled by direct copies start at 16-byte boundaries (even
  // offsets); those whose sources have no fixed alignment get one double of
  // slack
  auto al = [](double* x) { return x + (reinterpret_cast<uintptr_t>(x) & 8 ? 1 : 0); };
  double* q = al(base);
  L.dsb = q; q += p.max_pre;
  L.st = q; q += p.max_blob;
  q = al(q);
  L.prv = q; q += p.NR;
  L.pri = reinterpret_cast<int*>(q); q += (p.NR + 1) / 2;
  L.misc = q; q += 2 + p.D;
  q = al(q);
  L.dsl = reinterpret_cast<DsPlan*>(q); q += p.D * DSPLAN_DOUBLES;
  L.thb = q; q += p.P + 1;
  L.th = L.thb;
  q = al(q);
  L.Ssb = q; q += p.max_S * K + 1;
  L.Ss = L.Ssb;
  q = al(q);
  L.lamb = q; q += Nb + 1;
  L.lam = L.lamb;
  q = al(q);
  L.Hs = q; q += K;
  L.grad = q; q += p.P;
  L.coef = q; q += CF_SIZE;
  L.red = q; q += red_doubles(NT);
  L.Hk = q; q += K;
  L.mk = q; q += K;
  L.LF = q; q += K;
  L.LHs = q; q += K;
  L.eP = q; q += E;
  L.eR = q; q += E;
  L.fit = q; q += fit_lds_doubles(p.P, p.fit_m);
  int* r = reinterpret_cast<int*>(q);
  L.first = r; r += K + 2;
  L.flag = r;
  return L;
}

// Sum of N values (N <= 32) over the workgroup; every thread gets the
// totals, summed in a fixed order. Each wavefront reduce-scatters the values,
// sixteen at a time, over its 16-lane rows (padded to a power of two), one
// lane per (value, row) writes its row total to red[j * 4 NW + row], then
// four lanes per value each add a quarter of the 4 NW row totals of value j
// in order and combine them by two quad exchanges. The totals sit at
// red[32 * 4 NW + j], past every partial, so back-to-back calls do not
// overlap.
template <int NP>
__device__ __forceinline__ void row_partials(const double* v, int n, double* red, int R, int wid, int lane) {
  constexpr int LG = NP == 1 ? 0 : NP == 2 ? 1 : NP == 4 ? 2 : NP == 8 ? 3 : 4;
  double c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) c[j] = j < n ? v[j] : 0.0;
  const double x = row_reduce_scatter<NP>(c, lane);
  if (((lane & 15) >> LG) == 0) {
    int j = 0;
    if constexpr (LG > 0) j = (int)(__builtin_bitreverse32((unsigned)lane) >> (32 - LG));
    red[j * R + wid * 4 + (lane >> 4)] = x;
  }
}

template <int NT, int N>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  constexpr int NW = NT / 64, R = 4 * NW;
  static_assert(N >= 1 && N <= 32, "reduction scratch too small");
  constexpr int N1 = N < 16 ? N : 16, N2 = N - N1;
  constexpr int P1 = N1 <= 1 ? 1 : N1 <= 2 ? 2 : N1 <= 4 ? 4 : N1 <= 8 ? 8 : 16;
  constexpr int P2 = N2 <= 1 ? 1 : N2 <= 2 ? 2 : N2 <= 4 ? 4 : N2 <= 8 ? 8 : 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  row_partials<P1>(v, N1, red, R, wid, lane);
  if constexpr (N2 > 0) row_partials<P2>(v + 16, N2, red + 16 * R, R, wid, lane);
  __syncthreads();
  if (tid < 4 * N) {
    const int q = tid >> 2, part = tid & 3;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < R / 4; ++k) s += red[q * R + part * (R / 4) + k];
    s += dpp_swap<0xB1>(s);  // quad_perm [1,0,3,2]
    s += dpp_swap<0x4E>(s);  // quad_perm [2,3,0,1]
    if (part == 0) red[32 * R + q] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = red[32 * R + j];
}


}  // namespace nufold
#include "minimize.hpp"
namespace nufold {

// Asynchronous copies from global memory straight into LDS (global_load_lds:
// no registers, every load in flight at once). dma_lds<NT, B> moves nbytes (a
// multiple of B) in chunks of 64 B bytes, one per wavefront in turn starting
// with wavefront rot (so that many small copies spread over the waves), lane l
// the B bytes at l B of its chunk; B = 16 needs 16-byte aligned source and
// destination. The caller waits (s_waitcnt) and synchronises before reading.
typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef __attribute__((address_space(1))) const void* global_cvoid_ptr;
template <int NT, int B>
__device__ __forceinline__ void dma_lds(char* dst, const char* src, int nbytes, int rot = 0) {
  static_assert(B == 4 || B == 16, "4- or 16-byte units");
  constexpr int NW = NT / 64;
  static_assert((NW & (NW - 1)) == 0, "a power-of-two number of waves");
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // chunk addresses in scalar registers
  const int nunits = nbytes / B;
  for (int c = (wid - rot) & (NW - 1); c * 64 < nunits; c += NW) {
    const int idx = c * 64 + lane;
    if (idx < nunits) {
      const global_cvoid_ptr g = (global_cvoid_ptr)(src + (size_t)B * idx);
      const lds_void_ptr l = (lds_void_ptr)(dst + (size_t)(64 * B) * c);
      if constexpr (B == 16) __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
      else __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
    }
  }
}
// n doubles: 16-byte units when source and destination share their
// alignment modulo 16 (a leading or trailing double by 4-byte units), else
// 4-byte units throughout.
template <int NT>
__device__ __forceinline__ void copy_to_lds(double* dst, const double* src, int n, int rot = 0) {
  char* d = reinterpret_cast<char*>(dst);
  const char* s = reinterpret_cast<const char*>(src);
  const unsigned da = (unsigned)(uintptr_t)(lds_void_ptr)d;
  const unsigned sa = (unsigned)(uintptr_t)s;
  if (((da ^ sa) & 15u) != 0 || n < 4) {
    dma_lds<NT, 4>(d, s, 8 * n, rot);
    return;
  }
  const int head = (sa & 15u) ? 1 : 0;
  const int body = (n - head) & ~1;
  const int tail = n - head - body;
  if (head) dma_lds<NT, 4>(d, s, 8, rot + 1);
  dma_lds<NT, 16>(d + 8 * head, s + 8 * head, 8 * body, rot);
  if (tail) dma_lds<NT, 4>(d + 8 * (head + body), s + 8 * (head + body), 8, rot + 2);
}


// ---------------------------------------------------------------- inputs
// The fold's rows were written by the fold kernel (single evaluation: plain
// loads) or by this workgroup's phase A (batched: coherent agent-scope loads).
struct FineRows { // adjoint: the oscillation-slot derivative rows
  double g[4];
};

__device__ __forceinline__ double ld(const double* p, int coherent) { return coherent ? load_agent(p) : *p; }

__device__ __forceinline__ void load_rows(const EvalIO& io, const DsPlan& ds, int k, FineRows& r) {
  const int K = ds.K, co = io.fused ? 0 : 1;
  const double* b = io.bin + 6 * (int64_t)ds.kt0;
#pragma unroll
  for (int j = 0; j < 4; ++j) r.g[j] = ld(b + (j + 1) * K + k, co);
}

// LDS destination for a copy from src into a region with one double of
// slack: the same alignment modulo 16 bytes as the source.
__device__ __forceinline__ double* matched(double* region, const double* src) {
  return region + ((reinterpret_cast<uintptr_t>(src) >> 3) & 1);
}

// Single evaluation: a dataset's inputs reach LDS by direct copies in two
// rounds. The early round -- the background parameters of its static blob,
// its block of the fold launch's parameter pass (1 + F per fine bin,
// backgrounds and their factors, mapped edges), the fold's row 0 and the
// observed counts -- is issued together and waited for (s_waitcnt, then a
// barrier) before the edge and analysis-bin passes. The late round -- the
// flux modes by column, the norm lists and the per-source spectra, read only
// by the gradient's passes -- is issued after that barrier and lands while
// those passes run (waited for at the barrier after the analysis bins). A
// wavefront's issue of direct copies stalls while the compute unit's memory
// pipeline is busy, so every wavefront takes a share (one wavefront issuing
// the whole late round held the edge pass up by 2 us).
template <int NT>
__device__ __forceinline__ void gather_early(const DevPlan& p, const EvalIO& io, Lds<NT>& L, const DsPlan& ds,
                                             const BlobLayout& BL, int want_nll) {
  const double* dat = io.data + ds.data;
  L.lam = matched(L.lamb, dat);
  copy_to_lds<NT>(L.dsb, io.pre + ds.pre0, pre_layout(ds.K, ds.Nb, ds.nbkg).total, 0);
  copy_to_lds<NT>(L.st, p.dpool + ds.blob, BL.early, 3);
  copy_to_lds<NT>(L.Hs, io.bin + 6 * (int64_t)ds.kt0, ds.K, 5);
  if (want_nll) copy_to_lds<NT>(L.lam, dat, ds.Nb, 7);  // observed counts, replaced by lambda in (d)
}
template <int NT>
__device__ __forceinline__ void gather_late(const DevPlan& p, const EvalIO& io, Lds<NT>& L, const DsPlan& ds,
                                            const BlobLayout& BL) {
  const double* ss = io.Sseg + ds.seg0;
  L.Ss = matched(L.Ssb, ss);
  copy_to_lds<NT>(L.st + BL.early, p.dpool + ds.blob + BL.early, BL.hpart - BL.early, 0);
  copy_to_lds<NT>(L.Ss, ss, ds.S * ds.K, 4);
}

// A dataset plan read from LDS in one batch, every 32-bit word made
// wave-uniform (scalar registers).
__device__ __forceinline__ DsPlan uniform_plan(const DsPlan* src) {
  static_assert(sizeof(DsPlan) % 16 == 0, "DsPlan is read in 16-byte units");
  DsPlan r;
  const int4* s = reinterpret_cast<const int4*>(src);
  int* o = reinterpret_cast<int*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(DsPlan) / 16); ++i) {
    const int4 v = s[i];
    o[4 * i] = __builtin_amdgcn_readfirstlane(v.x);
    o[4 * i + 1] = __builtin_amdgcn_readfirstlane(v.y);
    o[4 * i + 2] = __builtin_amdgcn_readfirstlane(v.z);
    o[4 * i + 3] = __builtin_amdgcn_readfirstlane(v.w);
  }
  return r;
}

// Serial bin stages, NLL, priors and adjoint of one evaluation; returns the
// NLL (+inf when out of domain) to every thread; the gradient is in L.grad.
// On entry the parameters are in LDS (waited for and synchronised), the
// gradient and flag are clear, the prior rows are in L.prv / L.pri, and
// prior_e is this thread's part of the prior NLL (batched; a single
// evaluation takes the prior NLL from L.misc, and dataset 0's early inputs
// are in LDS already).
//
// Per dataset: (a, b) inputs -- single evaluation: every one by direct copies
// in two rounds (gather_early, gather_late); batched: the static blob's LDS
// part by direct copies, then a parameter pass: 1 + F per fine bin, the background
// expectation and its factors per analysis bin, the mapped edges; (c) H and m
// per fine bin, per mapped edge the densities, the spline integral up to the
// edge and its density, and the edge-index table; (d) per analysis bin the
// signal, expectation, deviance, lambda and the background and energy-scale
// sums; (e) per fine bin the adjoint; one block reduction of every summed
// gradient; (f) source norms, flux modes, priors.
constexpr int ACC_SRC = 16;  // sources reduced together with the other sums
template <int NT>
__device__ double serial_stages(const DevPlan& p, const EvalIO& io, Lds<NT>& L, double prior_e, int want_nll,
                                int want_grad) {
  const int tid = threadIdx.x;
  double nll_total = 0.0;  // identical in every thread (block sums broadcast)

#pragma unroll 1
  for (int dloop = 0; dloop < p.D; ++dloop) {
    // an opaque copy of the dataset index: nothing derived from the dataset
    // is hoisted out of the loop (where it would hold registers throughout)
    int d = dloop;
    asm volatile("" : "+s"(d));
    const DsPlan ds = uniform_plan(L.dsl + d);
    const int K = ds.K, Nb = ds.Nb, S = ds.S, E = Nb + 1, M = ds.M, NB = ds.nbkg;
    const double wf = ds.wf, iwf = 1.0 / wf, y0 = ds.y0, yK = ds.y0 + ds.wf * K;
    const BlobLayout BL = blob_layout(E, NB, Nb, ds.nnz, M, S, ds.nl, K, ds.fw);
    const double* blob = p.dpool + ds.blob;

    // ---- (a) inputs and (b) parameter pass
    point_dataset<NT>(L, ds, BL);
    if (io.pre) {
      // single evaluation: everything by direct copies (dataset 0's early
      // round was issued at kernel start, together with the parameters)
      if (d > 0) {
        gather_early<NT>(p, io, L, ds, BL, want_nll);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
      }
      if (want_grad) gather_late<NT>(p, io, L, ds, BL);
    } else {
      copy_to_lds<NT>(L.st, blob, BL.hpart);
      // written by this workgroup's phase A: coherent loads, then LDS stores
      for (int j = tid; j < S * K; j += NT) L.Ss[j] = load_agent(io.Sseg + ds.seg0 + j);
      const double* hsrow = io.bin + 6 * (int64_t)ds.kt0;
      const double c0 = pval(L.th, ds.cidx[0], 0.0);
      const double c2 = pval(L.th, ds.cidx[2], 0.0);
      const double bb = 1.0 + pval(L.th, ds.cidx[1], 0.0);
      if (tid == 0 && !map_ok(bb, c2, y0, yK)) atomicOr(&L.flag[0], ST_DOMAIN);
      if (d == 0) {
        for (int i = tid; i < p.P; i += NT)
          if (!isfinite(L.th[i])) atomicOr(&L.flag[0], ST_DOMAIN);
        if (tid == 0 && !osc_domain_ok(p.osc, L.th)) atomicOr(&L.flag[0], ST_DOMAIN);
      }
      for (int k = tid; k < K; k += NT) {
        L.F1[k] = flux_factor(L.th, blob, BL, ds.fw, k);
        L.Hs[k] = load_agent(hsrow + k);
      }
      for (int i = tid; i < Nb; i += NT) {
        L.Bv[i] = background(L.th, blob, BL, NB, Nb, i, L.bkr + i, L.bks + i);
        if (want_nll) L.lam[i] = io.data[ds.data + i];  // the observed count, replaced by lambda in (d)
      }
      for (int e = tid; e < E; e += NT) {
        const MappedEdge m = map_edge(blob[BL.edges + e], c0, bb, c2, y0, yK, wf, iwf, K);
        L.ek[e] = m.k;
        L.eT[e] = m.t;
        L.eY[e] = m.y;
        L.eQ[e] = m.ifp;
      }
      // the blob's copy (background parameters, read from (d) on) has landed
      // once every wave has waited for its own and passed the barrier
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }

    // the adjoint's inputs of this thread's fine bin, in flight during (c) and (d)
    FineRows rows;
    if (tid < K && want_grad) load_rows(io, ds, tid, rows);

    // m_k = H_k / w with H_k = Hs_k (1 + F_k), in the one order that (c)
    // and the later passes (through L.mk) share
    auto mof = [&](int k) { return L.Hs[k] * L.F1[k] * iwf; };
    auto dens = [&](int k) {  // d_k, 0 <= k <= K
      if (k == 0) return mof(0);
      if (k == K) return mof(K - 1);
      const double a = mof(k - 1), b = mof(k);
      return (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0;
    };
    auto clampK = [&](int k) { return k < 0 ? 0 : (k > K ? K : k); };

    // ---- (c) H and m per fine bin; per mapped edge the spline integral from
    // its fine bin's lower edge, P_k(t), and the density there over f'(y);
    // edge-index table
    if (io.pre && tid == 0 && (L.misc[2 + d] != 0.0 || (d == 0 && L.misc[1] != 0.0)))
      atomicOr(&L.flag[0], ST_DOMAIN);
    for (int k = tid; k < K; k += NT) {
      const double H = L.Hs[k] * L.F1[k];
      L.Hk[k] = H;
      L.mk[k] = H * iwf;
    }
    for (int e = tid; e < E; e += NT) {
      const int k = L.ek[e];
      double piece = 0.0, rr = 0.0;
      if (k >= 0 && k < K) {
        const double t = L.eT[e];
        const double dl = dens(k), dh = dens(k + 1), mk = mof(k);
        const double q = 0.5 * t * t - t * t * t * (1.0 / 3.0), c = 6.0 * (mk - 0.5 * (dl + dh));
        piece = wf * (dl * (t - 0.5 * t * t) + dh * 0.5 * t * t + c * q);
        const double rho = dl * (1.0 - t) + dh * t + c * t * (1.0 - t);
        rr = rho * L.eQ[e];
      }
      L.eP[e] = piece;
      L.eR[e] = rr;
      // first[q] = e for kk_{e-1} < q <= kk_e (edge 0 from q = 0); the top
      // edge's thread also writes the entries past it
      const int kk = clampK(k);
      const int kp = e > 0 ? clampK(L.ek[e - 1]) : -1;
      for (int q = kp + 1; q <= kk; ++q) L.first[q] = e;
      if (e == E - 1)
        for (int q = kk + 1; q <= K + 1; ++q) L.first[q] = E;
    }
    __syncthreads();

    // acc: 0 NLL, 1..3 energy scale c0..c2, 4..7 oscillation slots,
    // 8..15 background rates, 16..31 the first sixteen source norms
    double acc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] = 0.0;

    // ---- (d) analysis bins: signal, expectation, deviance, lambda_mu,
    // background and energy-scale gradients
    for (int i = tid; i < Nb; i += NT) {
      const int k0 = clampK(L.ek[i]), k1 = clampK(L.ek[i + 1]);
      double s = 0.0;
      for (int k = k0; k < k1; ++k) s += L.Hk[k];
      s += L.eP[i + 1];
      s -= L.eP[i];
      const double mu = s + L.Bv[i];
      if (io.mu_out) io.mu_out[ds.bins0 + i] = mu;
      double lam = 0.0;
      if (want_nll) {
        const double n = L.lam[i];
        if (!(mu > 0.0)) atomicOr(&L.flag[0], ST_DOMAIN);
        acc[0] += (n > 0.0) ? (mu - n + n * log(n / mu)) : mu;
        lam = 1.0 - n / mu;
        if (want_grad) {
#pragma unroll
          for (int b = 0; b < MAX_BKG; ++b)
            if (b < NB) {
              acc[8 + b] += lam * L.bkr[b * Nb + i];
              const int sp = L.bki[b * Nb + i];
              if (sp >= 0) atomicAdd(&L.grad[sp], lam * L.bks[b * Nb + i]);
            }
          // ds_i/dc_j = -rho_b (1, y_b, y_b^2)_j / f'(y_b) + rho_a (1, y_a, y_a^2)_j / f'(y_a)
          const double ya = L.eY[i], yb = L.eY[i + 1];
          const double la = lam * L.eR[i], lb = lam * L.eR[i + 1];
          acc[1] += la - lb;
          acc[2] += la * ya - lb * yb;
          acc[3] += la * ya * ya - lb * yb * yb;
        }
      }
      L.lam[i] = lam;
    }
    if (d == 0) acc[0] += io.pre ? (tid == 0 && want_nll ? L.misc[0] : 0.0) : prior_e;
    // (single evaluation) the late copies have landed once every wave has
    // waited for its own and passed the next barrier
    __builtin_amdgcn_s_waitcnt(0);
    if (!want_grad) {
      block_sum<NT, 1>(acc, L.red);
      nll_total += acc[0];
      __syncthreads();
      continue;
    }
    __syncthreads();

    // ---- (e) fine bins: lambda_H from the covering analysis bin and the edges
    // in fine bins k-1, k, k+1; rescale adjoint (lambda_F, oscillation slots, sources)
    const int nsrc = S < ACC_SRC ? S : ACC_SRC;
    for (int k = tid; k < K; k += NT) {
      FineRows x;
      if (k == tid) x = rows;
      else load_rows(io, ds, k, x);
      auto fe = [&](int q) { const int v = L.first[q]; return v < 0 ? 0 : (v > E ? E : v); };
      const int ic = fe(k + 1) - 1;  // analysis bin whose mapped range holds fine bin k whole
      double lH = (ic >= 0 && ic < Nb) ? L.lam[ic] : 0.0;
      double lmd = 0.0, ldk = 0.0, ldk1 = 0.0;
      const int j0 = fe(k > 0 ? k - 1 : 0), j1 = fe(k + 2);
      for (int j = j0; j < j1; ++j) {
        const int kj = L.ek[j];
        if (kj < k - 1 || kj > k + 1 || kj < 0 || kj >= K) continue;
        const double lx = (j >= 1 ? L.lam[j - 1] : 0.0) - (j < Nb ? L.lam[j] : 0.0);
        const double t = L.eT[j];
        const double q = 0.5 * t * t - t * t * t * (1.0 / 3.0);
        const double elo = wf * (t - 0.5 * t * t - 3.0 * q), ehi = wf * (0.5 * t * t - 3.0 * q);
        if (kj == k) {
          lmd += lx * wf * 6.0 * q;
          ldk += lx * elo;
          ldk1 += lx * ehi;
        } else if (kj == k - 1) {
          ldk += lx * ehi;
        } else {
          ldk1 += lx * elo;
        }
      }
      const double mk = L.mk[k];
      double lm = lmd;
      if (k == 0) {
        lm += ldk;  // d_0 = m_0
      } else {
        const double a = L.mk[k - 1];
        if (a * mk > 0.0) {
          const double den = a + mk;
          lm += ldk * 2.0 * a * a / (den * den);
        }
      }
      if (k == K - 1) {
        lm += ldk1;  // d_K = m_{K-1}
      } else {
        const double b = L.mk[k + 1];
        if (mk * b > 0.0) {
          const double den = mk + b;
          lm += ldk1 * 2.0 * b * b / (den * den);
        }
      }
      lH += lm * iwf;
      const double lhs = lH * L.F1[k];
      L.LF[k] = lH * L.Hs[k];
      L.LHs[k] = lhs;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[4 + j] += lhs * x.g[j];
#pragma unroll
      for (int q = 0; q < ACC_SRC; ++q)
        if (q < nsrc) acc[16 + q] += lhs * L.Ss[q * K + k];
    }
    if (S > 0) block_sum<NT, 32>(acc, L.red);
    else block_sum<NT, 16>(acc, L.red);
    nll_total += acc[0];
    double gA = 0.0;  // dNLL/dA_s of the source this thread applies (thread s)
#pragma unroll
    for (int q = 0; q < ACC_SRC; ++q)
      if (q == tid) gA = acc[16 + q];
    // sources past the first sixteen, in further reductions of 16
#pragma unroll 1
    for (int s0 = nsrc; s0 < S; s0 += 16) {
      const int ns = S - s0 < 16 ? S - s0 : 16;
      double a2[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) a2[j] = 0.0;
      for (int k = tid; k < K; k += NT) {
        const double lhs = L.LHs[k];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < ns) a2[q] += lhs * L.Ss[(s0 + q) * K + k];
      }
      block_sum<NT, 16>(a2, L.red);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q == tid - s0) gA = a2[q];
    }

    // ---- (f) gradient of the reduced sums; source norms by the product rule
    // over each source's norm list; flux modes by a gather of lambda_F over
    // each mode's fine bins (CSC); priors. Every gradient entry of this pass
    // may receive several contributions: all adds are atomic.
    if (tid < S) {
      // the list's parameter indices, then their values, each read in one
      // batch (lists of up to NL_FAST entries; longer ones term by term)
      constexpr int NL_FAST = 4;
      const int* nlp = reinterpret_cast<const int*>(L.st + BL.nlp);
      const int* nli = reinterpret_cast<const int*>(L.st + BL.nli);
      const int b = nlp[tid], e = nlp[tid + 1];
      if (e - b <= NL_FAST) {
        int ix[NL_FAST];
        double tv[NL_FAST];
#pragma unroll
        for (int q = 0; q < NL_FAST; ++q) ix[q] = b + q < e ? nli[b + q] : -1;
#pragma unroll
        for (int q = 0; q < NL_FAST; ++q) tv[q] = ix[q] >= 0 ? L.th[ix[q]] : 1.0;
#pragma unroll
        for (int q = 0; q < NL_FAST; ++q) {
          double prod = 1.0;
#pragma unroll
          for (int r = 0; r < NL_FAST; ++r)
            if (r != q && r < e - b) prod *= tv[r];
          if (q < e - b) atomicAdd(&L.grad[ix[q]], gA * prod);
        }
      } else {
        for (int q = b; q < e; ++q) {
          double prod = 1.0;
          for (int r = b; r < e; ++r)
            if (r != q) prod *= L.th[nli[r]];
          atomicAdd(&L.grad[nli[q]], gA * prod);
        }
      }
    }
    if (tid == NT - 1) {  // a thread with no source to apply (S <= MAX_SOURCES < NT)
      for (int j = 0; j < 3; ++j)
        if (ds.cidx[j] >= 0) atomicAdd(&L.grad[ds.cidx[j]], acc[1 + j]);
      for (int j = 0; j < NSLOT; ++j)
        if (p.osc.slot_param[j] >= 0) atomicAdd(&L.grad[p.osc.slot_param[j]], acc[4 + j]);
#pragma unroll
      for (int b = 0; b < MAX_BKG; ++b)
        if (b < NB && L.brt[b] >= 0) atomicAdd(&L.grad[L.brt[b]], acc[8 + b]);
    }
    {
      const int* mdcol = reinterpret_cast<const int*>(L.st + BL.mdcol);
      const int* mdk = reinterpret_cast<const int*>(L.st + BL.mdk);
      const double* mdc = L.st + BL.mdc;
      const int* mdp = reinterpret_cast<const int*>(L.st + BL.mdp);
      // four lanes (a quad) per mode, each taking blocks of four entries in
      // turn: the index and coefficient reads of a block, then its lambda_F
      // reads, are independent (two LDS round trips per sixteen entries);
      // the quad's sums are combined in a fixed order
      const int lq = tid & 3;
      for (int m = tid >> 2; m < M; m += NT / 4) {
        double gm = 0.0;
        const int e0 = mdcol[m], e1 = mdcol[m + 1];
        for (int e = e0 + 4 * lq; e < e1; e += 16) {
          int kq[4];
          double cq[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool in = e + q < e1;
            kq[q] = in ? mdk[e + q] : 0;
            cq[q] = in ? mdc[e + q] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) gm += L.LF[kq[q]] * cq[q];
        }
        gm += dpp_swap<0xB1>(gm);  // quad_perm [1,0,3,2]
        gm += dpp_swap<0x4E>(gm);  // quad_perm [2,3,0,1]
        if (lq == 0) atomicAdd(&L.grad[mdp[m]], gm);
      }
    }
    if (d == 0)
      for (int r = tid; r < p.NR; r += NT) atomicAdd(&L.grad[L.pri[r]], L.prv[r]);
    __syncthreads();
  }

  const bool bad = (L.flag[0] & ST_DOMAIN) || !isfinite(nll_total);
  if (io.fused && !io.keep_rows) {
    // the fold kernel accumulates rows 0..4 into zeroed memory: clear them
    // for the next launch (issued with the outputs, after every read)
    for (int d = 0; d < p.D; ++d) {
      const DsPlan& ds = d == 0 ? p.ds0 : L.dsl[d];
      double* b = io.bin + 6 * (int64_t)ds.kt0;
      const int n = 5 * ds.K;
      for (int j = tid; j < n; j += NT) b[j] = 0.0;
    }
  }
  if (io.out && want_nll && tid == 0) io.out[0] = bad ? INFINITY : nll_total;
  if (io.out && want_grad && want_nll)
    for (int i = tid; i < p.P; i += NT) io.out[1 + i] = bad ? 0.0 : L.grad[i];
  if (io.status && tid == 0) *io.status = bad ? ST_DOMAIN : 0;
  return bad ? INFINITY : nll_total;
}

// Launch prologue of the batched bin stages: clears the gradient and flag
// and evaluates the prior rows from the parameters in LDS into L.prv / L.pri.
// Returns this thread's part of the prior NLL. The caller synchronises before
// the serial stages read the rows.
template <int NT>
__device__ __forceinline__ double prologue(const DevPlan& p, Lds<NT>& L, int want_nll) {
  const int tid = threadIdx.x;
  for (int i = tid; i < p.P; i += NT) L.grad[i] = 0.0;
  if (tid == 0) L.flag[0] = 0;
  double e_sum = 0.0;
  if (!want_nll) return e_sum;
  for (int r = tid; r < p.NR; r += NT) {
    int idx;
    double v, e;
    prior_row(p, L.th, r, idx, v, e);
    L.prv[r] = v;
    L.pri[r] = idx;
    e_sum += e;
  }
  return e_sum;
}

// Single evaluation: one workgroup; the fold kernel has already reduced the
// events to fine-bin rows 0..4 and per-segment S.
template <int NT>
__global__ __launch_bounds__(NT) void tail_kernel(TailArgs a) {
  extern __shared__ double smem[];
  if (a.skip && *a.skip != FIT_RUNNING) return;
  const DevPlan& p = a.plan;
  Lds<NT> L = carve<NT>(smem, p);

  const EvalIO io{a.theta, nullptr, a.data, a.out, a.status, a.mu_out, const_cast<double*>(a.Sseg),
                  const_cast<double*>(a.bin), 1, a.keep_rows, a.pre};
  // The fold launch has applied the oscillation coefficients and, in its
  // parameter pass, evaluated everything that depends on the parameters (the
  // domain checks included). The parameters, the dataset plans (dataset 0's
  // comes with the kernel arguments), the prior rows, the domain flags and
  // every input of dataset 0 go to LDS by direct copies: one round trip.
  const int tid = threadIdx.x;
  L.th = matched(L.thb, a.theta);
  copy_to_lds<NT>(L.th, a.theta, p.P, 2);
  copy_to_lds<NT>(reinterpret_cast<double*>(L.dsl), reinterpret_cast<const double*>(p.ds), p.D * DSPLAN_DOUBLES, 5);
  copy_to_lds<NT>(L.prv, a.pre + p.pre_prv, p.pre_glob, 7);
  {
    const DsPlan& ds = p.ds0;
    const BlobLayout BL = blob_layout(ds.Nb + 1, ds.nbkg, ds.Nb, ds.nnz, ds.M, ds.S, ds.nl, ds.K, ds.fw);
    gather_early<NT>(p, io, L, ds, BL, a.want_nll);
  }
  for (int i = tid; i < p.P; i += NT) L.grad[i] = 0.0;
  if (tid == 0) L.flag[0] = 0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const double f = serial_stages<NT>(p, io, L, 0.0, a.want_nll, a.want_grad);
  if (a.has_fit) lbfgs_step<NT>(a.fit, p.P, L.th, f, L.grad, L.fit, L.red);
}

// ---------------------------------------------------------------- batched
// One workgroup per fit: phase A inside the workgroup (thread per segment,
// then per fine bin), the same serial stages, then the fit's minimiser step.
__device__ inline FitArgs fit_of(const FitArgs& F, int f, int P) {
  FitArgs r = F;
  const int64_t o = (int64_t)f * P, oh = (int64_t)f * F.m * P, om = (int64_t)f * F.m;
  r.hdr = F.hdr + f;
  r.x = F.x + o;
  r.g = F.g + o;
  r.p = F.p + o;
  r.d2 = F.d2 + o;
  r.freem = F.freem + o;
  r.S = F.S + oh;
  r.Y = F.Y + oh;
  r.rho = F.rho + om;
  r.gam = F.gam + om;
  r.theta_next = F.theta_next + o;
  return r;
}

template <int NT>
__global__ __launch_bounds__(NT) void batch_tail_kernel(BatchTailArgs a) {
  extern __shared__ double smem[];
  const int f = blockIdx.x;
  if (f >= a.B) return;
  if (a.has_fit && a.fit.hdr[f].status != FIT_RUNNING) return;
  const DevPlan& p = a.plan;
  Lds<NT> L = carve<NT>(smem, p);
  const int tid = threadIdx.x;
  const int P = p.P, G = p.G, KT = p.KT;
  const int NMOM = num_moments(p.osc.formula);
  const double* th = a.theta + (int64_t)f * P;
  for (int i = tid; i < P; i += NT) L.th[i] = th[i];
  {
    const double* src = reinterpret_cast<const double*>(p.ds);
    double* dst = reinterpret_cast<double*>(L.dsl);
    for (int i = tid; i < p.D * DSPLAN_DOUBLES; i += NT) dst[i] = src[i];
  }
  // outside the domain the coefficients are not used for any reported value:
  // the serial stages flag the same cases from the parameters
  if (tid == 0) (void)osc_coefficients(p.osc, th, L.coef);
  __syncthreads();
  const int drow = a.data_idx ? a.data_idx[f] : f;
  const int prow = a.part_idx ? a.part_idx[f] : f;
  const EvalIO io{th,
                  a.part + (int64_t)prow * NMOM * p.nitems,
                  a.want_nll ? a.data + (int64_t)drow * p.nbins_total : nullptr,
                  a.out ? a.out + (int64_t)f * (1 + P) : nullptr,
                  a.status ? a.status + f : nullptr,
                  a.mu_out ? a.mu_out + (int64_t)f * p.nbins_total : nullptr,
                  a.Sseg + (int64_t)f * G,
                  a.bin + (int64_t)f * 6 * KT,
                  0, 0, nullptr};
  double* tmp = a.segtmp + (int64_t)f * 5 * G;
  // phase A, per segment
  for (int g = tid; g < G; g += NT) {
    // moments held in registers: every index below is a compile-time one
    double M[MAX_MOM + 1];
    M[0] = p.Wseg[g];
#pragma unroll
    for (int c = 1; c <= MAX_MOM; ++c) M[c] = 0.0;
    const int ib = p.seg_item[g], ie = p.seg_item[g + 1];
    for (int it = ib; it < ie; ++it) {
#pragma unroll
      for (int c = 0; c < MAX_MOM; ++c)
        if (c < NMOM) M[1 + c] += io.part[(int64_t)c * p.nitems + it];
    }
    const int* nl = p.ipool + p.fs_nl + NLMAX * p.ipool[p.seg_fs + g];
    double A = 1.0;
#pragma unroll
    for (int q = 0; q < NLMAX; ++q)
      if (nl[q] >= 0) A *= L.th[nl[q]];
    double Sv = 0.0;
#pragma unroll
    for (int c = 0; c <= MAX_MOM; ++c) Sv += L.coef[c] * M[c];  // unused coefficients are zero
    store_agent(&io.Sseg[g], Sv);
    tmp[g] = A * Sv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double gj = 0.0;
#pragma unroll
      for (int c = 0; c <= MAX_MOM; ++c) gj += L.coef[CF_STRIDE * (j + 1) + c] * M[c];
      tmp[(int64_t)(1 + j) * G + g] = A * gj;
    }
  }
  __syncthreads();
  // per fine bin: sum over sources
  for (int kt = tid; kt < KT; kt += NT) {
    const int* info = p.ipool + p.kt_info + 5 * kt;
    const int g0 = info[0], K = info[1], S = info[2], kt0 = info[4];
    const int k = kt - kt0;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < S; ++s)
      for (int j = 0; j < 5; ++j) v[j] += tmp[(int64_t)j * G + g0 + s * K];
    double* bb = io.bin + 6 * (int64_t)kt0;
    for (int j = 0; j < 5; ++j) store_agent(&bb[j * K + k], v[j]);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const double pe = prologue<NT>(p, L, a.want_nll);
  __syncthreads();
  const double fval = serial_stages<NT>(p, io, L, pe, a.want_nll, a.want_nll ? a.want_grad : 0);
  if (a.has_fit) {
    if (a.osc_last && tid < NSLOT) {
      const int q = p.osc.slot_param[tid];
      a.osc_last[4 * f + tid] = q >= 0 ? L.th[q] : p.osc.slot_value[tid];
    }
    lbfgs_step<NT>(fit_of(a.fit, f, P), P, L.th, fval, L.grad, L.fit, L.red);
  }
}

__global__ void zero_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_batch_tail(const BatchTailArgs& a, int nt, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  const size_t lds = tail_lds_bytes(a.plan, nt);
  const dim3 grid(a.B);
  switch (nt) {
    case 256:
      hipLaunchKernelGGL(batch_tail_kernel<256>, grid, dim3(256), lds, stream, a);
      break;
    case 512:
      hipLaunchKernelGGL(batch_tail_kernel<512>, grid, dim3(512), lds, stream, a);
      break;
    default:
      hipLaunchKernelGGL(batch_tail_kernel<1024>, grid, dim3(1024), lds, stream, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream, hipEvent_t start, hipEvent_t stop) {
  const size_t lds = tail_lds_bytes(a.plan, nt);
  const dim3 grid(1);
  auto go = [&](auto kernel, int threads) {
    if (start || stop) hipExtLaunchKernelGGL(kernel, grid, dim3(threads), (uint32_t)lds, stream, start, stop, 0, a);
    else hipLaunchKernelGGL(kernel, grid, dim3(threads), lds, stream, a);
  };
  switch (nt) {
    case 256:
      go(tail_kernel<256>, 256);
      break;
    case 512:
      go(tail_kernel<512>, 512);
      break;
    default:
      go(tail_kernel<1024>, 1024);
      break;
  }
  return hipGetLastError();
}

hipError_t tail_set_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tail_kernel<256>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(tail_kernel<512>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(tail_kernel<1024>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch_tail_kernel<256>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch_tail_kernel<512>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(batch_tail_kernel<1024>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace nufold
