// Bin stages, NLL and adjoint gradient of one model evaluation.
//
// Phase A (many workgroups, one wavefront per fine bin, lane s = source):
// sum the fold's partial moments of each (dataset, source, fine-bin) segment
// in a fixed order, turn them into the oscillated fine spectrum S and its
// derivatives with respect to the four oscillation slots (linear in the
// moments), apply the source normalisation A_s and reduce over sources; the
// same wavefront evaluates the flux-shape factor 1 + F_k. Further wavefronts
// evaluate the prior rows (Gaussian and correlated-Gaussian, independent of
// the fold). Phase A results are written with agent-scope (write-through)
// atomic stores; each workgroup waits for its stores to complete and then
// bumps a counter; the last workgroup runs the serial part, reading those
// results with agent-scope atomic loads, and resets the counter. No L2
// write-back is needed for the hand-off.
//
// Serial part (one workgroup; bin stages are latency-bound), per dataset
// (paper, "Structure of the framework", steps 2 and 3, and Eq. 3-6, 9):
//   Hs[k] = sum_s A_s S[s][k],  H[k] = Hs[k] (1 + F_k)
//   m_k = H_k/w, d_k = harmonic mean of neighbouring m (ends: m_0, m_{K-1}),
//   C(y) = C_k + w [d_k (t - t^2/2) + d_{k+1} t^2/2 + 6 (m_k - (d_k+d_{k+1})/2)(t^2/2 - t^3/3)]
//   X_i = C(g(x_i)),  g = inverse of f(E) = c0 + (1+c1) E + c2 E^2
//   s_i = X_{i+1} - X_i,  mu_i = s_i + sum_b scale_b R_b T_bi (1 + beta_bi)
//   NLL += sum_i [mu - n + n ln(n/mu)]   (n = 0: mu)
// then the prior rows. A dataset's static inputs (one packed blob) and its
// dynamic inputs are staged in LDS with two batched copies.
//
// Reverse pass (exact adjoint; replaces numerical gradients):
//   lambda_mu = 1 - n/mu -> background rates and shapes; lambda_X from
//   s_i = X_{i+1} - X_i; each X_i depends on C_k, m_k, d_k, d_{k+1} of its
//   fine bin and on y = g(x; c) (energy-scale coefficients, dC/dy = rho);
//   C_k = sum_{j<k} H_j gives a suffix sum; d_k depends on m_{k-1}, m_k;
//   lambda_H -> flux modes, source norms, and, through the forward-mode
//   derivative rows of the fold moments, the oscillation parameters.
//
// All arithmetic is FP64. Gradient contributions are gathered in a fixed
// order except where contributions can hit one shared parameter within a
// phase (LDS atomics), which only affects the last bits.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace nufold {

__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT>
struct Lds {
  double* th;     // P
  double* grad;   // P
  double* coef;   // 40
  double* red;    // reduction scratch
  double* dyn;    // 6K + S*K + Nb: Hs, G0..G3, F1, Ss (per-source spectra), observed counts
  double* Hs;
  double* Gs;     // 4K
  double* F1;
  double* Ss;
  double* nD;
  double* D;      // K+1  edge densities
  double* C;      // K+1  cumulative, later lambda_C, then lambda_H
  double* Ld;     // K+1  lambda_d, later lambda_F
  double* Suf;    // K+1  suffix sums of lambda_C
  double* LH;     // K    H (scan input), lambda_m (direct), later lambda_Hs
  double* eT;     // E    t, later e_m
  double* eY;     // E    y, later e_dlo
  double* eH;     // E    e_dhi
  double* mu;     // Nb   lambda_mu
  double* st;     // static blob of the current dataset (edges become X, then lambda_X)
  double* fit;    // minimiser scratch
  int* kidx;      // E
  int* flag;      // 2
};

template <int NT>
__device__ Lds<NT> carve(double* base, const DevPlan& p) {
  Lds<NT> L;
  const int K = p.max_K, E = p.max_Nb + 1, Nb = p.max_Nb;
  double* q = base;
  L.th = q; q += p.P;
  L.grad = q; q += p.P;
  L.coef = q; q += 40;
  L.red = q; q += 16 * (NT / 64) + 16;
  L.dyn = q; q += 6 * K + p.max_S * K + Nb;
  L.D = q; q += K + 1;
  L.C = q; q += K + 1;
  L.Ld = q; q += K + 1;
  L.Suf = q; q += K + 1;
  L.LH = q; q += K;
  L.eT = q; q += E;
  L.eY = q; q += E;
  L.eH = q; q += E;
  L.mu = q; q += Nb;
  L.st = q; q += p.max_blob;
  L.fit = q; q += fit_lds_doubles(p.P, p.fit_m);
  int* r = reinterpret_cast<int*>(q);
  L.kidx = r; r += E;
  L.flag = r;
  L.Hs = L.Gs = L.F1 = L.Ss = L.nD = nullptr;
  return L;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of N values over the workgroup; every thread gets the totals. Wave
// partials go to red[j*NW + w]; groups of NW lanes finish them with shuffles.
template <int NT, int N>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  constexpr int NW = NT / 64;
  static_assert(N <= 16, "reduction scratch too small");
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) red[j * NW + wid] = v[j];
  }
  __syncthreads();
  if (wid < (N * NW + 63) / 64) {  // whole wavefronts take part in the shuffles
    double x = tid < N * NW ? red[tid] : 0.0;
#pragma unroll
    for (int off = NW / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (tid < N * NW && (tid % NW) == 0) red[16 * NW + tid / NW] = x;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = red[16 * NW + j];
}

// out[i] = sum of x[j] for j < i (i = 0..n), or, with reverse, out[i] = sum of
// x[j] for j > i (i = 0..n-1). Contiguous chunks per thread, fixed order.
template <int NT>
__device__ void block_scan(const double* x, double* out, int n, bool reverse, double* red) {
  constexpr int NW = NT / 64;
  const int per = (n + NT - 1) / NT;
  const int lo = threadIdx.x * per;
  const int hi = min(lo + per, n);
  double s = 0.0;
  for (int i = lo; i < hi; ++i) s += reverse ? x[n - 1 - i] : x[i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  if (lane == 63) red[wid] = v;
  __syncthreads();
  if (wid == 0) {  // exclusive scan of the wave totals
    const double w = lane < NW ? red[lane] : 0.0;
    double incl = w;
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const double t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane < NW) red[NW + lane] = incl - w;
  }
  __syncthreads();
  double acc = red[NW + wid] + v - s;  // exclusive prefix of this thread's chunk
  if (!reverse) {
    for (int i = lo; i < hi; ++i) {
      out[i] = acc;
      acc += x[i];
    }
    if (hi == n && lo < hi) out[n] = acc;
    if (n == 0 && threadIdx.x == 0) out[0] = 0.0;
  } else {
    for (int i = lo; i < hi; ++i) {
      out[n - 1 - i] = acc;
      acc += x[n - 1 - i];
    }
  }
  __syncthreads();
}

// Cooperative copy global -> LDS with U independent loads in flight per thread.
template <int NT, int U>
__device__ __forceinline__ void stage(double* dst, const double* src, int n) {
  for (int base = 0; base < n; base += NT * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + (int)threadIdx.x;
      v[u] = i < n ? src[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + (int)threadIdx.x;
      if (i < n) dst[i] = v[u];
    }
  }
}

__device__ __forceinline__ int lower_bound_int(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double pval(const double* th, int idx, double dflt) {
  return idx >= 0 ? th[idx] : dflt;
}

// Oscillation coefficient rows: row 0 gives S, rows 1..4 dS/d(slot j), each a
// linear combination of (W, M_1..M_NM). Returns false outside the domain.
__device__ bool osc_coefficients(const OscPlan& o, const double* th, double* cf) {
  double v[NSLOT];
  for (int j = 0; j < NSLOT; ++j) v[j] = o.slot_param[j] >= 0 ? th[o.slot_param[j]] : o.slot_value[j];
  for (int i = 0; i < 40; ++i) cf[i] = 0.0;
  bool ok = true;
  for (int j = 0; j < NSLOT; ++j) ok = ok && isfinite(v[j]);
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
    double* r0 = cf;
    r0[0] = 1.0 - 0.5 * s - 0.5 * A; r0[1] = 0.5 * s; r0[2] = 0.5 * A;
    double* r1 = cf + 8;   // d/d sin^2(2 th13)
    r1[0] = -0.5 - 0.5 * dA_ds; r1[1] = 0.5; r1[2] = 0.5 * dA_ds;
    double* r2 = cf + 16;  // d/d dm2_ee
    r2[3] = -0.5 * s * aee;
    double* r3 = cf + 24;  // d/d sin^2 th12
    r3[0] = -0.5 * dA_ds12; r3[2] = 0.5 * dA_ds12;
    double* r4 = cf + 32;  // d/d dm2_21
    r4[4] = -0.5 * A * a21;
  } else {
    // moments: 1 C_21, 2 C_31, 3 C_32, 4 Q_21, 5 Q_31, 6 Q_32
    const double s12 = v[0], s13 = v[1];
    const double c12 = 1.0 - s12, c13 = 1.0 - s13;
    const double K21 = 4.0 * c12 * s12 * c13 * c13;
    const double K31 = 4.0 * c12 * c13 * s13;
    const double K32 = 4.0 * s12 * c13 * s13;
    const double a21 = TWO_PHASE_K * UNIT_1EM5, a31 = TWO_PHASE_K * UNIT_1EM3;
    double* r0 = cf;
    r0[0] = 1.0 - 0.5 * (K21 + K31 + K32);
    r0[1] = 0.5 * K21; r0[2] = 0.5 * K31; r0[3] = 0.5 * K32;
    const double d12[3] = {4.0 * (1.0 - 2.0 * s12) * c13 * c13, -4.0 * c13 * s13, 4.0 * c13 * s13};
    const double d13[3] = {-8.0 * c12 * s12 * c13, 4.0 * c12 * (1.0 - 2.0 * s13),
                           4.0 * s12 * (1.0 - 2.0 * s13)};
    double* r1 = cf + 8;
    double* r2 = cf + 16;
    r1[0] = -0.5 * (d12[0] + d12[1] + d12[2]);
    r2[0] = -0.5 * (d13[0] + d13[1] + d13[2]);
    for (int j = 0; j < 3; ++j) {
      r1[1 + j] = 0.5 * d12[j];
      r2[1 + j] = 0.5 * d13[j];
    }
    double* r3 = cf + 24;  // d/d dm2_21: x21 grows, x32 = x31 - x21 shrinks
    r3[4] = -0.5 * K21 * a21; r3[6] = 0.5 * K32 * a21;
    double* r4 = cf + 32;  // d/d dm2_31
    r4[5] = -0.5 * K31 * a31; r4[6] = -0.5 * K32 * a31;
  }
  return ok;
}

}  // namespace nufold
#include "minimize.hpp"
namespace nufold {

// ---------------------------------------------------------------- phase A
// Wavefront w < KT: global fine bin w. Wavefront KT + r: prior rows 64 r .. 64 r + 63.
template <int NT>
__device__ void phase_a(const DevPlan& p, const EvalIO& io, const Lds<NT>& L, int w) {
  const int lane = threadIdx.x & 63;
  const int NMOM = num_moments(p.osc.formula);
  if (w < p.KT) {
    const int* info = p.ipool + p.kt_info + 5 * w;
    const int g0 = info[0], K = info[1], S = info[2], fs0 = info[3], kt0 = info[4];
    const int k = w - kt0;
    double hs = 0.0, gsum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = lane; s < S; s += 64) {
      const int g = g0 + s * K;
      double M[MAX_MOM + 1];
      M[0] = p.Wseg[g];
      for (int c = 1; c <= MAX_MOM; ++c) M[c] = 0.0;
      const int ib = p.seg_item[g], ie = p.seg_item[g + 1];
      for (int it = ib; it < ie; ++it)
        for (int c = 0; c < NMOM; ++c) M[1 + c] += io.part[(int64_t)c * p.nitems + it];
      const int* nl = p.ipool + p.fs_nl + NLMAX * (fs0 + s);
      double A = 1.0;
#pragma unroll
      for (int q = 0; q < NLMAX; ++q)
        if (nl[q] >= 0) A *= L.th[nl[q]];
      double Sv = 0.0;
      for (int c = 0; c <= NMOM; ++c) Sv += L.coef[c] * M[c];
      store_agent(&io.Sseg[g], Sv);
      hs += A * Sv;
      for (int j = 0; j < 4; ++j) {
        double gj = 0.0;
        for (int c = 0; c <= NMOM; ++c) gj += L.coef[8 * (j + 1) + c] * M[c];
        gsum[j] += A * gj;
      }
    }
    // flux-shape factor of this fine bin
    double F = 0.0;
    const int rb = p.ipool[p.kt_row + w], re = p.ipool[p.kt_row + w + 1];
    for (int e = rb + lane; e < re; e += 64) F += L.th[p.ipool[p.kt_par + e]] * p.dpool[p.kt_coef + e];
    hs = wave_sum(hs);
    for (int j = 0; j < 4; ++j) gsum[j] = wave_sum(gsum[j]);
    F = wave_sum(F);
    if (lane == 0) {
      double* b = io.bin + 6 * (int64_t)kt0;
      store_agent(&b[k], hs);
      for (int j = 0; j < 4; ++j) store_agent(&b[(1 + j) * K + k], gsum[j]);
      store_agent(&b[5 * K + k], 1.0 + F);
    }
  } else {
    const int r = (w - p.KT) * 64 + lane;
    if (r < p.NR) {
      double v, e;
      if (r < p.ngauss) {
        const double z = L.th[p.ipool[p.gidx + r]] - p.dpool[p.gmean + r];
        v = z * p.dpool[p.ginv + r];
        e = 0.5 * z * v;
      } else {
        const int bl = p.ipool[p.prow_blk + r - p.ngauss];
        const int b = p.ipool[p.blk_ptr + bl], n = p.ipool[p.blk_ptr + bl + 1] - b;
        const int row = r - p.ngauss - b;
        const double* Vi = p.dpool + p.ipool[p.blk_inv + bl] + (int64_t)row * n;
        v = 0.0;
#pragma unroll 8
        for (int c = 0; c < n; ++c)
          v += Vi[c] * (L.th[p.ipool[p.blk_idx + b + c]] - p.dpool[p.blk_mean + b + c]);
        e = 0.5 * (L.th[p.ipool[p.blk_idx + b + row]] - p.dpool[p.blk_mean + b + row]) * v;
      }
      store_agent(&io.prior[r], v);
      store_agent(&io.prior[p.NR + r], e);
    }
  }
}

// Serial bin stages, NLL, priors and adjoint of one evaluation; returns the
// NLL (+inf when out of domain) to every thread; the gradient is in L.grad.
template <int NT>
__device__ double serial_stages(const DevPlan& p, const EvalIO& io, Lds<NT>& L, int want_nll, int want_grad) {
  const int tid = threadIdx.x;
  for (int i = tid; i < p.P; i += NT)
    if (!isfinite(L.th[i])) atomicOr(&L.flag[0], ST_DOMAIN);

  double nll_total = 0.0;  // identical in every thread (block sums broadcast)

  for (int d = 0; d < p.D; ++d) {
    const DsPlan& ds = p.ds[d];
    const int K = ds.K, Nb = ds.Nb, S = ds.S, E = Nb + 1, M = ds.M, NB = ds.nbkg;
    const double wf = ds.wf, y0 = ds.y0, yK = ds.y0 + ds.wf * K;
    const BlobLayout BL = blob_layout(E, NB, Nb, ds.nnz, M, S, ds.nl);
    double* X = L.st + BL.edges;  // edges, then X, then lambda_X
    const double* tmpl = L.st + BL.tmpl;
    const double* shp = L.st + BL.shp;
    const double* bsc = L.st + BL.bsc;
    const double* brt = L.st + BL.brt;
    L.Hs = L.dyn;
    L.Gs = L.dyn + K;
    L.F1 = L.dyn + 5 * K;
    L.Ss = L.dyn + 6 * K;
    L.nD = L.dyn + 6 * K + S * K;

    // ---- stage: static blob (plain loads), phase-A results and data
    stage<NT, 8>(L.st, p.dpool + ds.blob, ds.blob_n);
    {
      const int n1 = 6 * K, n2 = n1 + S * K, n3 = n2 + (want_nll ? Nb : 0);
      const double* b = io.bin + 6 * (int64_t)ds.kt0;
      const double* sg = io.Sseg + ds.seg0;
      const double* dt = io.data + ds.data;
      constexpr int U = 8;
      for (int base = 0; base < n3; base += NT * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = base + u * NT + tid;
          v[u] = i < n1 ? load_agent(b + i) : i < n2 ? load_agent(sg + (i - n1)) : i < n3 ? dt[i - n2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = base + u * NT + tid;
          if (i < n3) L.dyn[i] = v[u];
        }
      }
    }
    __syncthreads();

    // ---- spline: edge densities and cumulative
    for (int k = tid; k <= K; k += NT) {
      double dk;
      if (k == 0) dk = L.Hs[0] * L.F1[0] / wf;
      else if (k == K) dk = L.Hs[K - 1] * L.F1[K - 1] / wf;
      else {
        const double ma = L.Hs[k - 1] * L.F1[k - 1] / wf, mb = L.Hs[k] * L.F1[k] / wf;
        dk = (ma * mb > 0.0) ? 2.0 * ma * mb / (ma + mb) : 0.0;
      }
      L.D[k] = dk;
      if (k < K) L.LH[k] = L.Hs[k] * L.F1[k];  // H (scan input)
    }
    __syncthreads();
    block_scan<NT>(L.LH, L.C, K, false, L.red);

    // ---- energy scale and analysis edges
    const double c0 = pval(L.th, ds.cidx[0], 0.0);
    const double c1 = pval(L.th, ds.cidx[1], 0.0);
    const double c2 = pval(L.th, ds.cidx[2], 0.0);
    const double bb = 1.0 + c1;
    if (tid == 0 && !(bb > 0.0 && bb + 2.0 * c2 * y0 > 0.0 && bb + 2.0 * c2 * yK > 0.0))
      atomicOr(&L.flag[0], ST_DOMAIN);
    for (int i = tid; i < E; i += NT) {
      const double z = X[i] - c0;
      const double disc = bb * bb + 4.0 * c2 * z;
      double y;
      if (disc < 0.0) y = c2 < 0.0 ? INFINITY : -INFINITY;
      else y = 2.0 * z / (bb + sqrt(disc));
      int k;
      double t = 0.0, Xi;
      if (!(y >= y0)) {
        k = -1;
        Xi = 0.0;
      } else if (y >= yK) {
        k = K;
        Xi = L.C[K];
      } else {
        k = (int)floor((y - y0) / wf);
        k = k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
        t = (y - (y0 + k * wf)) / wf;
        const double mk = L.Hs[k] * L.F1[k] / wf;
        const double dl = L.D[k], dh = L.D[k + 1];
        const double q = 0.5 * t * t - t * t * t / 3.0;
        Xi = L.C[k] + wf * (dl * (t - 0.5 * t * t) + dh * 0.5 * t * t + 6.0 * (mk - 0.5 * (dl + dh)) * q);
      }
      L.kidx[i] = k;
      L.eT[i] = t;
      L.eY[i] = y;
      X[i] = Xi;
    }
    __syncthreads();

    // ---- expectations, deviance, lambda_mu; background rate/shape gradients
    double acc[1 + MAX_BKG];
    for (int j = 0; j <= MAX_BKG; ++j) acc[j] = 0.0;
    for (int i = tid; i < Nb; i += NT) {
      double B = 0.0;
      for (int b = 0; b < NB; ++b) {
        const double beta = pval(L.th, (int)shp[b * Nb + i], 0.0);
        B += bsc[b] * pval(L.th, (int)brt[b], 1.0) * tmpl[b * Nb + i] * (1.0 + beta);
      }
      const double mu = (X[i + 1] - X[i]) + B;
      if (io.mu_out) io.mu_out[ds.bins0 + i] = mu;
      double lam = 0.0;
      if (want_nll) {
        const double n = L.nD[i];
        if (!(mu > 0.0)) atomicOr(&L.flag[0], ST_DOMAIN);
        acc[0] += (n > 0.0) ? (mu - n + n * log(n / mu)) : mu;
        lam = 1.0 - n / mu;
        if (want_grad) {
          for (int b = 0; b < NB; ++b) {
            const int sp = (int)shp[b * Nb + i];
            const double stv = bsc[b] * tmpl[b * Nb + i];
            acc[1 + b] += lam * stv * (1.0 + pval(L.th, sp, 0.0));
            if (sp >= 0) atomicAdd(&L.grad[sp], lam * stv * pval(L.th, (int)brt[b], 1.0));
          }
        }
      }
      L.mu[i] = lam;
    }
    block_sum<NT, 1 + MAX_BKG>(acc, L.red);
    nll_total += acc[0];
    if (!want_grad) {
      __syncthreads();
      continue;
    }
    if (tid == 0)
      for (int b = 0; b < NB; ++b)
        if ((int)brt[b] >= 0) L.grad[(int)brt[b]] += acc[1 + b];

    // ---- adjoint per edge: lambda_X, energy-scale coefficients, spline pieces
    double gc[4] = {0.0, 0.0, 0.0, 0.0};  // c0, c1, c2, out-of-range-above total
    for (int i = tid; i < E; i += NT) {
      const double lx = (i >= 1 ? L.mu[i - 1] : 0.0) - (i < Nb ? L.mu[i] : 0.0);
      const int k = L.kidx[i];
      double em = 0.0, elo = 0.0, ehi = 0.0;
      if (k == K) {
        gc[3] += lx;
      } else if (k >= 0) {
        const double t = L.eT[i], y = L.eY[i];
        const double mk = L.Hs[k] * L.F1[k] / wf;
        const double dl = L.D[k], dh = L.D[k + 1];
        const double q = 0.5 * t * t - t * t * t / 3.0;
        const double rho = dl * (1.0 - t) + dh * t + 6.0 * (mk - 0.5 * (dl + dh)) * t * (1.0 - t);
        const double fp = bb + 2.0 * c2 * y;
        const double ly = lx * rho / fp;
        gc[0] -= ly;
        gc[1] -= ly * y;
        gc[2] -= ly * y * y;
        em = lx * wf * 6.0 * q;
        elo = lx * wf * (t - 0.5 * t * t - 3.0 * q);
        ehi = lx * wf * (0.5 * t * t - 3.0 * q);
      }
      X[i] = (k >= 0 && k < K) ? lx : 0.0;
      L.eT[i] = em;
      L.eY[i] = elo;
      L.eH[i] = ehi;
    }
    block_sum<NT, 4>(gc, L.red);
    if (tid == 0)
      for (int j = 0; j < 3; ++j)
        if (ds.cidx[j] >= 0) L.grad[ds.cidx[j]] += gc[j];
    const double top = gc[3];

    // ---- gather per fine bin: lambda_C -> C, lambda_m (direct) -> LH, lambda_d -> Ld
    for (int k = tid; k <= K; k += NT) {
      const int b0 = lower_bound_int(L.kidx, E, k);
      const int b1 = lower_bound_int(L.kidx, E, k + 1);
      double lc = 0.0, lm = 0.0, ld = 0.0;
      if (k < K) {
        for (int i = b0; i < b1; ++i) {
          lc += X[i];
          lm += L.eT[i];
          ld += L.eY[i];
        }
      }
      if (k >= 1) {
        const int a0 = lower_bound_int(L.kidx, E, k - 1);
        for (int i = a0; i < b0; ++i) ld += L.eH[i];
      }
      L.Ld[k] = ld;
      if (k < K) {
        L.LH[k] = lm;
        L.C[k] = lc;
      }
    }
    __syncthreads();
    // C_k = sum_{j<k} H_j: lambda_H[j] collects sum_{k>j} lambda_C[k]
    block_scan<NT>(L.C, L.Suf, K, true, L.red);

    // ---- lambda_H per fine bin -> C
    for (int k = tid; k < K; k += NT) {
      const double mk = L.Hs[k] * L.F1[k] / wf;
      double lm = L.LH[k];
      if (k == 0) lm += L.Ld[0];
      if (k == K - 1) lm += L.Ld[K];
      if (k >= 1) {  // d_k = harmonic(m_{k-1}, m_k)
        const double ma = L.Hs[k - 1] * L.F1[k - 1] / wf;
        if (ma * mk > 0.0) {
          const double den = ma + mk;
          lm += L.Ld[k] * 2.0 * ma * ma / (den * den);
        }
      }
      if (k + 1 <= K - 1) {  // d_{k+1} = harmonic(m_k, m_{k+1})
        const double mb = L.Hs[k + 1] * L.F1[k + 1] / wf;
        if (mk * mb > 0.0) {
          const double den = mk + mb;
          lm += L.Ld[k + 1] * 2.0 * mb * mb / (den * den);
        }
      }
      L.C[k] = L.Suf[k] + top + lm / wf;
    }
    __syncthreads();

    // ---- rescale adjoint: lambda_Hs -> LH, lambda_F -> Ld; oscillation parameters
    double go[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < K; k += NT) {
      const double lh = L.C[k];
      const double lhs = lh * L.F1[k];
      L.LH[k] = lhs;
      L.Ld[k] = lh * L.Hs[k];
      for (int j = 0; j < 4; ++j) go[j] += lhs * L.Gs[j * K + k];
    }
    block_sum<NT, 4>(go, L.red);
    if (tid == 0)
      for (int j = 0; j < NSLOT; ++j)
        if (p.osc.slot_param[j] >= 0) L.grad[p.osc.slot_param[j]] += go[j];

    // ---- flux modes (CSC gather per mode)
    {
      const double* mdcol = L.st + BL.mdcol;
      const double* mdk = L.st + BL.mdk;
      const double* mdc = L.st + BL.mdc;
      const double* mdp = L.st + BL.mdp;
      for (int m = tid; m < M; m += NT) {
        double gm = 0.0;
        const int e1 = (int)mdcol[m + 1];
        for (int e = (int)mdcol[m]; e < e1; ++e) gm += L.Ld[(int)mdk[e]] * mdc[e];
        atomicAdd(&L.grad[(int)mdp[m]], gm);
      }
    }
    // ---- source norms: one wavefront per source
    {
      const double* nlp = L.st + BL.nlp;
      const double* nli = L.st + BL.nli;
      const int lane = tid & 63, wid = tid >> 6;
      for (int s = wid; s < S; s += NT / 64) {
        double gA = 0.0;
        for (int k = lane; k < K; k += 64) gA += L.LH[k] * L.Ss[s * K + k];
        gA = wave_sum(gA);
        if (lane == 0) {
          const int b = (int)nlp[s], e = (int)nlp[s + 1];
          for (int q = b; q < e; ++q) {
            double prod = 1.0;
            for (int r = b; r < e; ++r)
              if (r != q) prod *= L.th[(int)nli[r]];
            atomicAdd(&L.grad[(int)nli[q]], gA * prod);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- priors (Eq. 6; third line of Eq. 9), rows evaluated in phase A
  {
    double pr[1] = {0.0};
    for (int r = tid; r < p.NR; r += NT) {
      pr[0] += load_agent(&io.prior[p.NR + r]);
      if (want_grad) {
        const int i = r < p.ngauss ? p.ipool[p.gidx + r] : p.ipool[p.blk_idx + (r - p.ngauss)];
        atomicAdd(&L.grad[i], load_agent(&io.prior[r]));
      }
    }
    block_sum<NT, 1>(pr, L.red);
    nll_total += pr[0];
  }
  __syncthreads();

  const bool bad = (L.flag[0] & ST_DOMAIN) || !isfinite(nll_total);
  if (io.out && want_nll && tid == 0) io.out[0] = bad ? INFINITY : nll_total;
  if (io.out && want_grad && want_nll)
    for (int i = tid; i < p.P; i += NT) io.out[1 + i] = bad ? 0.0 : L.grad[i];
  if (io.status && tid == 0) *io.status = bad ? ST_DOMAIN : 0;
  return bad ? INFINITY : nll_total;
}

template <int NT>
__global__ __launch_bounds__(NT) void tail_kernel(TailArgs a) {
  extern __shared__ double smem[];
  if (a.skip && *a.skip != FIT_RUNNING) return;
  const DevPlan& p = a.plan;
  Lds<NT> L = carve<NT>(smem, p);
  const int tid = threadIdx.x;

  for (int i = tid; i < p.P; i += NT) {
    L.th[i] = a.theta[i];
    L.grad[i] = 0.0;
  }
  if (tid == 0) {
    L.flag[0] = 0;
    bool ok = osc_coefficients(p.osc, L.th, L.coef);
    if (!ok) L.flag[0] |= ST_DOMAIN;
  }
  __syncthreads();
  const EvalIO io{a.theta, a.part, a.data, a.out, a.status, a.mu_out, a.Sseg, a.bin, a.prior};
  phase_a<NT>(p, io, L, (int)((blockIdx.x * NT + threadIdx.x) >> 6));

  // ---- hand-off: our write-through stores are complete before we count
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    const int done = __hip_atomic_fetch_add(a.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    L.flag[1] = (done == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!L.flag[1]) return;
  if (tid == 0) __hip_atomic_store(a.counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  const double f = serial_stages<NT>(p, io, L, a.want_nll, a.want_grad);
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
  const int P = p.P, G = p.G, KT = p.KT, NR = p.NR;
  const int NMOM = num_moments(p.osc.formula);
  const double* th = a.theta + (int64_t)f * P;
  for (int i = tid; i < P; i += NT) {
    L.th[i] = th[i];
    L.grad[i] = 0.0;
  }
  if (tid == 0) {
    L.flag[0] = 0;
    if (!osc_coefficients(p.osc, L.th, L.coef)) L.flag[0] |= ST_DOMAIN;
  }
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
                  a.prior + (int64_t)f * 2 * NR};
  double* tmp = a.segtmp + (int64_t)f * 5 * G;
  // phase A, per segment
  for (int g = tid; g < G; g += NT) {
    double M[MAX_MOM + 1];
    M[0] = p.Wseg[g];
    for (int c = 1; c <= MAX_MOM; ++c) M[c] = 0.0;
    const int ib = p.seg_item[g], ie = p.seg_item[g + 1];
    for (int it = ib; it < ie; ++it)
      for (int c = 0; c < NMOM; ++c) M[1 + c] += io.part[(int64_t)c * p.nitems + it];
    const int* nl = p.ipool + p.fs_nl + NLMAX * p.ipool[p.seg_fs + g];
    double A = 1.0;
#pragma unroll
    for (int q = 0; q < NLMAX; ++q)
      if (nl[q] >= 0) A *= L.th[nl[q]];
    double Sv = 0.0;
    for (int c = 0; c <= NMOM; ++c) Sv += L.coef[c] * M[c];
    store_agent(&io.Sseg[g], Sv);
    tmp[g] = A * Sv;
    for (int j = 0; j < 4; ++j) {
      double gj = 0.0;
      for (int c = 0; c <= NMOM; ++c) gj += L.coef[8 * (j + 1) + c] * M[c];
      tmp[(int64_t)(1 + j) * G + g] = A * gj;
    }
  }
  // prior rows
  for (int r = tid; r < NR; r += NT) {
    double v, e;
    if (r < p.ngauss) {
      const double z = L.th[p.ipool[p.gidx + r]] - p.dpool[p.gmean + r];
      v = z * p.dpool[p.ginv + r];
      e = 0.5 * z * v;
    } else {
      const int bl = p.ipool[p.prow_blk + r - p.ngauss];
      const int b = p.ipool[p.blk_ptr + bl], n = p.ipool[p.blk_ptr + bl + 1] - b;
      const int row = r - p.ngauss - b;
      const double* Vi = p.dpool + p.ipool[p.blk_inv + bl] + (int64_t)row * n;
      v = 0.0;
      for (int c = 0; c < n; ++c)
        v += Vi[c] * (L.th[p.ipool[p.blk_idx + b + c]] - p.dpool[p.blk_mean + b + c]);
      e = 0.5 * (L.th[p.ipool[p.blk_idx + b + row]] - p.dpool[p.blk_mean + b + row]) * v;
    }
    store_agent(&io.prior[r], v);
    store_agent(&io.prior[NR + r], e);
  }
  __syncthreads();
  // per fine bin: sum over sources, flux factor
  for (int kt = tid; kt < KT; kt += NT) {
    const int* info = p.ipool + p.kt_info + 5 * kt;
    const int g0 = info[0], K = info[1], S = info[2], kt0 = info[4];
    const int k = kt - kt0;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < S; ++s)
      for (int j = 0; j < 5; ++j) v[j] += tmp[(int64_t)j * G + g0 + s * K];
    double F = 0.0;
    const int rb = p.ipool[p.kt_row + kt], re = p.ipool[p.kt_row + kt + 1];
    for (int e = rb; e < re; ++e) F += L.th[p.ipool[p.kt_par + e]] * p.dpool[p.kt_coef + e];
    double* bb = io.bin + 6 * (int64_t)kt0;
    for (int j = 0; j < 5; ++j) store_agent(&bb[j * K + k], v[j]);
    store_agent(&bb[5 * K + k], 1.0 + F);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const double fval = serial_stages<NT>(p, io, L, a.want_nll, a.want_nll ? a.want_grad : 0);
  if (a.has_fit) {
    if (a.osc_last && tid < NSLOT) {
      const int q = p.osc.slot_param[tid];
      a.osc_last[4 * f + tid] = q >= 0 ? L.th[q] : p.osc.slot_value[tid];
    }
    lbfgs_step<NT>(fit_of(a.fit, f, P), P, L.th, fval, L.grad, L.fit, L.red);
  }
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

int tail_blocks(const DevPlan& p, int nt) {
  const int waves = p.KT + (p.NR + 63) / 64;
  const int b = (waves + nt / 64 - 1) / (nt / 64);
  return b < 1 ? 1 : b;
}

hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream) {
  const size_t lds = tail_lds_bytes(a.plan, nt);
  const dim3 grid(tail_blocks(a.plan, nt));
  switch (nt) {
    case 256:
      hipLaunchKernelGGL(tail_kernel<256>, grid, dim3(256), lds, stream, a);
      break;
    case 512:
      hipLaunchKernelGGL(tail_kernel<512>, grid, dim3(512), lds, stream, a);
      break;
    default:
      hipLaunchKernelGGL(tail_kernel<1024>, grid, dim3(1024), lds, stream, a);
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
