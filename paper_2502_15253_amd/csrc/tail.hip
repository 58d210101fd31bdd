// Bin stages, NLL and adjoint gradient of one model evaluation.
//
// Inputs per fine bin k of a dataset: Hs[k] = sum_s A_s S[s][k] (oscillated
// spectrum with source norms) and its derivatives with respect to the four
// oscillation slots, and S[s][k] per source. For a single evaluation the fold
// kernel has produced them; for a batch of fits each fit's workgroup first
// sums the fold's partial moments itself (phase A, one thread per segment,
// then per fine bin).
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
#include <hip/hip_ext.h>

#include "kernels.hpp"
#include "osc.hpp"

namespace nufold {


template <int NT>
struct Lds {
  double* th;     // P
  double* grad;   // P
  double* coef;   // 40
  DsPlan* dsl;    // D dataset plans (copied from global memory once per launch)
  double* red;    // reduction scratch
  double* dyn;    // 6K + S*K + Nb: Hs, G0..G3, F1, Ss (per-source spectra), observed counts
  double* Hs;
  double* Gs;     // 4K
  double* F1;
  double* Ss;
  double* nD;
  double* D;      // K+1  edge densities
  double* C;      // K+1  cumulative, later lambda_C, then lambda_H
  double* Ld;     // K+1  lambda_d
  double* Suf;    // K+1  suffix sums of lambda_C, later lambda_F
  double* LH;     // K    H (scan input), lambda_m (direct), later lambda_Hs
  double* eT;     // E    t, later e_m
  double* eY;     // E    y, later e_dlo
  double* eH;     // E    e_dhi
  double* mu;     // Nb   lambda_mu
  double* st;     // static blob of the current dataset (edges become X, then lambda_X)
  double* fit;    // minimiser scratch
  int* kidx;      // E    fine bin of each mapped analysis edge (monotone)
  int* first;     // K+3  first[k + 1] = first edge with kidx >= k, k = -1 .. K+1
  int* flag;      // 2
};

template <int NT>
__device__ Lds<NT> carve(double* base, const DevPlan& p) {
  Lds<NT> L;
  const int K = p.max_K, E = p.max_Nb + 1, Nb = p.max_Nb;
  // regions filled by direct copies start at 16-byte boundaries (even offsets)
  auto al = [](double* x) { return x + (reinterpret_cast<uintptr_t>(x) & 8 ? 1 : 0); };
  double* q = base;
  L.th = q; q += p.P;
  L.grad = q; q += p.P;
  L.coef = q; q += 40;
  q = al(q);
  L.dsl = reinterpret_cast<DsPlan*>(q); q += p.D * DSPLAN_DOUBLES;
  L.red = q; q += NT + 16;
  q = al(q);
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
  q = al(q);
  L.st = q; q += p.max_blob;

  L.fit = q; q += fit_lds_doubles(p.P, p.fit_m);
  int* r = reinterpret_cast<int*>(q);
  L.kidx = r; r += E;
  L.first = r; r += K + 3;
  L.flag = r;
  L.Hs = L.Gs = L.F1 = L.Ss = L.nD = nullptr;
  return L;
}

// Launch prologue: parameters into LDS, gradient cleared, and the dataset
// plans copied to LDS so every later stage reads them without a global round
// trip. The caller synchronises.
template <int NT>
__device__ __forceinline__ void load_params(const DevPlan& p, const double* th, Lds<NT>& L) {
  const int tid = threadIdx.x;
  for (int i = tid; i < p.P; i += NT) {
    L.th[i] = th[i];
    L.grad[i] = 0.0;
  }
  const double* src = reinterpret_cast<const double*>(p.ds);
  double* dst = reinterpret_cast<double*>(L.dsl);
  for (int i = tid; i < p.D * DSPLAN_DOUBLES; i += NT) dst[i] = src[i];
}

// Sum of N values (N <= 16) over the workgroup; every thread gets the
// totals, summed in a fixed order. Each wavefront reduce-scatters the values
// over its 16-lane rows (padded to a power of two), one lane per (value, row)
// writes its row total to red[j * 4 NW + row], then thread j adds the 4 NW
// row totals of value j in order. red holds NT + 16 doubles; the totals sit
// at red[NT + j], past every partial, so back-to-back calls do not overlap.
template <int NT, int N>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  constexpr int NW = NT / 64, R = 4 * NW;
  static_assert(N >= 1 && N <= 16, "reduction scratch too small");
  constexpr int NP = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : 16;
  constexpr int LG = NP == 1 ? 0 : NP == 2 ? 1 : NP == 4 ? 2 : NP == 8 ? 3 : 4;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) c[j] = j < N ? v[j] : 0.0;
  const double x = row_reduce_scatter<NP>(c, lane);
  if (((lane & 15) >> LG) == 0) {
    int j = 0;
    if constexpr (LG > 0) j = (int)(__builtin_bitreverse32((unsigned)lane) >> (32 - LG));
    red[j * R + wid * 4 + (lane >> 4)] = x;
  }
  __syncthreads();
  // four lanes per value (4 N <= 64: all in wavefront 0), each summing a
  // quarter of the R partials, then two quad exchanges; fixed order
  if (tid < 4 * N) {
    const int q = tid >> 2, part = tid & 3;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < R / 4; ++k) s += red[q * R + part * (R / 4) + k];
    s += dpp_swap<0xB1>(s);  // quad_perm [1,0,3,2]
    s += dpp_swap<0x4E>(s);  // quad_perm [2,3,0,1]
    if (part == 0) red[16 * R + q] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = red[16 * R + j];
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
  const double v = wave_scan_incl(s);
  if (lane == 63) red[wid] = v;
  __syncthreads();
  // the totals of the waves before this one, added in wave order
  double pre = 0.0;
  for (int w = 0; w < wid; ++w) pre += red[w];
  double acc = pre + v - s;  // exclusive prefix of this thread's chunk
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

__device__ __forceinline__ double pval(const double* th, int idx, double dflt) {
  return idx >= 0 ? th[idx] : dflt;
}

}  // namespace nufold
#include "minimize.hpp"
namespace nufold {

// ---------------------------------------------------------------- priors
// Prior row r (Eq. 6; third line of Eq. 9): v = its gradient contribution to
// the row's parameter, e = its NLL contribution. Rows < ngauss are
// independent Gaussians; the rest are rows of correlated blocks (V^-1 r).
__device__ __forceinline__ void prior_row(const DevPlan& p, const double* th, int r, int& idx, double& v,
                                          double& e) {
  if (r < p.ngauss) {
    idx = p.ipool[p.gidx + r];
    const double z = th[idx] - p.dpool[p.gmean + r];
    v = z * p.dpool[p.ginv + r];
    e = 0.5 * z * v;
  } else {
    const int bl = p.ipool[p.prow_blk + r - p.ngauss];
    const int b = p.ipool[p.blk_ptr + bl], n = p.ipool[p.blk_ptr + bl + 1] - b;
    const int row = r - p.ngauss - b;
    const double* Vi = p.dpool + p.ipool[p.blk_inv + bl] + (int64_t)row * n;
    v = 0.0;
#pragma unroll 8
    for (int c = 0; c < n; ++c) v += Vi[c] * (th[p.ipool[p.blk_idx + b + c]] - p.dpool[p.blk_mean + b + c]);
    idx = p.ipool[p.blk_idx + b + row];
    e = 0.5 * (th[idx] - p.dpool[p.blk_mean + b + row]) * v;
  }
}

// Asynchronous copies from global memory straight into LDS (global_load_lds:
// no registers, every load in flight at once). dma_lds<NT, B> moves nbytes (a
// multiple of B) in chunks of 64 B bytes, one per wavefront in turn, lane l
// the B bytes at l B of its chunk; B = 16 needs 16-byte aligned source and
// destination. The caller waits (s_waitcnt) and synchronises before reading.
typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef __attribute__((address_space(1))) const void* global_cvoid_ptr;
template <int NT, int B>
__device__ __forceinline__ void dma_lds(char* dst, const char* src, int nbytes) {
  static_assert(B == 4 || B == 16, "4- or 16-byte units");
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nunits = nbytes / B;
  for (int c = wid; c * 64 < nunits; c += NW) {
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
__device__ __forceinline__ void copy_to_lds(double* dst, const double* src, int n) {
  char* d = reinterpret_cast<char*>(dst);
  const char* s = reinterpret_cast<const char*>(src);
  const unsigned da = (unsigned)(uintptr_t)(lds_void_ptr)d;
  const unsigned sa = (unsigned)(uintptr_t)s;
  if (((da ^ sa) & 15u) != 0 || n < 4) {
    dma_lds<NT, 4>(d, s, 8 * n);
    return;
  }
  const int head = (sa & 15u) ? 1 : 0;
  const int body = (n - head) & ~1;
  const int tail = n - head - body;
  if (head) dma_lds<NT, 4>(d, s, 8);
  dma_lds<NT, 16>(d + 8 * head, s + 8 * head, 8 * body);
  if (tail) dma_lds<NT, 4>(d + 8 * (head + body), s + 8 * (head + body), 8);
}

// Stage dataset d's inputs in LDS: the static blob, the fine-bin rows,
// per-segment S and the data. Fused (single evaluation): rows 0..4 and S were
// written by the fold kernel in an earlier launch, so every array is copied
// straight into LDS with direct global-to-LDS loads; row 5 = 1 + F is formed
// later from the blob's flux rows. Otherwise all six rows were written by this
// workgroup's phase A with agent-scope stores and are read back with coherent
// loads, U per thread in flight before the LDS writes. No barrier: the caller
// synchronises.
template <int NT>
__device__ __forceinline__ void stage_fused(const DevPlan& p, const EvalIO& io, Lds<NT>& L, const DsPlan& ds,
                                            int want_nll) {
  const int K = ds.K;
  const int n1 = 6 * K, n2 = n1 + ds.S * K;
  copy_to_lds<NT>(L.st, p.dpool + ds.blob, ds.blob_n);
  copy_to_lds<NT>(L.dyn, io.bin + 6 * (int64_t)ds.kt0, 5 * K);
  copy_to_lds<NT>(L.dyn + n1, io.Sseg + ds.seg0, n2 - n1);
  if (want_nll) copy_to_lds<NT>(L.dyn + n2, io.data + ds.data, ds.Nb);
}

template <int NT>
__device__ __forceinline__ void stage_dataset(const DevPlan& p, const EvalIO& io, Lds<NT>& L, int d, int want_nll) {
  const int tid = threadIdx.x;
  const DsPlan& ds = L.dsl[d];
  const int K = ds.K, Nb = ds.Nb, S = ds.S;
  const int nbl = ds.blob_n;
  const int n1 = 6 * K, n2 = n1 + S * K, n3 = n2 + (want_nll ? Nb : 0);
  const double* blob = p.dpool + ds.blob;
  const double* b = io.bin + 6 * (int64_t)ds.kt0;
  const double* sg = io.Sseg + ds.seg0;
  const double* dt = io.data + ds.data;
  if (io.fused) {
    // dataset 0 was staged with the parameters in the launch prologue
    if (d > 0) stage_fused<NT>(p, io, L, ds, want_nll);
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  const int total = nbl + n3;
  constexpr int U = 16;
  for (int base = 0; base < total; base += NT * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + tid;
      const int j = i - nbl;
      v[u] = i < nbl ? blob[i]
           : j < n1 ? load_agent(b + j) : j < n2 ? load_agent(sg + (j - n1)) : j < n3 ? dt[j - n2] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * NT + tid;
      const int j = i - nbl;
      if (i < nbl) L.st[i] = v[u];
      else if (j < n3) L.dyn[j] = v[u];
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
  if (tid == 0 && !osc_domain_ok(p.osc, L.th)) atomicOr(&L.flag[0], ST_DOMAIN);

  double nll_total = 0.0;  // identical in every thread (block sums broadcast)

  for (int d = 0; d < p.D; ++d) {
    const DsPlan& ds = L.dsl[d];
    const int K = ds.K, Nb = ds.Nb, S = ds.S, E = Nb + 1, M = ds.M, NB = ds.nbkg;
    const double wf = ds.wf, y0 = ds.y0, yK = ds.y0 + ds.wf * K;
    const double iwf = 1.0 / wf;  // densities m = H (1 + F) / w as products
    const BlobLayout BL = blob_layout(E, NB, Nb, ds.nnz, M, S, ds.nl, K);
    double* X = L.st + BL.edges;  // edges, then X, then lambda_X
    const double* tmpl = L.st + BL.tmpl;
    const int* shp = reinterpret_cast<const int*>(L.st + BL.shp);
    const double* bsc = L.st + BL.bsc;
    const int* brt = reinterpret_cast<const int*>(L.st + BL.brt);
    L.Hs = L.dyn;
    L.Gs = L.dyn + K;
    L.F1 = L.dyn + 5 * K;
    L.Ss = L.dyn + 6 * K;
    L.nD = L.dyn + 6 * K + S * K;

    stage_dataset<NT>(p, io, L, d, want_nll);
    __syncthreads();

    // ---- spline: edge densities and cumulative. In fused evaluations each
    // thread forms 1 + F of its own and the previous fine bin from the blob's
    // flux rows (no extra barrier).
    {
      const int* frow = reinterpret_cast<const int*>(L.st + BL.frow);
      const int* fpar = reinterpret_cast<const int*>(L.st + BL.fpar);
      const double* fcf = L.st + BL.fcf;
      auto f1 = [&](int k) {
        if (!io.fused) return L.F1[k];
        double F = 0.0;
        const int e1 = (int)frow[k + 1];
        for (int e = (int)frow[k]; e < e1; ++e) F += L.th[(int)fpar[e]] * fcf[e];
        return 1.0 + F;
      };
      for (int k = tid; k <= K; k += NT) {
        const double fa = k > 0 ? f1(k - 1) : 0.0;
        const double fb = k < K ? f1(k) : 0.0;
        double dk;
        if (k == 0) dk = L.Hs[0] * fb * iwf;
        else if (k == K) dk = L.Hs[K - 1] * fa * iwf;
        else {
          const double ma = L.Hs[k - 1] * fa * iwf, mb = L.Hs[k] * fb * iwf;
          dk = (ma * mb > 0.0) ? 2.0 * ma * mb / (ma + mb) : 0.0;
        }
        L.D[k] = dk;
        if (k < K) {
          L.LH[k] = L.Hs[k] * fb;  // H (scan input)
          if (io.fused) L.F1[k] = fb;
        }
      }
    }
    // the scan's first read is each thread's own element when K <= NT (one
    // per thread, as written above); its own barrier then orders D
    if (K > NT) __syncthreads();
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
        t = (y - (y0 + k * wf)) * iwf;
        const double mk = L.Hs[k] * L.F1[k] * iwf;
        const double dl = L.D[k], dh = L.D[k + 1];
        const double q = 0.5 * t * t - t * t * t * (1.0 / 3.0);
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
    if (!want_grad) {
      if (NB <= 2) block_sum<NT, 3>(acc, L.red);
      else block_sum<NT, 1 + MAX_BKG>(acc, L.red);
      nll_total += acc[0];
      __syncthreads();
      continue;
    }
    // the deviance and background sums are reduced together with the edge
    // pass's sums below; the edge pass only needs lambda_mu
    __syncthreads();

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
        const double mk = L.Hs[k] * L.F1[k] * iwf;
        const double dl = L.D[k], dh = L.D[k + 1];
        const double q = 0.5 * t * t - t * t * t * (1.0 / 3.0);
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
      // edge-index table: first[k + 1] = i for kidx[i-1] < k <= kidx[i]
      const int kp = i > 0 ? L.kidx[i - 1] : -2;
      for (int q = kp + 1; q <= k; ++q) L.first[q + 1] = i;
      if (i == E - 1)
        for (int q = k + 1; q <= K + 1; ++q) L.first[q + 1] = E;
    }
    {
      // one block reduction: gc[0..3], then the deviance and background sums
      double v[4 + 1 + MAX_BKG];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = gc[j];
#pragma unroll
      for (int j = 0; j <= MAX_BKG; ++j) v[4 + j] = acc[j];
      if (NB <= 2) block_sum<NT, 7>(v, L.red);
      else block_sum<NT, 5 + MAX_BKG>(v, L.red);
#pragma unroll
      for (int j = 0; j < 4; ++j) gc[j] = v[j];
#pragma unroll
      for (int j = 0; j <= MAX_BKG; ++j) acc[j] = v[4 + j];
    }
    nll_total += acc[0];
    if (tid == 0) {
      for (int b = 0; b < NB; ++b)
        if ((int)brt[b] >= 0) L.grad[(int)brt[b]] += acc[1 + b];
      for (int j = 0; j < 3; ++j)
        if (ds.cidx[j] >= 0) L.grad[ds.cidx[j]] += gc[j];
    }
    const double top = gc[3];

    // ---- gather per fine bin: lambda_C -> C, lambda_m (direct) -> LH, lambda_d -> Ld
    // (bounds clamped: with an invalid energy map, which is flagged as out of
    // domain, the edge index need not be monotone)
    for (int k = tid; k <= K; k += NT) {
      const int b0 = min(max(L.first[k + 1], 0), E);
      const int b1 = min(max(L.first[k + 2], b0), E);
      double lc = 0.0, lm = 0.0, ld = 0.0;
      if (k < K) {
        for (int i = b0; i < b1; ++i) {
          lc += X[i];
          lm += L.eT[i];
          ld += L.eY[i];
        }
      }
      if (k >= 1) {
        const int a0 = min(max(L.first[k], 0), b0);
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
      const double mk = L.Hs[k] * L.F1[k] * iwf;
      double lm = L.LH[k];
      if (k == 0) lm += L.Ld[0];
      if (k == K - 1) lm += L.Ld[K];
      if (k >= 1) {  // d_k = harmonic(m_{k-1}, m_k)
        const double ma = L.Hs[k - 1] * L.F1[k - 1] * iwf;
        if (ma * mk > 0.0) {
          const double den = ma + mk;
          lm += L.Ld[k] * 2.0 * ma * ma / (den * den);
        }
      }
      if (k + 1 <= K - 1) {  // d_{k+1} = harmonic(m_k, m_{k+1})
        const double mb = L.Hs[k + 1] * L.F1[k + 1] * iwf;
        if (mk * mb > 0.0) {
          const double den = mk + mb;
          lm += L.Ld[k + 1] * 2.0 * mb * mb / (den * den);
        }
      }
      L.C[k] = L.Suf[k] + top + lm * iwf;
    }
    // no barrier: the next pass reads only its own fine bins' lambda_H and
    // writes lambda_F over the suffix sums it has read (same thread mapping)

    // ---- rescale adjoint, oscillation parameters and source norms in one
    // pass over the fine bins with one block reduction (in groups of up to
    // 12 sources): lambda_Hs = lambda_H (1 + F), lambda_F -> Suf; the
    // oscillation slots take sum_k lambda_Hs G_j, source s takes
    // dNLL/dA_s = sum_k lambda_Hs S[s][k], then the product rule over its
    // norm list
    {
      const int* nlp = reinterpret_cast<const int*>(L.st + BL.nlp);
      const int* nli = reinterpret_cast<const int*>(L.st + BL.nli);
      auto apply = [&](int s, double gA) {
        const int b = (int)nlp[s], e = (int)nlp[s + 1];
        for (int q = b; q < e; ++q) {
          double prod = 1.0;
          for (int r = b; r < e; ++r)
            if (r != q) prod *= L.th[(int)nli[r]];
          atomicAdd(&L.grad[(int)nli[q]], gA * prod);
        }
      };
      for (int s0 = 0; s0 == 0 || s0 < S; s0 += 12) {
        const int ns = min(S - s0, 12);
        double acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0;
        for (int k = tid; k < K; k += NT) {
          const double lh = L.C[k];
          const double lhs = lh * L.F1[k];
          if (s0 == 0) {
            L.Suf[k] = lh * L.Hs[k];  // lambda_F
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] += lhs * L.Gs[j * K + k];
          }
#pragma unroll
          for (int q = 0; q < 12; ++q)
            if (q < ns) acc[4 + q] += lhs * L.Ss[(s0 + q) * K + k];
        }
        if (ns <= 4) block_sum<NT, 8>(acc, L.red);
        else block_sum<NT, 16>(acc, L.red);
        if (s0 == 0 && tid == NT - 1)  // a thread with no source to apply
          for (int j = 0; j < NSLOT; ++j)
            if (p.osc.slot_param[j] >= 0) L.grad[p.osc.slot_param[j]] += acc[j];
        if (tid < ns) {
          double gA = 0.0;  // acc[4 + tid] without a dynamically indexed register array
#pragma unroll
          for (int q = 0; q < 12; ++q)
            if (q == tid) gA = acc[4 + q];
          apply(s0 + tid, gA);
        }
      }
    }
    // ---- flux modes (CSC gather per mode of lambda_F, written before the
    // block reduction's barriers)
    {
      const int* mdcol = reinterpret_cast<const int*>(L.st + BL.mdcol);
      const int* mdk = reinterpret_cast<const int*>(L.st + BL.mdk);
      const double* mdc = L.st + BL.mdc;
      const int* mdp = reinterpret_cast<const int*>(L.st + BL.mdp);
      for (int m = tid; m < M; m += NT) {
        double gm = 0.0;
        const int e0 = (int)mdcol[m], e1 = (int)mdcol[m + 1];
        // four entries per step: their index and coefficient reads, then
        // their Ld reads, are independent (two LDS round trips per step)
        for (int e = e0; e < e1; e += 4) {
          int k[4];
          double c[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool in = e + q < e1;
            k[q] = in ? (int)mdk[e + q] : 0;
            c[q] = in ? mdc[e + q] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) gm += L.Suf[k[q]] * c[q];
        }
        atomicAdd(&L.grad[(int)mdp[m]], gm);
      }
    }
    __syncthreads();
  }

  // ---- priors (Eq. 6; third line of Eq. 9)
  {
    double pr[1] = {0.0};
    for (int r = tid; r < p.NR; r += NT) {
      int i;
      double v, e;
      prior_row(p, L.th, r, i, v, e);
      pr[0] += e;
      if (want_grad) atomicAdd(&L.grad[i], v);
    }
    block_sum<NT, 1>(pr, L.red);
    nll_total += pr[0];
  }
  __syncthreads();

  const bool bad = (L.flag[0] & ST_DOMAIN) || !isfinite(nll_total);
  if (io.fused) {
    // the fold kernel accumulates rows 0..4 into zeroed memory: clear them
    // for the next launch (issued with the outputs, after every read)
    for (int d = 0; d < p.D; ++d) {
      double* b = io.bin + 6 * (int64_t)L.dsl[d].kt0;
      const int n = 5 * L.dsl[d].K;
      for (int j = tid; j < n; j += NT) b[j] = 0.0;
    }
  }
  if (io.out && want_nll && tid == 0) io.out[0] = bad ? INFINITY : nll_total;
  if (io.out && want_grad && want_nll)
    for (int i = tid; i < p.P; i += NT) io.out[1 + i] = bad ? 0.0 : L.grad[i];
  if (io.status && tid == 0) *io.status = bad ? ST_DOMAIN : 0;
  return bad ? INFINITY : nll_total;
}

// Single evaluation: one workgroup; the fold kernel has already reduced the
// events to fine-bin rows 0..4 and per-segment S.
template <int NT>
__global__ __launch_bounds__(NT) void tail_kernel(TailArgs a) {
  extern __shared__ double smem[];
  if (a.skip && *a.skip != FIT_RUNNING) return;
  const DevPlan& p = a.plan;
  Lds<NT> L = carve<NT>(smem, p);
  const int tid = threadIdx.x;

  const EvalIO io{a.theta, nullptr, a.data, a.out, a.status, a.mu_out, const_cast<double*>(a.Sseg),
                  const_cast<double*>(a.bin), 1};
  // the fold kernel has applied the oscillation coefficients; the domain of
  // the oscillation parameters is checked from LDS in the serial stages.
  // Parameters, dataset plans and dataset 0's inputs go to LDS in one round
  // of direct copies (dataset 0's plan comes with the kernel arguments).
  copy_to_lds<NT>(L.th, a.theta, p.P);
  copy_to_lds<NT>(reinterpret_cast<double*>(L.dsl), reinterpret_cast<const double*>(p.ds), p.D * DSPLAN_DOUBLES);
  stage_fused<NT>(p, io, L, p.ds0, a.want_nll);
  for (int i = tid; i < p.P; i += NT) L.grad[i] = 0.0;
  if (tid == 0) L.flag[0] = 0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
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
  const int P = p.P, G = p.G, KT = p.KT;
  const int NMOM = num_moments(p.osc.formula);
  const double* th = a.theta + (int64_t)f * P;
  load_params<NT>(p, th, L);
  if (tid == 0) {
    L.flag[0] = 0;
    if (!osc_coefficients(p.osc, th, L.coef)) L.flag[0] |= ST_DOMAIN;
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
                  0};
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
