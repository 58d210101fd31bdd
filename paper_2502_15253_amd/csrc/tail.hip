// Bin stages, NLL and adjoint gradient for one model evaluation, executed by a
// single workgroup (they are latency-bound: a few hundred bins per dataset).
//
// Forward, per dataset (paper, "Structure of the framework", steps 2 and 3,
// and Eq. 3-6, 9):
//   S[s][k]  = W a0 + sum_c a_c M_c           oscillated fine spectrum from the
//                                              fold moments M (linear in M)
//   Hs[k]    = sum_s A_s S[s][k],  A_s = product of its norm parameters
//   H[k]     = Hs[k] (1 + F_k),    F_k = sum_m f_m phi_m(k)   (flux shape)
//   m_k = H_k/w, d_k = harmonic mean of neighbouring m (ends: m_0, m_{K-1}),
//   C(y) = C_k + w [d_k (t - t^2/2) + d_{k+1} t^2/2 + 6 (m_k - (d_k+d_{k+1})/2)(t^2/2 - t^3/3)]
//   X_i = C(g(x_i)),  g = inverse of f(E) = c0 + (1+c1) E + c2 E^2
//   s_i = X_{i+1} - X_i,  mu_i = s_i + sum_b scale_b R_b T_bi (1 + beta_bi)
//   NLL += sum_i [mu - n + n ln(n/mu)]   (n = 0: mu)
// then Gaussian and correlated-Gaussian priors.
//
// Reverse pass (exact adjoint of the above; replaces numerical gradients):
//   lambda_mu = 1 - n/mu -> background rates and shapes; lambda_X from
//   s_i = X_{i+1} - X_i; each X_i depends on C_k, m_k, d_k, d_{k+1} of its
//   fine bin and on y = g(x; c) (energy-scale coefficients, dC/dy = rho);
//   C_k = sum_{j<k} H_j gives a suffix sum; d_k depends on m_{k-1}, m_k;
//   lambda_H -> flux modes, source norms, and, through the forward-mode
//   derivative rows of the fold moments, the oscillation parameters.
//
// All arithmetic is FP64. Gradient contributions are gathered in a fixed order
// except where several contributions can hit one shared parameter within a
// phase (LDS atomics), which only affects the last bits.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace nufold {


template <int NT>
struct Lds {
  double* theta;  // P
  double* grad;   // P
  double* coef;   // 5 x 8
  double* A;      // max_S
  double* Hs;     // K
  double* F1;     // K
  double* Gs;     // 4 K
  double* D;      // K + 1  edge densities
  double* C;      // K + 1  cumulative, later lambda_C, then lambda_H
  double* Ld;     // K + 1  lambda_d, later lambda_F
  double* LH;     // K      H (scan input), lambda_m (direct), later lambda_Hs
  double* Suf;    // K + 1  suffix sums of lambda_C
  double* eT;     // E      t, later e_m
  double* eY;     // E      y, later e_dlo
  double* eX;     // E      X, later lambda_X
  double* eH;     // E      e_dhi
  double* mu;     // Nb     mu, later lambda_mu
  double* red;    // 8 * NT/64 + 8
  int* kidx;      // E
  int* flag;      // 1
};

template <int NT>
__device__ Lds<NT> carve(double* base, const DevPlan& p) {
  Lds<NT> L;
  const int K = p.max_K, E = p.max_Nb + 1;
  double* q = base;
  L.theta = q; q += p.P;
  L.grad = q; q += p.P;
  L.coef = q; q += 40;
  L.A = q; q += p.max_S;
  L.Hs = q; q += K;
  L.F1 = q; q += K;
  L.Gs = q; q += 4 * K;
  L.D = q; q += K + 1;
  L.C = q; q += K + 1;
  L.Ld = q; q += K + 1;
  L.LH = q; q += K;
  L.Suf = q; q += K + 1;
  L.eT = q; q += E;
  L.eY = q; q += E;
  L.eX = q; q += E;
  L.eH = q; q += E;
  L.mu = q; q += p.max_Nb;
  L.red = q; q += 8 * (NT / 64) + 8;
  L.kidx = reinterpret_cast<int*>(q);
  L.flag = L.kidx + E;
  return L;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of N values over the workgroup; every thread gets the totals.
template <int NT, int N>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) red[j * (NT / 64) + wid] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += red[j * (NT / 64) + i];
    v[j] = t;
  }
  __syncthreads();
}

// out[i] = sum of x[j] for j < i (i = 0..n), or, with reverse, out[i] = sum of
// x[j] for j > i (i = 0..n-1). Contiguous chunks per thread, fixed order.
template <int NT>
__device__ void block_scan(const double* x, double* out, int n, bool reverse, double* red) {
  const int per = (n + NT - 1) / NT;
  const int lo = threadIdx.x * per;
  const int hi = min(lo + per, n);
  auto at = [&](int i) { return reverse ? x[n - 1 - i] : x[i]; };
  double s = 0.0;
  for (int i = lo; i < hi; ++i) s += at(i);
  // inclusive scan of s over threads
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  __syncthreads();
  if (lane == 63) red[wid] = v;
  __syncthreads();
  double base = 0.0;
  for (int i = 0; i < wid; ++i) base += red[i];
  double acc = base + v - s;  // exclusive prefix of this thread's chunk
  if (!reverse) {
    for (int i = lo; i < hi; ++i) {
      out[i] = acc;
      acc += x[i];
    }
    if (hi == n && lo < hi) out[n] = acc;
    if (n == 0 && threadIdx.x == 0) out[0] = 0.0;
  } else {
    // position i in reversed order is element n-1-i; out[e] = sum over j > e
    for (int i = lo; i < hi; ++i) {
      out[n - 1 - i] = acc;
      acc += x[n - 1 - i];
    }
  }
  __syncthreads();
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

// Oscillation coefficient rows: row 0 gives S, rows 1..4 dS/d(slot j) as linear
// combinations of (W, M_1..M_NM). Returns false outside the parameter domain.
__device__ bool osc_coefficients(const OscPlan& o, const double* th, double* cf) {
  double v[NSLOT];
  for (int j = 0; j < NSLOT; ++j) v[j] = o.slot_param[j] >= 0 ? th[o.slot_param[j]] : o.slot_value[j];
  for (int i = 0; i < 40; ++i) cf[i] = 0.0;
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
    double* r1 = cf + 8;  // d/d sin^2(2 th13)
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
  return true;
}

template <int NT>
__global__ __launch_bounds__(NT) void tail_kernel(TailArgs a) {
  extern __shared__ double smem[];
  const DevPlan& p = a.plan;
  Lds<NT> L = carve<NT>(smem, p);
  const int tid = threadIdx.x;
  const int NMOM = num_moments(p.osc.formula);

  for (int i = tid; i < p.P; i += NT) {
    L.theta[i] = a.theta[i];
    L.grad[i] = 0.0;
  }
  if (tid == 0) *L.flag = 0;
  __syncthreads();
  if (tid == 0) {
    bool ok = osc_coefficients(p.osc, L.theta, L.coef);
    for (int i = 0; i < p.P; ++i)
      if (!isfinite(L.theta[i])) ok = false;
    if (!ok) *L.flag |= ST_DOMAIN;
  }
  __syncthreads();

  double nll_total = 0.0;  // meaningful in every thread (block sums broadcast)

  for (int d = 0; d < p.D; ++d) {
    const DsPlan ds = p.ds[d];
    const int K = ds.K, Nb = ds.Nb, S = ds.S, E = Nb + 1;
    const double wf = ds.wf, y0 = ds.y0, yK = ds.y0 + ds.wf * K;

    // ---- source normalisations
    for (int s = tid; s < S; s += NT) {
      const int b = p.ipool[ds.srcnorm_ptr + s], e = p.ipool[ds.srcnorm_ptr + s + 1];
      double A = 1.0;
      for (int q = b; q < e; ++q) A *= L.theta[p.ipool[q]];
      L.A[s] = A;
    }
    __syncthreads();

    // ---- moments -> S[s][k], Hs, Gs, flux factor
    for (int k = tid; k < K; k += NT) {
      double hs = 0.0, g[4] = {0.0, 0.0, 0.0, 0.0};
      for (int s = 0; s < S; ++s) {
        const int gseg = ds.seg0 + s * K + k;
        double M[MAX_MOM + 1];
        M[0] = p.Wseg[gseg];
        for (int c = 1; c <= MAX_MOM; ++c) M[c] = 0.0;
        const int ib = p.seg_item[gseg], ie = p.seg_item[gseg + 1];
        for (int it = ib; it < ie; ++it)
          for (int c = 0; c < NMOM; ++c) M[1 + c] += a.part[(int64_t)c * p.nitems + it];
        double Sv = 0.0;
        for (int c = 0; c <= NMOM; ++c) Sv += L.coef[c] * M[c];
        a.scratch[s * K + k] = Sv;
        const double As = L.A[s];
        hs += As * Sv;
        for (int j = 0; j < 4; ++j) {
          double gj = 0.0;
          for (int c = 0; c <= NMOM; ++c) gj += L.coef[8 * (j + 1) + c] * M[c];
          g[j] += As * gj;
        }
      }
      double F = 0.0;
      const int rb = p.ipool[ds.fx_row + k], re = p.ipool[ds.fx_row + k + 1];
      for (int e = rb; e < re; ++e)
        F += L.theta[p.ipool[ds.md_param + p.ipool[ds.fx_mode + e]]] * p.dpool[ds.fx_coef + e];
      L.Hs[k] = hs;
      L.F1[k] = 1.0 + F;
      for (int j = 0; j < 4; ++j) L.Gs[j * K + k] = g[j];
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
    }
    for (int k = tid; k < K; k += NT) L.LH[k] = L.Hs[k] * L.F1[k];  // H, temporarily
    __syncthreads();
    block_scan<NT>(L.LH, L.C, K, false, L.red);

    // ---- energy scale and analysis edges
    const double c0 = pval(L.theta, ds.cidx[0], 0.0);
    const double c1 = pval(L.theta, ds.cidx[1], 0.0);
    const double c2 = pval(L.theta, ds.cidx[2], 0.0);
    const double bb = 1.0 + c1;
    if (tid == 0) {
      if (!(bb > 0.0 && bb + 2.0 * c2 * y0 > 0.0 && bb + 2.0 * c2 * yK > 0.0)) *L.flag |= ST_DOMAIN;
    }
    for (int i = tid; i < E; i += NT) {
      const double x = p.dpool[ds.edges + i];
      const double z = x - c0;
      const double disc = bb * bb + 4.0 * c2 * z;
      double y;
      if (disc < 0.0) y = c2 < 0.0 ? INFINITY : -INFINITY;
      else y = 2.0 * z / (bb + sqrt(disc));
      int k;
      double t = 0.0, X;
      if (!(y >= y0)) {
        k = -1;
        X = 0.0;
      } else if (y >= yK) {
        k = K;
        X = L.C[K];
      } else {
        k = (int)floor((y - y0) / wf);
        k = k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
        t = (y - (y0 + k * wf)) / wf;
        const double mk = L.Hs[k] * L.F1[k] / wf;
        const double dl = L.D[k], dh = L.D[k + 1];
        const double q = 0.5 * t * t - t * t * t / 3.0;
        X = L.C[k] + wf * (dl * (t - 0.5 * t * t) + dh * 0.5 * t * t + 6.0 * (mk - 0.5 * (dl + dh)) * q);
      }
      L.kidx[i] = k;
      L.eT[i] = t;
      L.eY[i] = y;
      L.eX[i] = X;
    }
    __syncthreads();

    // ---- expectations, deviance, lambda_mu
    double nll_loc = 0.0;
    for (int i = tid; i < Nb; i += NT) {
      double B = 0.0;
      for (int b = 0; b < ds.nbkg; ++b) {
        const BkgPlan bk = p.bkg[ds.bkg0 + b];
        const double R = pval(L.theta, bk.rate, 1.0);
        const double beta = bk.shape >= 0 ? pval(L.theta, p.ipool[bk.shape + i], 0.0) : 0.0;
        B += bk.scale * R * p.dpool[bk.tmpl + i] * (1.0 + beta);
      }
      const double mu = (L.eX[i + 1] - L.eX[i]) + B;
      if (a.mu_out) a.mu_out[ds.bins0 + i] = mu;
      double lam = 0.0;
      if (a.want_nll) {
        const double n = a.data[ds.data + i];
        if (!(mu > 0.0)) atomicOr(L.flag, ST_DOMAIN);
        nll_loc += (n > 0.0) ? (mu - n + n * log(n / mu)) : mu;
        lam = 1.0 - n / mu;
      }
      L.mu[i] = lam;
    }
    {
      double v[1] = {nll_loc};
      block_sum<NT, 1>(v, L.red);
      nll_total += v[0];
    }
    if (!a.want_grad) continue;

    // ---- adjoint: backgrounds
    for (int b = 0; b < ds.nbkg; ++b) {
      const BkgPlan bk = p.bkg[ds.bkg0 + b];
      const double R = pval(L.theta, bk.rate, 1.0);
      double gr = 0.0;
      for (int i = tid; i < Nb; i += NT) {
        const double beta = bk.shape >= 0 ? pval(L.theta, p.ipool[bk.shape + i], 0.0) : 0.0;
        const double st = bk.scale * p.dpool[bk.tmpl + i];
        gr += L.mu[i] * st * (1.0 + beta);
        if (bk.shape >= 0) {
          const int pi = p.ipool[bk.shape + i];
          if (pi >= 0) atomicAdd(&L.grad[pi], L.mu[i] * st * R);
        }
      }
      double v[1] = {gr};
      block_sum<NT, 1>(v, L.red);
      if (tid == 0 && bk.rate >= 0) L.grad[bk.rate] += v[0];
    }

    // ---- adjoint: per edge (lambda_X, energy-scale coefficients, spline pieces)
    double gc[4] = {0.0, 0.0, 0.0, 0.0};  // c0, c1, c2, top
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
      L.eX[i] = (k >= 0 && k < K) ? lx : 0.0;  // lambda_X of in-range edges
      L.eT[i] = em;
      L.eY[i] = elo;
      L.eH[i] = ehi;
    }
    block_sum<NT, 4>(gc, L.red);  // contains the needed barrier
    if (tid == 0) {
      for (int j = 0; j < 3; ++j)
        if (ds.cidx[j] >= 0) L.grad[ds.cidx[j]] += gc[j];
    }
    const double top = gc[3];

    // ---- gather per fine bin: lambda_C -> C, lambda_m (direct) -> LH, lambda_d -> Ld
    for (int k = tid; k <= K; k += NT) {
      const int b0 = lower_bound_int(L.kidx, E, k);
      const int b1 = lower_bound_int(L.kidx, E, k + 1);
      double lc = 0.0, lm = 0.0, ld = 0.0;
      if (k < K) {
        for (int i = b0; i < b1; ++i) {
          lc += L.eX[i];
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
    // C_k = sum_{j<k} H_j: lambda_H[j] collects sum_{k>j} lambda_C[k] (suffix sums -> Suf)
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
    if (tid == 0) {
      for (int j = 0; j < NSLOT; ++j)
        if (p.osc.slot_param[j] >= 0) L.grad[p.osc.slot_param[j]] += go[j];
    }

    // ---- flux modes (CSC gather per mode)
    for (int m = tid; m < ds.M; m += NT) {
      const int cb = p.ipool[ds.md_col + m], ce = p.ipool[ds.md_col + m + 1];
      double gm = 0.0;
      for (int e = cb; e < ce; ++e) gm += L.Ld[p.ipool[ds.md_k + e]] * p.dpool[ds.md_coef + e];
      atomicAdd(&L.grad[p.ipool[ds.md_param + m]], gm);
    }
    // ---- source norms: one wavefront per source
    {
      const int lane = tid & 63, wid = tid >> 6;
      for (int s = wid; s < S; s += NT / 64) {
        double gA = 0.0;
        for (int k = lane; k < K; k += 64) gA += L.LH[k] * a.scratch[s * K + k];
        gA = wave_sum(gA);
        if (lane == 0) {
          const int b = p.ipool[ds.srcnorm_ptr + s], e = p.ipool[ds.srcnorm_ptr + s + 1];
          for (int q = b; q < e; ++q) {
            double prod = 1.0;
            for (int r = b; r < e; ++r)
              if (r != q) prod *= L.theta[p.ipool[r]];
            atomicAdd(&L.grad[p.ipool[q]], gA * prod);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- priors (Eq. 6; third line of Eq. 9)
  double pr = 0.0;
  for (int j = tid; j < p.ngauss; j += NT) {
    const int i = p.ipool[p.gidx + j];
    const double z = L.theta[i] - p.dpool[p.gmean + j];
    const double inv = p.dpool[p.ginv + j];
    pr += 0.5 * z * z * inv;
    if (a.want_grad) atomicAdd(&L.grad[i], z * inv);
  }
  for (int bl = 0; bl < p.nblk; ++bl) {
    const int b = p.ipool[p.blk_ptr + bl], e = p.ipool[p.blk_ptr + bl + 1];
    const int n = e - b;
    const double* Vi = p.dpool + p.ipool[p.blk_inv + bl];
    for (int r = tid; r < n; r += NT) {
      double v = 0.0;
      for (int c = 0; c < n; ++c)
        v += Vi[(int64_t)r * n + c] * (L.theta[p.ipool[p.blk_idx + b + c]] - p.dpool[p.blk_mean + b + c]);
      const double rr = L.theta[p.ipool[p.blk_idx + b + r]] - p.dpool[p.blk_mean + b + r];
      pr += 0.5 * rr * v;
      if (a.want_grad) atomicAdd(&L.grad[p.ipool[p.blk_idx + b + r]], v);
    }
  }
  {
    double v[1] = {pr};
    block_sum<NT, 1>(v, L.red);
    nll_total += v[0];
  }

  const bool bad = (*L.flag & ST_DOMAIN) || !isfinite(nll_total);
  if (a.want_nll && tid == 0) a.out[0] = bad ? INFINITY : nll_total;
  if (a.want_grad && a.want_nll) {
    for (int i = tid; i < p.P; i += NT) a.out[1 + i] = bad ? 0.0 : L.grad[i];
  }
  if (a.status && tid == 0) *a.status = bad ? ST_DOMAIN : 0;
}

hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream) {
  const size_t lds = tail_lds_bytes(a.plan, nt);
  switch (nt) {
    case 256:
      hipLaunchKernelGGL(tail_kernel<256>, dim3(1), dim3(256), lds, stream, a);
      break;
    case 512:
      hipLaunchKernelGGL(tail_kernel<512>, dim3(1), dim3(512), lds, stream, a);
      break;
    default:
      hipLaunchKernelGGL(tail_kernel<1024>, dim3(1), dim3(1024), lds, stream, a);
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
  return hipFuncSetAttribute(reinterpret_cast<const void*>(tail_kernel<1024>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace nufold
