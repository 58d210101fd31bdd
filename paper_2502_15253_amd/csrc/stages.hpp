// Parameter-only parts of the bin stages (they depend on theta, not on the
// event fold): the flux factor 1 + F of a fine bin, the map of an analysis
// edge through the inverse energy-scale polynomial, the background
// expectation of an analysis bin and its factors, and the prior rows. The
// single evaluation computes them in extra workgroups of the fold launch,
// alongside the event stream; batched evaluations compute them in the
// bin-stage workgroup. Both use these functions, so both get identical values.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace nufold {

__device__ __forceinline__ double pval(const double* th, int idx, double dflt) {
  return idx >= 0 ? th[idx] : dflt;
}

// Inverse energy map of an analysis edge x (paper: detector-response
// polynomial f(E) = c0 + (1 + c1) E + c2 E^2, inverted in the stable form
// 2 (x - c0) / (b + sqrt(b^2 + 4 c2 (x - c0))), b = 1 + c1; a negative
// discriminant maps to +inf (c2 < 0) or -inf): the fine bin k it falls in
// (-1 below y_0, K at or above y_K), its position t in that bin, y itself and
// 1 / f'(y).
struct MappedEdge {
  double t, y, ifp;
  int k;
};
__device__ __forceinline__ MappedEdge map_edge(double X, double c0, double bb, double c2, double y0, double yK,
                                               double wf, double iwf, int K) {
  MappedEdge m;
  const double z = X - c0;
  const double disc = bb * bb + 4.0 * c2 * z;
  double y;
  if (disc < 0.0) y = c2 < 0.0 ? INFINITY : -INFINITY;
  else y = 2.0 * z / (bb + sqrt(disc));
  int k;
  double t = 0.0;
  if (!(y >= y0)) {
    k = -1;
  } else if (y >= yK) {
    k = K;
  } else {
    k = (int)floor((y - y0) * iwf);
    k = k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
    t = (y - (y0 + k * wf)) * iwf;
  }
  m.k = k;
  m.t = t;
  m.y = y;
  m.ifp = 1.0 / (bb + 2.0 * c2 * y);
  return m;
}

// Whether the energy map is increasing on the fine range (b > 0 and f' > 0
// at both ends).
__device__ __forceinline__ bool map_ok(double bb, double c2, double y0, double yK) {
  return bb > 0.0 && bb + 2.0 * c2 * y0 > 0.0 && bb + 2.0 * c2 * yK > 0.0;
}

// 1 + F of fine bin k: the flux basis row of fixed width fw (parameter -1:
// unused entry).
__device__ __forceinline__ double flux_factor(const double* th, const double* blob, const BlobLayout& BL, int fw,
                                              int k) {
  const int* fpar = reinterpret_cast<const int*>(blob + BL.fpar);
  double F = 0.0;
#pragma unroll
  for (int j = 0; j < FLUX_FW_MAX; ++j)
    if (j < fw) {
      const int q = fpar[k * fw + j];
      if (q >= 0) F += th[q] * blob[BL.fcf + k * fw + j];
    }
  return 1.0 + F;
}

// Background expectation of analysis bin i, sum_b R_b T_bi (1 + beta_bi),
// T_bi = scale_b template_bi, and per background dmu/dR_b = T (1 + beta) and
// dmu/dbeta_bi = R T (written through the two pointers, stride Nb).
__device__ __forceinline__ double background(const double* th, const double* blob, const BlobLayout& BL, int NB,
                                             int Nb, int i, double* bkr, double* bks) {
  const int* brt = reinterpret_cast<const int*>(blob + BL.brt);
  const int* shp = reinterpret_cast<const int*>(blob + BL.shp);
  double B = 0.0;
  for (int b = 0; b < NB; ++b) {
    const double T = blob[BL.bsc + b] * blob[BL.tmpl + b * Nb + i];
    const double R = pval(th, brt[b], 1.0);
    const double f = 1.0 + pval(th, shp[b * Nb + i], 0.0);
    B += R * T * f;
    bkr[b * Nb] = T * f;
    bks[b * Nb] = R * T;
  }
  return B;
}

// Prior row r (Eq. 6; third line of Eq. 9): v = its gradient contribution to
// the row's parameter, e = its NLL contribution. Rows < ngauss are
// independent Gaussians; the rest are rows of correlated blocks (V^-1 r).
__device__ __forceinline__ int prior_index(const DevPlan& p, int r) {
  if (r < p.ngauss) return p.ipool[p.gidx + r];
  const int bl = p.ipool[p.prow_blk + r - p.ngauss];
  const int b = p.ipool[p.blk_ptr + bl];
  return p.ipool[p.blk_idx + b + (r - p.ngauss - b)];
}
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

}  // namespace nufold
