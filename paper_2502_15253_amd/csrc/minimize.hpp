// Device-resident minimiser step: limited-memory BFGS with a strong-Wolfe line
// search, run by the bin-stage kernel's serial workgroup right after it has
// produced f and grad f at the current trial point.
//
// The paper minimises -ln L until the estimated distance to the minimum (EDM)
// falls below a threshold ("Structure of the framework", Fig. 1). Here
// EDM = 1/2 g^T H g with H the L-BFGS inverse-Hessian estimate (Minuit's
// definition with its own metric), evaluated at every accepted point.
//
// State machine (one model evaluation per call):
//   INIT     first evaluation at the start point
//   BRACKET  trial steps alpha = 1, 2, 4, ... until the strong-Wolfe
//            conditions hold or a bracket is found (Nocedal & Wright, Alg. 3.5)
//   ZOOM     safeguarded cubic interpolation inside the bracket (Alg. 3.6)
//   FORCE    a zoom that ran out of steps re-evaluates its best sufficient-
//            decrease point and accepts it
// Convergence: EDM < tol and the last accepted step lowered f by less than
// tol (the limited-memory metric can underestimate the distance early on).
// Direction: two-loop recursion over the last m pairs (s, y) with
// H0 = gamma D, D a diagonal preconditioner (prior variances or a scale per
// parameter), gamma = s^T y / y^T D y of the newest pair. Fixed parameters
// have zero gradient and direction. A failed line search drops the history
// and retries along -D g; three failures end the fit.
#pragma once

#include "kernels.hpp"

namespace nufold {

constexpr int PH_INIT = 0, PH_BRACKET = 1, PH_ZOOM = 2, PH_FORCE = 3;
constexpr double LS_C1 = 1e-4, LS_C2 = 0.9, LS_AMAX = 64.0;
constexpr int LS_MAX_STEPS = 40;

template <int NT>
__device__ __forceinline__ double bdot(const double* a, const double* b, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += a[i] * b[i];
  double v[1] = {s};
  block_sum<NT, 1>(v, red);
  return v[0];
}

// Minimiser of the cubic through (a, fa, da), (b, fb, db), clipped to the
// inner 80% of [a, b]; bisection when the data are not finite.
__device__ inline double cubic_step(double a, double fa, double da, double b, double fb, double db) {
  const double lo = fmin(a, b), hi = fmax(a, b), w = hi - lo;
  double t = 0.5 * (a + b);
  if (isfinite(fa) && isfinite(fb) && isfinite(da) && isfinite(db)) {
    const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - da * db;
    if (disc >= 0.0) {
      const double sgn = (b > a) ? 1.0 : -1.0;
      const double d2 = sgn * sqrt(disc);
      const double den = db - da + 2.0 * d2;
      if (den != 0.0) t = b - (b - a) * (db + d2 - d1) / den;
    }
  } else if (isfinite(fa) && isfinite(da) && isfinite(fb)) {
    // quadratic through fa, da at a and fb at b
    const double h = b - a;
    const double c = (fb - fa - da * h) / (h * h);
    if (c > 0.0) t = a - da / (2.0 * c);
  }
  if (!(t >= lo + 0.1 * w && t <= hi - 0.1 * w)) t = 0.5 * (a + b);
  return t;
}

// Direction p = -H g (two-loop recursion); everything in LDS. Returns g^T p.
template <int NT>
__device__ double lbfgs_direction(const FitArgs& F, int P, int hn, int head, const double* g, double* q,
                                  double* r, double* pdir, const double* Sl, const double* Yl,
                                  const double* rho, const double* gam, double* alph, const double* D,
                                  const double* fr, double* red) {
  const int m = F.m;
  for (int i = threadIdx.x; i < P; i += NT) q[i] = g[i] * fr[i];
  for (int j = 0; j < hn; ++j) {
    const int idx = (head - 1 - j + m) % m;
    const double a = rho[idx] * bdot<NT>(Sl + (int64_t)idx * P, q, P, red);
    if (threadIdx.x == 0) alph[j] = a;
    for (int i = threadIdx.x; i < P; i += NT) q[i] -= a * Yl[(int64_t)idx * P + i];
  }
  const double gm = hn > 0 ? gam[(head - 1 + m) % m] : 1.0;
  for (int i = threadIdx.x; i < P; i += NT) r[i] = gm * D[i] * q[i];
  __syncthreads();
  for (int j = hn - 1; j >= 0; --j) {
    const int idx = (head - 1 - j + m) % m;
    const double b = rho[idx] * bdot<NT>(Yl + (int64_t)idx * P, r, P, red);
    const double a = alph[j];
    for (int i = threadIdx.x; i < P; i += NT) r[i] += (a - b) * Sl[(int64_t)idx * P + i];
  }
  for (int i = threadIdx.x; i < P; i += NT) pdir[i] = -r[i] * fr[i];
  return bdot<NT>(g, pdir, P, red);
}

// One minimiser step after an evaluation at theta_t (L.th): f_t, grad in Lg.
// lds: scratch of fit_lds_doubles(P, m) doubles.
template <int NT>
__device__ void lbfgs_step(const FitArgs& F, int P, const double* th_t, double f_t, const double* Lg,
                           double* lds, double* red) {
  FitHeader* H = F.hdr;
  const int tid = threadIdx.x;
  const int m = F.m;
  double* Sl = lds;                      // m P
  double* Yl = Sl + (int64_t)m * P;      // m P
  double* q = Yl + (int64_t)m * P;       // P
  double* r = q + P;                     // P
  double* pd = r + P;                    // P
  double* gx = pd + P;                   // P  gradient at the accepted point
  double* gt = gx + P;                   // P  masked trial gradient
  double* D = gt + P;                    // P
  double* fr = D + P;                    // P
  double* sm = fr + P;                   // small: rho m, gam m, alph m, misc 16
  double* rho = sm;
  double* gam = rho + m;
  double* alph = gam + m;
  double* misc = alph + m;

  // stage state (all threads read the header fields they need)
  const int phase = H->phase;
  int hn = H->hist_n, head = H->hist_head;
  for (int i = tid; i < P; i += NT) {
    D[i] = F.d2[i];
    fr[i] = F.freem[i];
    gx[i] = F.g[i];
    pd[i] = F.p[i];
    gt[i] = Lg[i] * F.freem[i];
  }
  for (int j = tid; j < m; j += NT) {
    rho[j] = F.rho[j];
    gam[j] = F.gam[j];
  }
  for (int j = 0; j < hn; ++j)
    for (int i = tid; i < P; i += NT) {
      Sl[(int64_t)j * P + i] = F.S[(int64_t)j * P + i];
      Yl[(int64_t)j * P + i] = F.Y[(int64_t)j * P + i];
    }
  __syncthreads();
  if (tid == 0) H->nevals += 1;

  bool accept = false, new_trial = false, restart = false;
  double alpha = H->alpha;

  if (phase == PH_INIT) {
    if (!isfinite(f_t)) {
      if (tid == 0) H->status = FIT_DOMAIN;
      return;
    }
    for (int i = tid; i < P; i += NT) {
      F.x[i] = th_t[i];
      gx[i] = gt[i];
    }
    if (tid == 0) H->f = f_t;
    restart = true;  // direction from -D g, first trial alpha = 1
  } else {
    const double f0 = H->f, d0 = H->dphi0;
    const double dphi = isfinite(f_t) ? bdot<NT>(gt, pd, P, red) : NAN;
    const bool armijo = isfinite(f_t) && f_t <= f0 + LS_C1 * alpha * d0;
    const bool curv = isfinite(dphi) && fabs(dphi) <= -LS_C2 * d0;
    double alo = H->a_lo, flo = H->f_lo, dlo = H->d_lo, ahi = H->a_hi, fhi = H->f_hi, dhi = H->d_hi;
    int ph = phase;
    if (ph == PH_FORCE) {
      if (isfinite(f_t) && f_t < f0) accept = true;
      else {
        restart = true;
        if (tid == 0) H->resets += 1;
      }
    } else if (ph == PH_BRACKET) {
      if (!armijo || (H->ls_steps > 0 && f_t >= H->f_prev)) {
        alo = H->a_prev; flo = H->f_prev; dlo = H->d_prev;
        ahi = alpha; fhi = isfinite(f_t) ? f_t : INFINITY; dhi = dphi;
        ph = PH_ZOOM;
      } else if (curv) {
        accept = true;
      } else if (dphi >= 0.0) {
        alo = alpha; flo = f_t; dlo = dphi;
        ahi = H->a_prev; fhi = H->f_prev; dhi = H->d_prev;
        ph = PH_ZOOM;
      } else {
        if (tid == 0) {
          H->a_prev = alpha;
          H->f_prev = f_t;
          H->d_prev = dphi;
        }
        alpha = fmin(2.0 * alpha, LS_AMAX);
        new_trial = true;
      }
    } else {  // ZOOM: the trial was inside the bracket
      if (!armijo || f_t >= flo) {
        ahi = alpha; fhi = isfinite(f_t) ? f_t : INFINITY; dhi = dphi;
      } else if (curv) {
        accept = true;
      } else {
        if (dphi * (ahi - alo) >= 0.0) {
          ahi = alo; fhi = flo; dhi = dlo;
        }
        alo = alpha; flo = f_t; dlo = dphi;
      }
    }
    if (!accept && ph == PH_ZOOM) {
      const int steps = H->ls_steps + 1;
      if (steps > LS_MAX_STEPS || fabs(ahi - alo) <= 1e-14 * fmax(1.0, fabs(alo))) {
        if (alo > 0.0 && flo < f0) {
          // accept the best sufficient-decrease point of the bracket: re-evaluate there
          alpha = alo;
          ph = PH_FORCE;
          new_trial = true;
        } else {
          restart = true;
          if (tid == 0) H->resets += 1;
        }
      } else {
        alpha = cubic_step(alo, flo, dlo, ahi, fhi, dhi);
        new_trial = true;
      }
    }
    if (tid == 0) {
      H->phase = ph;
      H->a_lo = alo; H->f_lo = flo; H->d_lo = dlo;
      H->a_hi = ahi; H->f_hi = fhi; H->d_hi = dhi;
      if (new_trial) H->ls_steps += 1;
    }
    if (accept) {
      // s = theta_t - x, y = g_t - g_x; push when curvature is positive
      for (int i = tid; i < P; i += NT) {
        q[i] = (th_t[i] - F.x[i]) * fr[i];
        r[i] = gt[i] - gx[i];
      }
      __syncthreads();
      const double sy = bdot<NT>(q, r, P, red);
      for (int i = tid; i < P; i += NT) pd[i] = D[i] * r[i];
      __syncthreads();
      const double yDy = bdot<NT>(r, pd, P, red);
      const double ss = bdot<NT>(q, q, P, red);
      const double yy = bdot<NT>(r, r, P, red);
      if (sy > 1e-12 * sqrt(ss * yy) && yDy > 0.0) {
        const int slot = head;
        for (int i = tid; i < P; i += NT) {  // ring slot, in global memory and in LDS
          F.S[(int64_t)slot * P + i] = q[i];
          F.Y[(int64_t)slot * P + i] = r[i];
          Sl[(int64_t)slot * P + i] = q[i];
          Yl[(int64_t)slot * P + i] = r[i];
        }
        if (tid == 0) {
          F.rho[slot] = 1.0 / sy;
          F.gam[slot] = sy / yDy;
        }
        __syncthreads();
        rho[slot] = 1.0 / sy;
        gam[slot] = sy / yDy;
        head = (head + 1) % m;
        hn = hn < m ? hn + 1 : m;
      }
      for (int i = tid; i < P; i += NT) {
        F.x[i] = th_t[i];
        gx[i] = gt[i];
      }
      if (tid == 0) {
        H->df = H->f - f_t;
        H->f = f_t;
        H->iter += 1;
        H->hist_n = hn;
        H->hist_head = head;
      }
      __syncthreads();
    }
  }

  if (accept || restart) {
    if (restart) {
      hn = 0;
      if (tid == 0) {
        H->hist_n = 0;
        H->hist_head = 0;
      }
      head = 0;
    }
    __syncthreads();
    double d0 = lbfgs_direction<NT>(F, P, hn, head, gx, q, r, pd, Sl, Yl, rho, gam, alph, D, fr, red);
    if (!(d0 < 0.0) && hn > 0) {  // not a descent direction: drop the history
      hn = 0;
      head = 0;
      d0 = lbfgs_direction<NT>(F, P, 0, 0, gx, q, r, pd, Sl, Yl, rho, gam, alph, D, fr, red);
      if (tid == 0) {
        H->hist_n = 0;
        H->hist_head = 0;
      }
    }
    const double edm = -0.5 * d0;
    int st = FIT_RUNNING;
    const bool small_step = H->iter > 0 && H->df < fmax(H->edm_tol, 1e-15 * fabs(H->f));
    if (!(d0 < 0.0) || (edm < H->edm_tol && small_step)) st = FIT_CONVERGED;
    else if (H->iter >= H->max_iter) st = FIT_MAXITER;
    else if (H->resets > 3) st = FIT_LSFAIL;
    for (int i = tid; i < P; i += NT) {
      F.g[i] = gx[i];
      F.p[i] = pd[i];
      F.theta_next[i] = F.x[i] + pd[i];
    }
    if (tid == 0) {
      H->edm = edm;
      H->dphi0 = d0;
      H->alpha = 1.0;
      H->phase = PH_BRACKET;
      H->ls_steps = 0;
      H->a_prev = 0.0;
      H->f_prev = H->f;
      H->d_prev = d0;
      H->status = st;
    }
  } else if (new_trial) {
    for (int i = tid; i < P; i += NT) F.theta_next[i] = F.x[i] + alpha * pd[i];
    if (tid == 0) H->alpha = alpha;
  }
  __syncthreads();
}

}  // namespace nufold
