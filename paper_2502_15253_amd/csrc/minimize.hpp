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
// Along directions the history has not explored, H is gamma D, and gamma
// (set by the stiffest recent directions) can make the EDM there far too
// small for a parameter whose D is only a scale guess (no prior, so its
// variance is unknown; such entries of D are stored negated). So a point
// that passes is checked once more with max(gamma, 1) in place of gamma on
// those parameters; if that EDM is not below tol, the fit goes on along the
// direction of the re-check (at most MAX_CHECKS times per fit). After such a
// re-check, a line search that fails or ends only by its forced step marks a
// domain boundary or a flat ridge rather than a missed minimum: the fit
// stops there as converged (its point passed the rule before).
// Direction: two-loop recursion over the last m pairs (s, y) with
// H0 = gamma D, D a diagonal preconditioner (prior variances or a scale per
// parameter), gamma = s^T y / y^T D y of the newest pair. Fixed parameters
// have zero gradient and direction. A failed line search drops the history
// and retries along -D g; a forced step that lowers f by less than tol also
// counts as a failure; more than three failures end the fit.
#pragma once

#include "kernels.hpp"

namespace nufold {

constexpr int PH_INIT = 0, PH_BRACKET = 1, PH_ZOOM = 2, PH_FORCE = 3;
constexpr double LS_C1 = 1e-4, LS_C2 = 0.9, LS_AMAX = 64.0;
constexpr int LS_MAX_STEPS = 40;
constexpr int MAX_CHECKS = 4;

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
// gfloor: lower bound on the scale gamma of H0 = gamma D on the parameters
// whose D is a scale guess (negative in F.d2).
template <int NT>
__device__ double lbfgs_direction(const FitArgs& F, int P, int hn, int head, const double* g, double* q,
                                  double* r, double* pdir, const double* Sl, const double* Yl,
                                  const double* rho, const double* gam, double* alph, const double* D,
                                  const double* fr, double* red, double gfloor = 0.0) {
  const int m = F.m;
  for (int i = threadIdx.x; i < P; i += NT) q[i] = g[i] * fr[i];
  for (int j = 0; j < hn; ++j) {
    const int idx = (head - 1 - j + m) % m;
    const double a = rho[idx] * bdot<NT>(Sl + (int64_t)idx * P, q, P, red);
    if (threadIdx.x == 0) alph[j] = a;
    for (int i = threadIdx.x; i < P; i += NT) q[i] -= a * Yl[(int64_t)idx * P + i];
  }
  const double gm = hn > 0 ? gam[(head - 1 + m) % m] : 1.0;
  if (gfloor > gm) {
    const double gg = gfloor;
    for (int i = threadIdx.x; i < P; i += NT) r[i] = (F.d2[i] < 0.0 ? gg : gm) * D[i] * q[i];
  } else {
    for (int i = threadIdx.x; i < P; i += NT) r[i] = gm * D[i] * q[i];
  }
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
//
// Every thread copies the fit header into registers before the first barrier
// and takes each decision from that copy, updating it identically; thread 0
// stores it back after the last barrier. No thread reads a header field that
// another thread of the same step may already have written, so all wavefronts
// take the same branches and pass the same barriers.
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

  FitHeader h = *H;  // private snapshot; written back by thread 0 at the end
  int hn = h.hist_n, head = h.hist_head;
  const bool forced_trial = h.phase == PH_FORCE;
  for (int i = tid; i < P; i += NT) {
    D[i] = fabs(F.d2[i]);
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
  h.nevals += 1;

  bool accept = false, new_trial = false, restart = false;
  double alpha = h.alpha;

  if (h.phase == PH_INIT) {
    if (!isfinite(f_t)) {
      h.status = FIT_DOMAIN;
      if (tid == 0) *H = h;
      return;
    }
    for (int i = tid; i < P; i += NT) {
      F.x[i] = th_t[i];
      gx[i] = gt[i];
    }
    h.f = f_t;
    restart = true;  // direction from -D g, first trial alpha = 1
  } else {
    const double f0 = h.f, d0 = h.dphi0;
    const double dphi = isfinite(f_t) ? bdot<NT>(gt, pd, P, red) : NAN;
    const bool armijo = isfinite(f_t) && f_t <= f0 + LS_C1 * alpha * d0;
    const bool curv = isfinite(dphi) && fabs(dphi) <= -LS_C2 * d0;
    double alo = h.a_lo, flo = h.f_lo, dlo = h.d_lo, ahi = h.a_hi, fhi = h.f_hi, dhi = h.d_hi;
    int ph = h.phase;
    if (ph == PH_FORCE) {
      if (isfinite(f_t) && f_t < f0) {
        accept = true;
        // a forced step that gains next to nothing (e.g. along a domain
        // boundary the direction keeps pointing across) counts as a failure
        if (f0 - f_t < fmax(h.edm_tol, 1e-15 * fabs(f0))) h.resets += 1;
      } else {
        restart = true;
        h.resets += 1;
      }
    } else if (ph == PH_BRACKET) {
      if (!armijo || (h.ls_steps > 0 && f_t >= h.f_prev)) {
        alo = h.a_prev; flo = h.f_prev; dlo = h.d_prev;
        ahi = alpha; fhi = isfinite(f_t) ? f_t : INFINITY; dhi = dphi;
        ph = PH_ZOOM;
      } else if (curv) {
        accept = true;
      } else if (dphi >= 0.0) {
        alo = alpha; flo = f_t; dlo = dphi;
        ahi = h.a_prev; fhi = h.f_prev; dhi = h.d_prev;
        ph = PH_ZOOM;
      } else {
        h.a_prev = alpha;
        h.f_prev = f_t;
        h.d_prev = dphi;
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
      const int steps = h.ls_steps + 1;
      if (steps > LS_MAX_STEPS || fabs(ahi - alo) <= 1e-14 * fmax(1.0, fabs(alo))) {
        if (alo > 0.0 && flo < f0) {
          // accept the best sufficient-decrease point of the bracket: re-evaluate there
          alpha = alo;
          ph = PH_FORCE;
          new_trial = true;
        } else {
          restart = true;
          h.resets += 1;
        }
      } else {
        alpha = cubic_step(alo, flo, dlo, ahi, fhi, dhi);
        new_trial = true;
      }
    }
    h.phase = ph;
    h.a_lo = alo; h.f_lo = flo; h.d_lo = dlo;
    h.a_hi = ahi; h.f_hi = fhi; h.d_hi = dhi;
    if (new_trial) h.ls_steps += 1;
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
      h.df = h.f - f_t;
      h.f = f_t;
      h.iter += 1;
      __syncthreads();
    }
  }

  if (accept || restart) {
    if (restart) {
      hn = 0;
      head = 0;
    }
    __syncthreads();
    double d0 = lbfgs_direction<NT>(F, P, hn, head, gx, q, r, pd, Sl, Yl, rho, gam, alph, D, fr, red);
    if (!(d0 < 0.0) && hn > 0) {  // not a descent direction: drop the history
      hn = 0;
      head = 0;
      d0 = lbfgs_direction<NT>(F, P, 0, 0, gx, q, r, pd, Sl, Yl, rho, gam, alph, D, fr, red);
    }
    double edm = -0.5 * d0;
    int st = FIT_RUNNING;
    const bool small_step = h.iter > 0 && h.df < fmax(h.edm_tol, 1e-15 * fabs(h.f));
    const bool stuck = h.checks > 0 && (restart || (accept && forced_trial));
    bool conv = stuck || !(d0 < 0.0) || (edm < h.edm_tol && small_step);
    if (!stuck && conv && d0 < 0.0 && hn > 0 && h.checks < MAX_CHECKS && gam[(head - 1 + m) % m] < 1.0) {
      // re-check with gamma at least 1 (uniform: every thread holds hn, head, gam)
      const double d1 = lbfgs_direction<NT>(F, P, hn, head, gx, q, r, pd, Sl, Yl, rho, gam, alph, D, fr, red, 1.0);
      if (d1 < 0.0 && -0.5 * d1 >= h.edm_tol) {
        conv = false;  // go on along the re-check's direction
        h.checks += 1;
        d0 = d1;
        edm = -0.5 * d1;
      }
    }
    if (conv) st = FIT_CONVERGED;
    else if (h.iter >= h.max_iter) st = FIT_MAXITER;
    else if (h.resets > 3) st = FIT_LSFAIL;
    for (int i = tid; i < P; i += NT) {
      F.g[i] = gx[i];
      F.p[i] = pd[i];
      F.theta_next[i] = F.x[i] + pd[i];
    }
    h.edm = edm;
    h.dphi0 = d0;
    h.alpha = 1.0;
    h.phase = PH_BRACKET;
    h.ls_steps = 0;
    h.a_prev = 0.0;
    h.f_prev = h.f;
    h.d_prev = d0;
    h.status = st;
  } else if (new_trial) {
    for (int i = tid; i < P; i += NT) F.theta_next[i] = F.x[i] + alpha * pd[i];
    h.alpha = alpha;
  }
  h.hist_n = hn;
  h.hist_head = head;
  __syncthreads();
  if (tid == 0) *H = h;
}

}  // namespace nufold
