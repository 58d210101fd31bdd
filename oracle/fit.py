"""Minimisation, EDM, covariance and profile scans (oracle; test infrastructure).

The paper minimises -ln L iteratively until the estimated distance to the
minimum (EDM) falls below a threshold ("Structure of the framework", Fig. 1),
uses the minimiser's covariance estimate at the minimum (goodness-of-fit
discussion under Eq. 8), and builds confidence intervals from the profile
statistic of Eq. 7, Lambda(eta) = 2 [min_xi NLL(eta, xi) - min NLL].

Here the minimiser is scipy's BFGS on the oracle NLL with its complex-step
gradient (a library routine as one step); EDM = 1/2 g^T H^-1 g with H the
central-difference Hessian of the complex-step gradient.
"""
import numpy as np
from scipy.optimize import minimize

from .likelihood import nll, nll_grad


def _free(model, fixed):
    fx = model.fixed.copy() if fixed is None else np.asarray(fixed, dtype=bool)
    return np.where(~fx)[0]


def hessian(model, events, data, theta, free, h=1e-5):
    n = len(free)
    Hm = np.zeros((n, n))
    for a, j in enumerate(free):
        tp = theta.copy(); tp[j] += h
        tm = theta.copy(); tm[j] -= h
        gp = nll_grad(model, events, data, tp)[1][free]
        gm = nll_grad(model, events, data, tm)[1][free]
        Hm[a] = (gp - gm) / (2 * h)
    return 0.5 * (Hm + Hm.T)


def fit(model, events, data, start, fixed=None, gtol=1e-7, maxiter=2000, want_cov=False):
    """Minimise the NLL over the free parameters from `start`.

    Returns dict(theta, nll, edm, cov (free x free or None), status, iters).
    """
    start = np.asarray(start, dtype=np.float64)
    free = _free(model, fixed)

    def fg(x):
        th = start.copy(); th[free] = x
        f, g = nll_grad(model, events, data, th)
        return f, g[free]

    res = minimize(fg, start[free], jac=True, method="BFGS",
                   options=dict(gtol=gtol, maxiter=maxiter))
    th = start.copy(); th[free] = res.x
    f, g = nll_grad(model, events, data, th)
    Hm = hessian(model, events, data, th, free)
    cov = np.linalg.inv(Hm)
    edm = 0.5 * g[free] @ cov @ g[free]
    return dict(theta=th, nll=float(f), edm=float(edm),
                cov=cov if want_cov else None, status=int(res.status), iters=int(res.nit))


def profile(model, events, data, start, eta_idx, eta_values, fixed=None, **kw):
    """Profile NLL over a list of eta points: eta fixed, nuisances minimised."""
    base_fixed = model.fixed.copy() if fixed is None else np.asarray(fixed, dtype=bool).copy()
    base_fixed[list(eta_idx)] = True
    out = []
    for eta in eta_values:
        th = np.asarray(start, dtype=np.float64).copy()
        th[list(eta_idx)] = eta
        out.append(fit(model, events, data, th, fixed=base_fixed, **kw)["nll"])
    return np.array(out)
