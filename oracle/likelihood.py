"""Binned Poisson likelihood with priors; complex-step gradient (oracle; test infrastructure).

Eq. 3-5: independent Poisson bins; Eq. 6 and the third line of Eq. 9: Gaussian
priors on single parameters and on correlated groups. Minimising
-ln L is done here in the deviance-normalised form (Baker & Cousins 1984,
halved), which drops theta-independent constants:
  NLL = sum_{d,i} [mu - n + n ln(n/mu)]          (n = 0 term: mu)
      + 1/2 sum_j ((theta_j - mean_j)/sigma_j)^2
      + 1/2 sum_blocks r^T V^-1 r,  r = theta_block - mean_block.
Then 2 NLL at the best fit is the saturated-model statistic Lambda_S of Eq. 8
(the saturated model mu = n has zero prior penalty), and differences of 2 NLL
are the profile statistic of Eq. 7.
If any expectation is <= 0 (or the energy map leaves its domain) the NLL is
+inf and the gradient is reported as zero.

Gradient: complex step (Squire & Trapp 1998), dNLL/dtheta_j = Im NLL(theta + i h e_j)/h
with h = 1e-30, exact to rounding and independent of any hand-derived adjoint.
Only the oscillation parameters change the event fold; every other parameter
re-evaluates the bin-level stages from the cached real fold.
"""
import numpy as np

from .fold import fold_all, fold_dataset
from .spectrum import rescale, energy_coeffs, energy_map_valid, rebin, backgrounds

H_STEP = 1e-30


def expected_dataset(ds, S, theta):
    """(signal s_i, background B_i, energy map valid) for one dataset."""
    c = energy_coeffs(ds, theta)
    ok = energy_map_valid(ds, c)
    H = rescale(ds, S, theta)
    s = rebin(ds, H, c)
    return s, backgrounds(ds, theta), ok


def expected(model, events, theta, folds=None):
    """Per-dataset expectations mu_i = s_i + B_i, plus a domain flag."""
    if folds is None:
        folds = fold_all(model, events, theta)
    mus, ok = [], True
    for ds, S in zip(model.datasets, folds):
        s, B, v = expected_dataset(ds, S, theta)
        ok = ok and v
        mus.append(s + B)
    return mus, ok


def poisson_deviance_half(n, mu):
    """sum [mu - n + n ln(n/mu)] with the n = 0 term equal to mu."""
    n = np.asarray(n, dtype=np.float64)
    pos = n > 0
    safe_n = np.where(pos, n, 1.0)
    term = np.where(pos, mu - n + safe_n * np.log(safe_n / mu), mu)
    return term.sum()


def prior_terms(model, theta):
    out = 0.0
    for i, mean, sigma in model.gauss:
        z = (theta[i] - mean) / sigma
        out = out + 0.5 * z * z
    for idx, mean, cov in model.blocks:
        r = theta[idx] - mean
        out = out + 0.5 * (r @ np.linalg.solve(cov, r))
    return out


def nll_from_mu(model, mus, ok, data, theta):
    if not ok or any(np.any(np.real(mu) <= 0) for mu in mus):
        return np.inf
    total = 0.0
    for mu, n in zip(mus, data):
        total = total + poisson_deviance_half(n, mu)
    return total + prior_terms(model, theta)


def nll(model, events, data, theta, folds=None):
    theta = np.asarray(theta)
    mus, ok = expected(model, events, theta, folds)
    return nll_from_mu(model, mus, ok, data, theta)


def prior_curvature(model):
    """Diagonal of the priors' second derivatives: 1/sigma^2 and diag(V^-1)."""
    c = np.zeros(model.P)
    for i, mean, sigma in model.gauss:
        c[i] += 1.0 / sigma ** 2
    for idx, mean, cov in model.blocks:
        c[np.asarray(idx)] += np.diag(np.linalg.inv(cov))
    return c


def nll_grad(model, events, data, theta, folds=None, fisher=False):
    """(NLL, gradient) with the complex-step gradient. With fisher=True also
    the diagonal of the Fisher information of the Poisson bins plus the prior
    curvature, F_jj = sum_i (dmu_i/dtheta_j)^2 / mu_i + prior, whose
    derivatives of mu come from the same complex steps (returned third)."""
    theta = np.asarray(theta, dtype=np.float64)
    if folds is None:
        folds = fold_all(model, events, theta)
    mus0, ok0 = expected(model, events, theta, folds)
    f0 = nll_from_mu(model, mus0, ok0, data, theta)
    g = np.zeros(model.P)
    F = prior_curvature(model) if fisher else None
    if not np.isfinite(f0):
        return (f0, g, F) if fisher else (f0, g)
    for j in range(model.P):
        th = theta.astype(np.complex128)
        th[j] += 1j * H_STEP
        if j in model.osc_params:
            fj = [fold_dataset(model, ds, ev, model.osc_values(th))
                  for ds, ev in zip(model.datasets, events)]
        else:
            fj = folds
        mus, ok = expected(model, events, th, fj)
        g[j] = np.imag(nll_from_mu(model, mus, ok, data, th)) / H_STEP
        if fisher:
            for mu0, mu in zip(mus0, mus):
                dmu = np.imag(mu) / H_STEP
                F[j] += np.sum(dmu ** 2 / np.real(mu0))
    return (float(f0), g, F) if fisher else (float(f0), g)


def saturated_statistic(nll_min):
    """Lambda_S of Eq. 8 from the deviance-normalised NLL at the best fit."""
    return 2.0 * nll_min
