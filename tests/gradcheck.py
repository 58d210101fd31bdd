"""Per-component gradient agreement (test helper, CPU; oracle only).

A gradient component is compared at the scale that matters to a fit. Near a
minimum the NLL is locally quadratic; an error e_j in dNLL/dtheta_j moves the
minimum along theta_j by e_j / F_jj, i.e. by e_j / sqrt(F_jj) standard
deviations of theta_j, where F_jj is the curvature of the NLL in theta_j: the
Poisson Fisher information sum_i (dmu_i/dtheta_j)^2 / mu_i of the binned
likelihood (Eq. 3-5) plus the curvature of the priors (Eq. 6, 9). So the bar
per component is

    |g_j - g_oracle_j| <= tol * max(|g_oracle_j|, sqrt(F_jj)),

relative to the component itself, with a floor of one standard deviation's
worth of gradient. The derivatives dmu/dtheta_j come from the oracle's own
expectations by complex step, as its gradient does (the oracle's nll_grad
returns the same diagonal from its own complex steps with fisher=True).
"""
import numpy as np

from oracle import likelihood as LK
from oracle.fold import fold_all, fold_dataset

H_STEP = 1e-30


def fisher_diagonal(model, events, theta, folds=None):
    """F_jj = sum_{d,i} (dmu_di/dtheta_j)^2 / mu_di + prior curvature (V^-1)_jj."""
    theta = np.asarray(theta, dtype=np.float64)
    if folds is None:
        folds = fold_all(model, events, theta)
    mus, _ = LK.expected(model, events, theta, folds)
    F = np.zeros(model.P)
    for j in range(model.P):
        th = theta.astype(np.complex128)
        th[j] += 1j * H_STEP
        if j in model.osc_params:
            fj = [fold_dataset(model, ds, ev, model.osc_values(th)) for ds, ev in zip(model.datasets, events)]
        else:
            fj = folds
        mj, _ = LK.expected(model, events, th, fj)
        for mu0, mu in zip(mus, mj):
            dmu = np.imag(mu) / H_STEP
            pos = np.real(mu0) > 0
            F[j] += np.sum(dmu[pos] ** 2 / np.real(mu0)[pos])
    return F + LK.prior_curvature(model)


def component_errors(g, g_ref, F):
    """(worst floored ratio, its index, worst plain relative error over
    components with g_ref != 0, its index)."""
    g = np.asarray(g, dtype=np.float64)
    g_ref = np.asarray(g_ref, dtype=np.float64)
    d = np.abs(g - g_ref)
    scale = np.maximum(np.abs(g_ref), np.sqrt(np.maximum(F, 0.0)))
    scale = np.where(scale > 0, scale, 1.0)
    r = d / scale
    nz = np.abs(g_ref) > 0
    rel = np.where(nz, d / np.where(nz, np.abs(g_ref), 1.0), 0.0)
    return float(r.max()), int(r.argmax()), float(rel.max()), int(rel.argmax())


def check(g, g_ref, F, tol, what="", names=None):
    """Assert the per-component bar and print the worst figures."""
    r, jr, rel, jrel = component_errors(g, g_ref, F)
    nm = (lambda j: names[j]) if names is not None else (lambda j: str(j))
    print(f"[grad] {what}: worst per-component error {r:.2e} of max(|g|, sqrt F) at {nm(jr)}; "
          f"worst plain relative {rel:.2e} at {nm(jrel)}", flush=True)
    assert r <= tol, f"{what}: gradient component {nm(jr)} off by {r:.3e} of its scale (tol {tol:.0e})"
    return r, rel
