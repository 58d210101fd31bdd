"""Raster scan of the 3+1 sterile-neutrino hypothesis with test statistics
from ensembles of pseudo-experiments (paper, "Extensions of the framework",
sterile neutrino searches: the tested parameters are sin^2(2 theta14) and
dm2_41, the test statistic is that of Eq. 7, and its distribution comes from
pseudo-experiments where Wilks' theorem does not hold).

Raster: at each dm2_41 value m of the grid, the statistic of a sin^2(2 theta14)
value s is

    t(s; m) = 2 [ min_xi NLL(s, m, xi) - min_{s', xi} NLL(s', m, xi) ],

the profile of Eq. 7 in s at fixed m (one tested parameter per raster line).
Its distribution at (s, m) comes from Poisson pseudo-experiments drawn from
the expectation at (s, m) with the nuisance parameters at their conditional
best fit to the observed data; a point is excluded at confidence level CL
when the observed t exceeds the CL quantile of its ensemble.

Every fit is a batched device fit (nf_fit_batch: batched fold, adjoint
gradient, L-BFGS) and every expectation a batched device evaluation
(nf_expected_batch); this module only lays out start vectors, data rows and
fixed-parameter masks, draws the Poisson counts and takes quantiles.
"""
from __future__ import annotations

import time

import numpy as np

from . import nufold as nf


class RasterScan:
    def __init__(self, eng, desc, s_name="osc.sin2_2t14", m_name="osc.dm2_41", edm_tol=1e-7, max_iter=3000):
        self.eng = eng
        names = [p["name"] for p in desc["params"]]
        self.i_s, self.i_m = names.index(s_name), names.index(m_name)
        self.base_fixed = np.array([bool(p.get("fixed", False)) for p in desc["params"]])
        self.start = np.array([p["start"] for p in desc["params"]], dtype=np.float64)
        self.edm_tol, self.max_iter = edm_tol, max_iter
        self.nfits = 0
        self.fit_seconds = 0.0

    def _mask(self, fix_s):
        fx = self.base_fixed.copy()
        fx[self.i_m] = True
        fx[self.i_s] = bool(fix_s)
        return fx

    def _fit(self, starts, fix_s, data_idx):
        t0 = time.perf_counter()
        r = self.eng.fit_batch(starts, fixed=self._mask(fix_s), data_idx=np.asarray(data_idx, np.int32),
                               edm_tol=self.edm_tol, max_iter=self.max_iter)
        self.fit_seconds += time.perf_counter() - t0
        self.nfits += len(starts)
        return r

    def _free_fit(self, starts, data_idx):
        """Fits with sin^2(2 theta14) free, each run twice: the second from
        the first's result with a fresh minimiser history, so that a fit that
        stopped on a flat direction of the first history continues (its lower
        NLL is kept)."""
        a = self._fit(starts, False, data_idx)
        b = self._fit(a["theta"], False, data_idx)
        take = b["nll"] < a["nll"]
        out = dict(a)
        out["nll"] = np.where(take, b["nll"], a["nll"])
        out["theta"] = np.where(take[:, None], b["theta"], a["theta"])
        out["status"] = np.where(take, b["status"], a["status"])
        return out

    def _points(self, s_values, m_values, base=None):
        S, M = len(s_values), len(m_values)
        th = np.tile(self.start if base is None else base, (S * M, 1))
        th[:, self.i_s] = np.repeat(s_values, M)
        th[:, self.i_m] = np.tile(m_values, S)
        return th

    def statistic(self, rows, s_values, m_values, starts=None):
        """t(s, m) for observed-count rows (R x bins): R x S x M statistics and
        the conditional best-fit parameter vectors R x S x M x P.
        starts (optional, R x S x M x P): start vectors of the conditional fits."""
        rows = np.atleast_2d(np.asarray(rows, dtype=np.float64))
        R, S, M = rows.shape[0], len(s_values), len(m_values)
        self.eng.set_data_batch(rows)
        pts = self._points(s_values, m_values)
        st = (np.tile(pts, (R, 1)) if starts is None else np.asarray(starts, np.float64).reshape(R * S * M, -1))
        didx = np.repeat(np.arange(R), S * M)
        cond = self._fit(st, True, didx)
        nll0 = cond["nll"].reshape(R, S, M)
        # free s at each m, started from the best conditional point of its line
        best_s = np.argmin(nll0, axis=1)  # R x M
        th_c = cond["theta"].reshape(R, S, M, -1)
        fst = th_c[np.arange(R)[:, None], best_s, np.arange(M)[None, :]].reshape(R * M, -1)
        free = self._free_fit(fst, np.repeat(np.arange(R), M))
        nll1 = np.minimum(free["nll"].reshape(R, M), nll0.min(axis=1))
        t = 2.0 * (nll0 - nll1[:, None, :])
        return np.maximum(t, 0.0), th_c, cond["status"].reshape(R, S, M), free["status"].reshape(R, M)

    def ensemble(self, theta_points, n_pe, seed):
        """Poisson pseudo-experiments at each parameter vector (K x P):
        their statistics at the generating (s, m), K x n_pe."""
        K = theta_points.shape[0]
        mu, code = self.eng.expected_batch(theta_points)
        if code != nf.NF_OK:
            raise RuntimeError("expectation out of domain at a raster point")
        rng = np.random.default_rng(seed)
        rows = rng.poisson(np.repeat(mu, n_pe, axis=0)).astype(np.float64)
        self.eng.set_data_batch(rows)
        st = np.repeat(theta_points, n_pe, axis=0)
        didx = np.arange(K * n_pe)
        cond = self._fit(st, True, didx)
        free = self._free_fit(cond["theta"], didx)
        t = 2.0 * (cond["nll"] - np.minimum(free["nll"], cond["nll"]))
        return np.maximum(t, 0.0).reshape(K, n_pe), cond["status"], free["status"]

    def run(self, data_row, s_values, m_values, n_pe=100, cl=0.9, seed=0):
        """The raster scan of one observed data set: observed statistics,
        critical values from the ensembles and the excluded region."""
        t0 = time.perf_counter()
        self.nfits, self.fit_seconds = 0, 0.0
        t_obs, th_c, st0, st1 = self.statistic(data_row, s_values, m_values)
        S, M = len(s_values), len(m_values)
        t_pe, s_c, s_f = self.ensemble(th_c.reshape(S * M, -1), n_pe, seed)
        crit = np.quantile(t_pe, cl, axis=1).reshape(S, M)
        wall = time.perf_counter() - t0
        # fits: device fits run (the free fits' second passes included);
        # results: the fits behind the statistics, converged: those with status 0
        return dict(t_obs=t_obs[0], t_crit=crit, excluded=t_obs[0] > crit, t_pe=t_pe.reshape(S, M, n_pe),
                    fits=self.nfits, fit_seconds=self.fit_seconds, seconds=wall,
                    results=int(st0.size + st1.size + s_c.size + s_f.size),
                    converged=int(np.sum(st0 == 0) + np.sum(st1 == 0) + np.sum(s_c == 0) + np.sum(s_f == 0)))
