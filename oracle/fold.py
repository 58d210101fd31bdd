"""Event binning and the oscillation-weighted fold (oracle; test infrastructure).

Step 1 of the signal calculation (paper, "Structure of the framework"): every
MC event is weighted by the survival probability of Eq. 1 (or the exact
three-flavour form that Eq. 10 rewrites) at its own L/E, and the weighted
events are summed into the fine reconstructed-energy bins of its dataset,
separately per reactor source:  S[s][k] = sum_{e in (s,k)} w_e P(L_s / E_true,e).

Fine bins are uniform, y_k = y0 + k*width, half-open [y_k, y_{k+1}); an event
on an edge belongs to the upper bin; events outside [y_0, y_K) are dropped.
"""
import numpy as np

from .oscillation import prob_eq1, prob_3nu, prob_4nu, prob_3nu_matter


def fine_edges(ds):
    return ds.y0 + ds.wf * np.arange(ds.K + 1, dtype=np.float64)


def fine_grid_from_edges(edges):
    """Uniform fine grid whose width is the greatest common divisor of the
    analysis bin widths (paper, Double Chooz likelihood: the flux parameters
    sit on the GCD grid). Widths are taken on a 1e-9 MeV integer lattice."""
    e = np.asarray(edges, dtype=np.float64)
    q = np.rint(np.diff(e) * 1e9).astype(np.int64)
    g = int(np.gcd.reduce(q))
    width = g * 1e-9
    n = int(round((e[-1] - e[0]) / width))
    return float(e[0]), width, n


def bin_events(ds, e_reco):
    """Fine-bin index of each event (largest k with y_k <= E_rec) and an in-range mask."""
    k = np.searchsorted(fine_edges(ds), e_reco, side="right") - 1
    keep = (k >= 0) & (k < ds.K)
    return k, keep


def baseline_over_energy(ds, events):
    src = np.asarray(events["source"], dtype=np.int64)
    if src.size and (src.min() < 0 or src.max() >= ds.S):
        raise ValueError("source index out of range")
    return ds.baselines[src] / np.asarray(events["e_true"], dtype=np.float64)


def survival(model, u, osc, L=None):
    """P at u = L/E (L in m, needed by the matter form only)."""
    if model.formula == "eq1":
        return prob_eq1(u, *osc)
    if model.formula == "3nu_matter":
        return prob_3nu_matter(u, L, *osc, model.rho_ye)
    if model.formula == "4nu":
        s13, m31, s14, m41 = osc
        s12, m21 = model.osc_constants
        return prob_4nu(u, s12, s13, m21, m31, s14, m41)
    return prob_3nu(u, *osc)


def fold_dataset(model, ds, events, osc):
    """S[s][k] for one dataset; complex-valued when `osc` is complex."""
    k, keep = bin_events(ds, events["e_reco"])
    u = baseline_over_energy(ds, events)[keep]
    w = np.asarray(events["weight"], dtype=np.float64)[keep]
    src = np.asarray(events["source"], dtype=np.int64)[keep]
    seg = src * ds.K + k[keep]
    p = survival(model, u, osc, ds.baselines[src])
    a = w * p
    n = ds.S * ds.K
    if np.iscomplexobj(a):
        out = (np.bincount(seg, weights=a.real, minlength=n)
               + 1j * np.bincount(seg, weights=a.imag, minlength=n))
    else:
        out = np.bincount(seg, weights=a, minlength=n)
    return out.reshape(ds.S, ds.K)


def fold_all(model, events, theta):
    osc = model.osc_values(theta)
    return [fold_dataset(model, ds, ev, osc) for ds, ev in zip(model.datasets, events)]


def dropped_events(model, events):
    return [int((~bin_events(ds, ev["e_reco"])[1]).sum()) for ds, ev in zip(model.datasets, events)]
