"""Seeded synthetic workloads: MC event samples, model descriptions, pseudo-data.

This module only draws random numbers and lays out the *inputs* of a fit:
events (true energy, reconstructed energy, source, weight), the model
description (parameters, priors, binning, flux-shape basis, background
templates) and Poisson pseudo-data drawn around a given expectation. It holds
none of the likelihood arithmetic (oscillation, folding, energy scale, Poisson
terms); both the HIP engine and the test oracle read what it produces.

Workloads stand in for the Double Chooz MC/data and the JUNO-like study of the
paper (Sections "Input model of Double Chooz" and "Application to medium
baseline reactor measurements"), which are not available: the shapes (datasets,
bin counts, parameter counts, dense covariances, baselines) follow those
sections, the numbers are synthetic.

Units: energies in MeV, baselines in m, dm2_ee and dm2_31 in 1e-3 eV^2,
dm2_21 in 1e-5 eV^2.
"""
from __future__ import annotations

import json
import numpy as np

TRUTH = dict(sin2_2t13=0.085, dm2_ee=2.50, sin2_t12=0.307, dm2_21=7.53,
             sin2_t13=0.0218, dm2_31=2.53)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def event_seed(config: int, dataset: int) -> int:
    return 1000 + 10 * config + dataset


def data_seed(config: int) -> int:
    return 2000 + config


def pseudo_seed(j: int) -> int:
    return 3000 + j


def cov_seed(dataset: int) -> int:
    return 4000 + dataset


# --------------------------------------------------------------------------
# events
# --------------------------------------------------------------------------

def falling_spectrum(e):
    """Synthetic reactor-like falling spectrum exp(-0.8 E) E^2 (MC weight shape)."""
    return np.exp(-0.8 * e) * e * e


def make_events(n, e_lo, e_hi, n_sources, rate, seed, resolution="c1",
                source_fracs=None):
    """Uniform true energies on [e_lo, e_hi], weighted to the falling spectrum.

    resolution "c1": E_rec = E - 0.78 + N(0, 0.08 sqrt(E))
    resolution "c3": E_vis = E - 0.78, E_rec = E_vis + N(0, 0.03 sqrt(E_vis))
    Weights sum to `rate` (expected signal events before oscillation).
    """
    rng = rng_for(seed)
    e_true = rng.uniform(e_lo, e_hi, n)
    z = rng.standard_normal(n)
    if resolution == "c1":
        e_reco = e_true - 0.78 + z * 0.08 * np.sqrt(e_true)
    elif resolution == "c3":
        e_vis = e_true - 0.78
        e_reco = e_vis + z * 0.03 * np.sqrt(e_vis)
    else:
        raise ValueError(resolution)
    if source_fracs is None:
        source = rng.integers(0, n_sources, n).astype(np.uint8)
    else:
        source = rng.choice(n_sources, size=n, p=source_fracs).astype(np.uint8)
    phi = falling_spectrum(e_true)
    weight = (rate * phi / phi.sum()).astype(np.float32)
    return dict(e_true=e_true, e_reco=e_reco, source=source, weight=weight)


# --------------------------------------------------------------------------
# model-description helpers (inputs: binning, bases, templates)
# --------------------------------------------------------------------------

def uniform_edges(lo, hi, n):
    return [float(lo + (hi - lo) * i / n) for i in range(n + 1)]


def fine_centres(y0, width, n):
    return [y0 + (k + 0.5) * width for k in range(n)]


def hat_basis(centres, nodes):
    """Piecewise-linear ('hat') basis evaluated at fine-bin centres.

    Returns an M x K list; outside the node range the end mode is 1 (clamped).
    """
    nodes = list(nodes)
    M, K = len(nodes), len(centres)
    B = [[0.0] * K for _ in range(M)]
    for k, y in enumerate(centres):
        if y <= nodes[0]:
            B[0][k] = 1.0
        elif y >= nodes[-1]:
            B[M - 1][k] = 1.0
        else:
            j = int(np.searchsorted(nodes, y, side="right")) - 1
            t = (y - nodes[j]) / (nodes[j + 1] - nodes[j])
            B[j][k] = 1.0 - t
            B[j + 1][k] = t
    return B


def indicator_basis(centres, edges):
    """Mode m = 1 on the fine bins inside analysis bin m; margins clamp to the end modes."""
    M = len(edges) - 1
    B = [[0.0] * len(centres) for _ in range(M)]
    for k, y in enumerate(centres):
        m = int(np.searchsorted(edges, y, side="right")) - 1
        B[min(max(m, 0), M - 1)][k] = 1.0
    return B


def template_flat(edges):
    w = np.diff(np.asarray(edges))
    return list(w / w.sum())


def template_exp(edges, tau):
    e = np.asarray(edges)
    t = np.exp(-e[:-1] / tau) - np.exp(-e[1:] / tau)
    return list(t / t.sum())


def template_seeded(edges, rng):
    e = np.asarray(edges)
    tau = rng.uniform(1.0, 4.0)
    c = 0.5 * (e[:-1] + e[1:])
    eps = rng.uniform(-1.0, 1.0, len(c))
    t = np.exp(-c / tau) * (1.0 + 0.1 * eps)
    return list(t / t.sum())


def correlated_cov(dim, seed, sigma):
    """Dense seeded covariance: A ~ N(0,1)^{dim x dim}, C = A A^T + dim I scaled to unit diagonal."""
    A = rng_for(seed).standard_normal((dim, dim))
    C = A @ A.T + dim * np.eye(dim)
    s = np.sqrt(np.diag(C))
    R = C / np.outer(s, s)
    return (sigma * sigma * R).tolist()


def param(name, start, prior=None, fixed=False):
    return dict(name=name, start=float(start),
                prior=None if prior is None else [float(prior[0]), float(prior[1])],
                fixed=bool(fixed))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

C1_EDGES = uniform_edges(1.0, 8.0, 40)
C1_FINE = dict(y0=0.3, width=0.175, n=59)
C3_EDGES = uniform_edges(0.8, 12.0, 400)
C3_FINE = dict(y0=0.576, width=0.028, n=416)


def escale_params(prefix):
    return [param(prefix + "c0", 0.0, (0.0, 0.02)),
            param(prefix + "c1", 0.0, (0.0, 0.01)),
            param(prefix + "c2", 0.0, (0.0, 0.002))]


def config1_model():
    """One detector at 1050 m, Eq. 1, 40 bins on 1-8 MeV, 12 parameters."""
    T = TRUTH
    params = [
        param("osc.sin2_2t13", T["sin2_2t13"]),
        param("osc.dm2_ee", T["dm2_ee"], (2.50, 0.10)),
        param("norm", 1.0, (1.0, 0.02)),
        *escale_params("escale."),
        param("bkg.flat.rate", 1.0, (1.0, 0.10)),
        param("bkg.exp.rate", 1.0),
        *[param(f"flux[{m}]", 0.0, (0.0, 0.05)) for m in range(4)],
    ]
    fine = C1_FINE
    cen = fine_centres(fine["y0"], fine["width"], fine["n"])
    ds = dict(
        name="FD", fine=dict(fine), edges=C1_EDGES,
        sources=[dict(baseline_m=1050.0, norm=[])],
        norm=["norm"],
        flux=dict(params=[f"flux[{m}]" for m in range(4)],
                  basis=hat_basis(cen, [1.0, 10.0 / 3.0, 17.0 / 3.0, 8.0])),
        escale=dict(c0="escale.c0", c1="escale.c1", c2="escale.c2"),
        backgrounds=[
            dict(name="flat", rate="bkg.flat.rate", scale=1.5e3,
                 template=template_flat(C1_EDGES), shape=None),
            dict(name="exp", rate="bkg.exp.rate", scale=2.0e3,
                 template=template_exp(C1_EDGES, 2.0), shape=None),
        ],
    )
    return dict(
        version=1,
        osc=dict(formula="eq1", sin2_2t13=dict(param="osc.sin2_2t13"),
                 dm2_ee=dict(param="osc.dm2_ee"),
                 sin2_t12=dict(value=T["sin2_t12"]), dm2_21=dict(value=T["dm2_21"])),
        params=params, cov_priors=[], datasets=[ds])


def config1_events(n=100_000):
    return [make_events(n, 1.8, 10.0, 1, 1.0e5, event_seed(1, 0), "c1")]


def config2_model():
    """FD-I, FD-II (1050 m) and ND (400 m), two reactors each, 3 x 40 bins, 302 parameters."""
    T = TRUTH
    names = ["FD-I", "FD-II", "ND"]
    rates = [4.0e4, 1.0e5, 2.0e5]
    base = [(997.5, 1102.5), (997.5, 1102.5), (380.0, 420.0)]
    params = [param("osc.sin2_2t13", T["sin2_2t13"]),
              param("osc.dm2_ee", T["dm2_ee"], (2.50, 0.10)),
              param("reactor0.norm", 1.0, (1.0, 0.015)),
              param("reactor1.norm", 1.0, (1.0, 0.015))]
    for d in range(3):
        params.append(param(f"ds{d}.eff", 1.0))
    cov_priors = [dict(params=[f"ds{d}.eff" for d in range(3)], mean=[1.0] * 3,
                       cov=(1e-4 * np.array([[1.0, 0.5, 0.5], [0.5, 1.0, 0.5],
                                             [0.5, 0.5, 1.0]])).tolist())]
    fine = C1_FINE
    cen = fine_centres(fine["y0"], fine["width"], fine["n"])
    edges = C1_EDGES
    nb = len(edges) - 1
    for d in range(3):
        fl = [f"ds{d}.flux[{m}]" for m in range(nb)]
        params += [param(n, 0.0) for n in fl]
        cov_priors.append(dict(params=fl, mean=[0.0] * nb,
                               cov=correlated_cov(nb, cov_seed(d), 0.02)))
    for d in range(3):
        params += [param(f"ds{d}.bkg1.rate", 1.0, (1.0, 0.05)),
                   param(f"ds{d}.bkg2.rate", 1.0)]
    for d in range(3):
        params += [param(f"ds{d}.bkg1.shape[{i}]", 0.0, (0.0, 0.10)) for i in range(nb)]
    params += [param(f"bkg2.shape[{i}]", 0.0, (0.0, 0.10)) for i in range(nb)]
    for d in range(3):
        params += escale_params(f"ds{d}.escale.")
    datasets = []
    trng = rng_for(4100)
    for d in range(3):
        datasets.append(dict(
            name=names[d], fine=dict(fine), edges=edges,
            sources=[dict(baseline_m=base[d][0], norm=["reactor0.norm"]),
                     dict(baseline_m=base[d][1], norm=["reactor1.norm"])],
            norm=[f"ds{d}.eff"],
            flux=dict(params=[f"ds{d}.flux[{m}]" for m in range(nb)],
                      basis=indicator_basis(cen, edges)),
            escale=dict(c0=f"ds{d}.escale.c0", c1=f"ds{d}.escale.c1", c2=f"ds{d}.escale.c2"),
            backgrounds=[
                dict(name="bkg1", rate=f"ds{d}.bkg1.rate", scale=0.03 * rates[d],
                     template=template_seeded(edges, trng),
                     shape=[f"ds{d}.bkg1.shape[{i}]" for i in range(nb)]),
                dict(name="bkg2", rate=f"ds{d}.bkg2.rate", scale=0.02 * rates[d],
                     template=template_seeded(edges, trng),
                     shape=[f"bkg2.shape[{i}]" for i in range(nb)]),
            ]))
    return dict(
        version=1,
        osc=dict(formula="eq1", sin2_2t13=dict(param="osc.sin2_2t13"),
                 dm2_ee=dict(param="osc.dm2_ee"),
                 sin2_t12=dict(value=T["sin2_t12"]), dm2_21=dict(value=T["dm2_21"])),
        params=params, cov_priors=cov_priors, datasets=datasets)


def config2_events(n=1_000_000):
    rates = [4.0e4, 1.0e5, 2.0e5]
    return [make_events(n, 1.8, 10.0, 2, rates[d], event_seed(2, d), "c1",
                        source_fracs=[0.5, 0.5]) for d in range(3)]


def config3_model():
    """Medium baseline (52-53 km, 10 cores), exact three-flavour P, 400 bins, 120 parameters."""
    T = TRUTH
    params = [param("osc.sin2_t12", T["sin2_t12"], (0.307, 0.013)),
              param("osc.sin2_t13", T["sin2_t13"]),
              param("osc.dm2_21", T["dm2_21"], (7.53, 0.18)),
              param("osc.dm2_31", T["dm2_31"])]
    params += [param(f"src{j}.norm", 1.0, (1.0, 0.008)) for j in range(10)]
    params.append(param("norm", 1.0, (1.0, 0.02)))
    params += escale_params("escale.")
    params += [param(f"flux[{m}]", 0.0, (0.0, 0.01)) for m in range(100)]
    params += [param("bkg.flat.rate", 1.0, (1.0, 0.05)), param("bkg.exp.rate", 1.0)]
    fine = C3_FINE
    cen = fine_centres(fine["y0"], fine["width"], fine["n"])
    nodes = list(np.linspace(0.8, 12.0, 100))
    base = list(np.linspace(52.0e3, 53.0e3, 10))
    ds = dict(
        name="FAR", fine=dict(fine), edges=C3_EDGES,
        sources=[dict(baseline_m=float(b), norm=[f"src{j}.norm"]) for j, b in enumerate(base)],
        norm=["norm"],
        flux=dict(params=[f"flux[{m}]" for m in range(100)], basis=hat_basis(cen, nodes)),
        escale=dict(c0="escale.c0", c1="escale.c1", c2="escale.c2"),
        backgrounds=[
            dict(name="flat", rate="bkg.flat.rate", scale=2.0e3,
                 template=template_flat(C3_EDGES), shape=None),
            dict(name="exp", rate="bkg.exp.rate", scale=1.5e3,
                 template=template_exp(C3_EDGES, 2.0), shape=None),
        ])
    return dict(
        version=1,
        osc=dict(formula="3nu", sin2_t12=dict(param="osc.sin2_t12"),
                 sin2_t13=dict(param="osc.sin2_t13"), dm2_21=dict(param="osc.dm2_21"),
                 dm2_31=dict(param="osc.dm2_31")),
        params=params, cov_priors=[], datasets=[ds])


def config3_matter_model(rho_ye=1.3):
    """The medium-baseline model with the exact three-flavour probability in
    matter of constant density (crust: rho about 2.6 g/cm^3, Y_e about 0.5)."""
    m = config3_model()
    m["osc"]["formula"] = "3nu_matter"
    m["osc"]["rho_ye"] = float(rho_ye)
    return m


def config3_events(n=10_000_000):
    return [make_events(n, 1.8, 12.0, 10, 1.0e5, event_seed(3, 0), "c3")]


# Conditional splitting of datasets (paper, "Conditional splitting of
# datasets"): the three Double Chooz histograms FD-I, FD-II and ND split by
# the reactors in operation (both, reactor 1 only, reactor 2 only: a single
# source has a unique baseline) and by the neutron-capture type (Gd, H: other
# binning and other backgrounds), 3 x 3 x 2 = 18 histograms of uneven sizes,
# plus the reactor-off phases of FD-I and FD-II as one-bin rate terms (second
# line of Eq. 9: the Poisson probability of the total reactor-off rate; their
# small residual antineutrino signal is folded like the others).
SPLIT_PHASES = ("FD-I", "FD-II", "ND")
SPLIT_REACTORS = ("both", "R1", "R2")
SPLIT_CAPTURES = ("Gd", "H")
SPLIT_BASE = {"FD-I": (997.5, 1102.5), "FD-II": (997.5, 1102.5), "ND": (380.0, 420.0)}
SPLIT_EDGES = {"Gd": uniform_edges(1.0, 7.65, 38), "H": uniform_edges(1.35, 5.9, 26)}
SPLIT_OFF_EDGES = [1.0, 8.0]


def _split_rate(phase, reactors, capture):
    base = {"FD-I": 4.0e4, "FD-II": 1.0e5, "ND": 2.0e5}[phase]
    frac = {"both": 0.7, "R1": 0.16, "R2": 0.14}[reactors]
    return base * frac * (1.0 if capture == "Gd" else 0.45)


def split_model():
    """18 uneven histograms plus two one-bin reactor-off rate terms."""
    T = TRUTH
    params = [param("osc.sin2_2t13", T["sin2_2t13"]),
              param("osc.dm2_ee", T["dm2_ee"], (2.50, 0.10)),
              param("reactor0.norm", 1.0, (1.0, 0.015)),
              param("reactor1.norm", 1.0, (1.0, 0.015)),
              param("residual.norm", 1.0, (1.0, 0.3))]
    cov_priors = []
    for cap in SPLIT_CAPTURES:
        eff = [f"{ph}.{cap}.eff" for ph in SPLIT_PHASES]
        params += [param(n, 1.0) for n in eff]
        cov_priors.append(dict(params=eff, mean=[1.0] * 3,
                               cov=(1e-4 * np.array([[1.0, 0.5, 0.5], [0.5, 1.0, 0.5],
                                                     [0.5, 0.5, 1.0]])).tolist()))
    fine = C1_FINE
    cen = fine_centres(fine["y0"], fine["width"], fine["n"])
    for cap in SPLIT_CAPTURES:
        nb = len(SPLIT_EDGES[cap]) - 1
        params += [param(f"{cap}.flux[{m}]", 0.0, (0.0, 0.03)) for m in range(6)]
        params += [param(f"{cap}.li9.shape[{i}]", 0.0, (0.0, 0.10)) for i in range(nb)]
        for ph in SPLIT_PHASES:
            params += escale_params(f"{ph}.{cap}.escale.")
    for ph in SPLIT_PHASES:
        params += [param(f"{ph}.li9.rate", 1.0), param(f"{ph}.fn.rate", 1.0, (1.0, 0.1))]
        for r in SPLIT_REACTORS:
            for cap in SPLIT_CAPTURES:
                params.append(param(f"{ph}.{r}.{cap}.acc.rate", 1.0, (1.0, 0.05)))
    trng = rng_for(4200)
    tmpl = {(cap, kind): template_seeded(SPLIT_EDGES[cap], trng)
            for cap in SPLIT_CAPTURES for kind in ("li9", "fn", "acc")}
    datasets = []
    for ph in SPLIT_PHASES:
        for r in SPLIT_REACTORS:
            for cap in SPLIT_CAPTURES:
                edges = SPLIT_EDGES[cap]
                nb = len(edges) - 1
                rate = _split_rate(ph, r, cap)
                b0, b1 = SPLIT_BASE[ph]
                srcs = {"both": [dict(baseline_m=b0, norm=["reactor0.norm"]),
                                 dict(baseline_m=b1, norm=["reactor1.norm"])],
                        "R1": [dict(baseline_m=b0, norm=["reactor0.norm"])],
                        "R2": [dict(baseline_m=b1, norm=["reactor1.norm"])]}[r]
                nodes = list(np.linspace(edges[0], edges[-1], 6))
                bk = 0.05 if cap == "Gd" else 0.25  # H capture: larger accidental background
                datasets.append(dict(
                    name=f"{ph}.{r}.{cap}", fine=dict(fine), edges=edges, sources=srcs,
                    norm=[f"{ph}.{cap}.eff"],
                    flux=dict(params=[f"{cap}.flux[{m}]" for m in range(6)],
                              basis=hat_basis(cen, nodes)),
                    escale=dict(c0=f"{ph}.{cap}.escale.c0", c1=f"{ph}.{cap}.escale.c1",
                                c2=f"{ph}.{cap}.escale.c2"),
                    backgrounds=[
                        dict(name="li9", rate=f"{ph}.li9.rate", scale=0.02 * rate,
                             template=tmpl[(cap, "li9")],
                             shape=[f"{cap}.li9.shape[{i}]" for i in range(nb)]),
                        dict(name="fn", rate=f"{ph}.fn.rate", scale=0.01 * rate,
                             template=tmpl[(cap, "fn")], shape=None),
                        dict(name="acc", rate=f"{ph}.{r}.{cap}.acc.rate", scale=bk * rate,
                             template=tmpl[(cap, "acc")], shape=None),
                    ]))
    for ph in ("FD-I", "FD-II"):
        b0, b1 = SPLIT_BASE[ph]
        datasets.append(dict(
            name=f"{ph}.off", fine=dict(fine), edges=list(SPLIT_OFF_EDGES),
            sources=[dict(baseline_m=b0, norm=["residual.norm"]),
                     dict(baseline_m=b1, norm=["residual.norm"])],
            norm=[], flux=None, escale=dict(c0=None, c1=None, c2=None),
            backgrounds=[
                dict(name="li9", rate=f"{ph}.li9.rate", scale=60.0, template=[1.0], shape=None),
                dict(name="fn", rate=f"{ph}.fn.rate", scale=25.0, template=[1.0], shape=None)]))
    return dict(
        version=1,
        osc=dict(formula="eq1", sin2_2t13=dict(param="osc.sin2_2t13"),
                 dm2_ee=dict(param="osc.dm2_ee"),
                 sin2_t12=dict(value=T["sin2_t12"]), dm2_21=dict(value=T["dm2_21"])),
        params=params, cov_priors=cov_priors, datasets=datasets)


def split_events(scale=1.0):
    """Events of the split workload: 1e5 per reactor-on histogram at scale 1
    (uneven: the single-reactor and H-capture histograms get fewer), 2e4 per
    reactor-off term with a residual rate of 2 events."""
    out = []
    j = 0
    for ph in SPLIT_PHASES:
        for r in SPLIT_REACTORS:
            for cap in SPLIT_CAPTURES:
                ns = 1 if r != "both" else 2
                n = int(scale * 1.0e5 * (1.0 if r == "both" else 0.4) * (1.0 if cap == "Gd" else 0.6))
                out.append(make_events(max(n, 8), 1.8, 10.0, ns, _split_rate(ph, r, cap),
                                       event_seed(6, j), "c1",
                                       source_fracs=None if ns == 1 else [0.5, 0.5]))
                j += 1
    for _ in ("FD-I", "FD-II"):
        out.append(make_events(max(int(scale * 2.0e4), 8), 1.8, 10.0, 2, 2.0, event_seed(6, j), "c1",
                               source_fracs=[0.5, 0.5]))
        j += 1
    return out


# Sterile-neutrino search (paper, "Extensions of the framework"): the
# near/far short-baseline layout with the 3+1 survival probability; the
# tested parameters are sin^2(2 theta14) and dm2_41 (1e-3 eV^2 units), the
# conventional oscillation parameters are nuisances (sin^2 theta13 free,
# dm2_31 with a prior; theta12 and dm2_21 fixed at their world averages).
STERILE_DM2_41 = 50.0  # 0.05 eV^2 start value


def sterile_model():
    """Near (400 m) and far (1050 m) detector, two reactors each, 40 bins each, 3+1."""
    T = TRUTH
    params = [param("osc.sin2_t13", T["sin2_t13"]),
              param("osc.dm2_31", T["dm2_31"], (2.53, 0.05)),
              param("osc.sin2_2t14", 0.0),
              param("osc.dm2_41", STERILE_DM2_41, fixed=True),
              param("reactor0.norm", 1.0, (1.0, 0.015)),
              param("reactor1.norm", 1.0, (1.0, 0.015))]
    params += [param(f"flux[{m}]", 0.0, (0.0, 0.05)) for m in range(4)]
    names, base, rates = ["FD", "ND"], [(997.5, 1102.5), (380.0, 420.0)], [1.0e5, 2.0e5]
    fine = C1_FINE
    cen = fine_centres(fine["y0"], fine["width"], fine["n"])
    datasets = []
    for d, nm in enumerate(names):
        params += [param(f"{nm}.eff", 1.0, (1.0, 0.01)), *escale_params(f"{nm}.escale."),
                   param(f"{nm}.bkg.flat.rate", 1.0, (1.0, 0.10)), param(f"{nm}.bkg.exp.rate", 1.0)]
        datasets.append(dict(
            name=nm, fine=dict(fine), edges=C1_EDGES,
            sources=[dict(baseline_m=base[d][0], norm=["reactor0.norm"]),
                     dict(baseline_m=base[d][1], norm=["reactor1.norm"])],
            norm=[f"{nm}.eff"],
            flux=dict(params=[f"flux[{m}]" for m in range(4)],
                      basis=hat_basis(cen, [1.0, 10.0 / 3.0, 17.0 / 3.0, 8.0])),
            escale=dict(c0=f"{nm}.escale.c0", c1=f"{nm}.escale.c1", c2=f"{nm}.escale.c2"),
            backgrounds=[
                dict(name="flat", rate=f"{nm}.bkg.flat.rate", scale=0.015 * rates[d],
                     template=template_flat(C1_EDGES), shape=None),
                dict(name="exp", rate=f"{nm}.bkg.exp.rate", scale=0.02 * rates[d],
                     template=template_exp(C1_EDGES, 2.0), shape=None)]))
    return dict(
        version=1,
        osc=dict(formula="4nu", sin2_t13=dict(param="osc.sin2_t13"), dm2_31=dict(param="osc.dm2_31"),
                 sin2_2t14=dict(param="osc.sin2_2t14"), dm2_41=dict(param="osc.dm2_41"),
                 sin2_t12=dict(value=T["sin2_t12"]), dm2_21=dict(value=T["dm2_21"])),
        params=params, cov_priors=[], datasets=datasets)


def sterile_events(n=100_000):
    rates = [1.0e5, 2.0e5]
    return [make_events(n, 1.8, 10.0, 2, rates[d], event_seed(7, d), "c1", source_fracs=[0.5, 0.5])
            for d in range(2)]


def model_and_events(config, n_events=None):
    if config == 1:
        return config1_model(), config1_events(*(() if n_events is None else (n_events,)))
    if config == 2:
        return config2_model(), config2_events(*(() if n_events is None else (n_events,)))
    if config == 3:
        return config3_model(), config3_events(*(() if n_events is None else (n_events,)))
    if config == "c3_matter":
        return config3_matter_model(), config3_events(*(() if n_events is None else (n_events,)))
    if config == "sterile":
        return sterile_model(), sterile_events(*(() if n_events is None else (n_events,)))
    if config == "split":
        return split_model(), split_events(*(() if n_events is None else (n_events,)))
    raise ValueError(config)


def start_vector(model):
    return np.array([p["start"] for p in model["params"]], dtype=np.float64)


def param_index(model, name):
    for i, p in enumerate(model["params"]):
        if p["name"] == name:
            return i
    raise KeyError(name)


def osc_theta_list(model, count, seed=77, spread=0.05):
    """`count` parameter vectors around the start point with varied oscillation
    parameters (so cached fold results cannot be reused between them)."""
    rng = rng_for(seed)
    base = start_vector(model)
    osc_names = [v["param"] for k, v in model["osc"].items()
                 if isinstance(v, dict) and "param" in v]
    out = []
    for _ in range(count):
        th = base.copy()
        for n in osc_names:
            i = param_index(model, n)
            th[i] = base[i] * (1.0 + spread * rng.uniform(-1, 1))
        out.append(th)
    return np.array(out)


def poisson_data(mu_list, seed):
    """One Poisson draw per bin around the given expectations (list per dataset)."""
    rng = rng_for(seed)
    return [rng.poisson(np.asarray(mu)).astype(np.float64) for mu in mu_list]


# --------------------------------------------------------------------------
# small random models for parity and edge-case tests
# --------------------------------------------------------------------------

def tiny_model(seed, formula="eq1", n_datasets=2, n_sources=2, fine_n=12, nb=8,
               n_flux=3, shape_params=True, escale=True):
    """Small random model: a few datasets, sources and bins, every feature switched on."""
    rng = rng_for(seed)
    y0, width = 0.5, 0.5
    lo_bin = 2
    edges = [y0 + width * (lo_bin + i * ((fine_n - 2 * lo_bin) // nb)) for i in range(nb + 1)]
    cen = fine_centres(y0, width, fine_n)
    params = []
    if formula == "eq1":
        params += [param("osc.sin2_2t13", 0.085 * (1 + 0.2 * rng.uniform(-1, 1))),
                   param("osc.dm2_ee", 2.5 * (1 + 0.1 * rng.uniform(-1, 1)), (2.5, 0.1))]
        osc = dict(formula="eq1", sin2_2t13=dict(param="osc.sin2_2t13"),
                   dm2_ee=dict(param="osc.dm2_ee"),
                   sin2_t12=dict(value=0.307), dm2_21=dict(value=7.53))
    elif formula == "4nu":
        params += [param("osc.sin2_t13", 0.0218 * (1 + 0.1 * rng.uniform(-1, 1))),
                   param("osc.dm2_31", 2.53, (2.53, 0.05)),
                   param("osc.sin2_2t14", 0.05 * (1 + 0.5 * rng.uniform(-1, 1))),
                   param("osc.dm2_41", float(rng.choice([5.0, 50.0, 500.0])) * (1 + 0.1 * rng.uniform(-1, 1)))]
        osc = dict(formula="4nu", sin2_t13=dict(param="osc.sin2_t13"), dm2_31=dict(param="osc.dm2_31"),
                   sin2_2t14=dict(param="osc.sin2_2t14"), dm2_41=dict(param="osc.dm2_41"),
                   sin2_t12=dict(value=0.307), dm2_21=dict(value=7.53))
    else:
        params += [param("osc.sin2_t12", 0.307, (0.307, 0.013)),
                   param("osc.sin2_t13", 0.0218),
                   param("osc.dm2_21", 7.53, (7.53, 0.18)),
                   param("osc.dm2_31", 2.53 * (1 if rng.uniform() < 0.5 else -1))]
        osc = dict(formula="3nu", sin2_t12=dict(param="osc.sin2_t12"),
                   sin2_t13=dict(param="osc.sin2_t13"), dm2_21=dict(param="osc.dm2_21"),
                   dm2_31=dict(param="osc.dm2_31"))
        if formula == "3nu_matter":
            # a density far above the Earth's, so that matter changes P at
            # these short baselines (A comparable to dm2_31 at a few MeV)
            osc["formula"] = "3nu_matter"
            osc["rho_ye"] = float(rng.uniform(800.0, 2500.0))
    params += [param(f"src{s}.norm", 1.0 + 0.01 * rng.uniform(-1, 1), (1.0, 0.02))
               for s in range(n_sources)]
    cov_priors = []
    datasets = []
    for d in range(n_datasets):
        params.append(param(f"ds{d}.norm", 1.0 + 0.01 * rng.uniform(-1, 1), (1.0, 0.03)))
        fl = [f"ds{d}.flux[{m}]" for m in range(n_flux)]
        params += [param(n, 0.02 * rng.uniform(-1, 1)) for n in fl]
        cov_priors.append(dict(params=fl, mean=[0.0] * n_flux,
                               cov=correlated_cov(n_flux, 4500 + 10 * seed + d, 0.05)))
        if escale:
            params += [param(f"ds{d}.c0", 0.01 * rng.uniform(-1, 1), (0.0, 0.02)),
                       param(f"ds{d}.c1", 0.005 * rng.uniform(-1, 1), (0.0, 0.01)),
                       param(f"ds{d}.c2", 0.001 * rng.uniform(-1, 1), (0.0, 0.002))]
        params.append(param(f"ds{d}.bkg.rate", 1.0 + 0.05 * rng.uniform(-1, 1), (1.0, 0.1)))
        shape = None
        if shape_params:
            shape = [f"ds{d}.bkg.shape[{i}]" for i in range(nb)]
            params += [param(n, 0.05 * rng.uniform(-1, 1), (0.0, 0.1)) for n in shape]
        nodes = list(np.linspace(edges[0], edges[-1], n_flux))
        datasets.append(dict(
            name=f"ds{d}", fine=dict(y0=y0, width=width, n=fine_n), edges=edges,
            sources=[dict(baseline_m=float(rng.uniform(300, 1200)), norm=[f"src{s}.norm"])
                     for s in range(n_sources)],
            norm=[f"ds{d}.norm"],
            flux=dict(params=fl, basis=hat_basis(cen, nodes)),
            escale=(dict(c0=f"ds{d}.c0", c1=f"ds{d}.c1", c2=f"ds{d}.c2") if escale
                    else dict(c0=None, c1=None, c2=None)),
            backgrounds=[dict(name="bkg", rate=f"ds{d}.bkg.rate",
                              scale=float(rng.uniform(10, 100)),
                              template=template_seeded(edges, rng), shape=shape)]))
    return dict(version=1, osc=osc, params=params, cov_priors=cov_priors, datasets=datasets)


def tiny_events(model, n_per_dataset, seed):
    out = []
    for d, ds in enumerate(model["datasets"]):
        f = ds["fine"]
        rng = rng_for(seed + d)
        lo, hi = f["y0"] - 0.2, f["y0"] + f["width"] * f["n"] + 0.2
        e_reco = rng.uniform(lo, hi, n_per_dataset)
        e_true = np.clip(e_reco + 0.78 + rng.normal(0, 0.1, n_per_dataset), 0.5, None)
        src = rng.integers(0, len(ds["sources"]), n_per_dataset).astype(np.uint8)
        w = rng.uniform(0.5, 2.0, n_per_dataset).astype(np.float32)
        out.append(dict(e_true=e_true, e_reco=e_reco, source=src, weight=w))
    return out


def to_json(model) -> str:
    return json.dumps(model)
