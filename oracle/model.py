"""Model description parsing (oracle; test infrastructure).

The model description is a plain dict (JSON-compatible):
  params      list of {name, start, prior: [mean, sigma] | None, fixed}
  cov_priors  list of {params: [names], mean: [...], cov: [[...]]}   (Eq. 6, Eq. 9 third line)
  osc         {formula: "eq1" | "3nu" | "4nu" | "3nu_matter", <slot>: {param: name} | {value: v}}
              eq1 slots: sin2_2t13, dm2_ee, sin2_t12, dm2_21   (Eq. 1)
              3nu slots: sin2_t12, sin2_t13, dm2_21, dm2_31    (exact vacuum form of Eq. 10)
              3nu_matter: the 3nu slots plus rho_ye (number, g/cm^3 x electrons per
                  nucleon): exact three flavours in matter of constant density
              4nu slots: sin2_t13, dm2_31, sin2_2t14, dm2_41   (vacuum 3+1, sterile searches)
                  plus fixed values sin2_t12, dm2_21: {value: v}
  datasets    list of {name, fine: {y0, width, n}, edges, sources: [{baseline_m, norm}],
              norm, flux: {params, basis (M x K)}, escale: {c0, c1, c2},
              backgrounds: [{rate, scale, template, shape}]}
Parameter namespaces (paper, "Structure of the framework") are dotted names.
"""
import numpy as np

EQ1_SLOTS = ("sin2_2t13", "dm2_ee", "sin2_t12", "dm2_21")
NU3_SLOTS = ("sin2_t12", "sin2_t13", "dm2_21", "dm2_31")
# 3+1: four slots that may be parameters, and the solar pair, which is fixed
NU4_SLOTS = ("sin2_t13", "dm2_31", "sin2_2t14", "dm2_41")
NU4_CONSTANTS = ("sin2_t12", "dm2_21")


class Dataset:
    def __init__(self, d, index):
        def idx(name):
            return None if name is None else index[name]

        self.name = d.get("name", "")
        f = d["fine"]
        self.y0 = float(f["y0"])
        self.wf = float(f["width"])
        self.K = int(f["n"])
        self.edges = np.asarray(d["edges"], dtype=np.float64)
        self.Nb = len(self.edges) - 1
        self.baselines = np.array([s["baseline_m"] for s in d["sources"]], dtype=np.float64)
        self.S = len(self.baselines)
        self.src_norm = [[index[n] for n in s.get("norm", [])] for s in d["sources"]]
        self.norm = [index[n] for n in d.get("norm", [])]
        fl = d.get("flux") or {"params": [], "basis": []}
        self.flux_idx = [index[n] for n in fl["params"]]
        self.flux_basis = (np.asarray(fl["basis"], dtype=np.float64).reshape(len(self.flux_idx), self.K)
                           if self.flux_idx else np.zeros((0, self.K)))
        es = d.get("escale") or {}
        self.escale = [idx(es.get(c)) for c in ("c0", "c1", "c2")]
        self.bkgs = []
        for b in d.get("backgrounds", []):
            shape = b.get("shape")
            self.bkgs.append(dict(
                rate=idx(b.get("rate")), scale=float(b["scale"]),
                template=np.asarray(b["template"], dtype=np.float64),
                shape=None if shape is None else [idx(n) for n in shape]))


class Model:
    def __init__(self, desc):
        self.desc = desc
        self.names = [p["name"] for p in desc["params"]]
        self.index = {n: i for i, n in enumerate(self.names)}
        if len(self.index) != len(self.names):
            raise ValueError("duplicate parameter names")
        self.P = len(self.names)
        self.start = np.array([p["start"] for p in desc["params"]], dtype=np.float64)
        self.fixed = np.array([bool(p.get("fixed", False)) for p in desc["params"]])
        self.gauss = [(i, p["prior"][0], p["prior"][1]) for i, p in enumerate(desc["params"])
                      if p.get("prior") is not None]
        self.blocks = []
        for c in desc.get("cov_priors", []):
            self.blocks.append(([self.index[n] for n in c["params"]],
                                np.asarray(c["mean"], dtype=np.float64),
                                np.asarray(c["cov"], dtype=np.float64)))
        osc = desc["osc"]
        self.formula = osc["formula"]
        if self.formula not in ("eq1", "3nu", "4nu", "3nu_matter"):
            raise ValueError(self.formula)
        slots = {"eq1": EQ1_SLOTS, "3nu": NU3_SLOTS, "4nu": NU4_SLOTS, "3nu_matter": NU3_SLOTS}[self.formula]
        self.rho_ye = float(osc["rho_ye"]) if self.formula == "3nu_matter" else 0.0
        self.osc_constants = ([float(osc[c]["value"]) for c in NU4_CONSTANTS]
                              if self.formula == "4nu" else [])
        self.osc_slots = []
        for s in slots:
            v = osc[s]
            if "param" in v:
                self.osc_slots.append((self.index[v["param"]], None))
            else:
                self.osc_slots.append((None, float(v["value"])))
        self.osc_params = {i for i, _ in self.osc_slots if i is not None}
        self.datasets = [Dataset(d, self.index) for d in desc["datasets"]]

    def osc_values(self, theta):
        return [theta[i] if i is not None else v for i, v in self.osc_slots]
