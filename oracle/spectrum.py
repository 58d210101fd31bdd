"""Signal rescale, energy-scale re-binning and backgrounds (oracle; test infrastructure).

Step 2 (paper, "Structure of the framework"; flux parameters in the Double
Chooz likelihood section): the oscillated fine spectrum of each source is
scaled by its rate normalisation and by the bin-to-bin flux-shape factor,
  H_k = sum_s A_s S[s][k] (1 + F_k),  A_s = prod of its norm parameters,
  F_k = sum_m f_m phi_m(k).
Step 3: the fine spectrum defines an area-conserving piecewise-quadratic
density, the detector response maps MC energy E to data energy
f(E) = c0 + (1 + c1) E + c2 E^2 (second-order polynomial), and the density is
integrated over the pre-images of the analysis bins:
  s_i = C(g(x_{i+1})) - C(g(x_i)),  g = f^-1,  C = cumulative of the density.
Backgrounds (data-driven templates, no energy correction):
  B_i = sum_b scale_b R_b T_{b,i} (1 + beta_{b,i}).

Readings of points the paper leaves open:
  * density in fine bin k, t = (y - y_k)/width in [0, 1]:
      rho(t) = d_k (1-t) + d_{k+1} t + 6 (m_k - (d_k + d_{k+1})/2) t (1-t),  m_k = H_k / width,
    edge densities d_k = 2 m_{k-1} m_k / (m_{k-1} + m_k) if m_{k-1} m_k > 0 else 0
    (harmonic mean), d_0 = m_0, d_K = m_{K-1}. Quadratic, integrates to H_k.
  * C(y) = 0 below y_0 and C_K = sum H above y_K.
  * inverse map in the cancellation-free form
      g(x) = 2 (x - c0) / (b + sqrt(b^2 + 4 c2 (x - c0))),  b = 1 + c1;
    where the discriminant is negative, x lies beyond the range of f:
    g = +inf for c2 < 0, -inf for c2 > 0.
  * the map is valid when b > 0 and f'(E) = b + 2 c2 E > 0 at y_0 and y_K;
    otherwise the evaluation is flagged out of domain.
Complex-valued inputs are supported (comparisons act on real parts).
"""
import numpy as np


def _val(theta, i, default):
    return default if i is None else theta[i]


def source_norms(ds, theta):
    """A_s = product of the dataset-level and source-level norm parameters."""
    out = []
    for s in range(ds.S):
        a = 1.0
        for i in ds.norm + ds.src_norm[s]:
            a = a * theta[i]
        out.append(a)
    return out


def flux_factor(ds, theta):
    F = np.zeros(ds.K, dtype=np.result_type(theta, np.float64))
    for m, i in enumerate(ds.flux_idx):
        F = F + theta[i] * ds.flux_basis[m]
    return F


def rescale(ds, S, theta):
    A = source_norms(ds, theta)
    F = flux_factor(ds, theta)
    H = 0.0
    for s in range(ds.S):
        H = H + A[s] * S[s]
    return H * (1.0 + F)


def energy_coeffs(ds, theta):
    return [_val(theta, i, 0.0) for i in ds.escale]


def energy_map_valid(ds, c):
    c0, c1, c2 = (np.real(v) for v in c)
    b = 1.0 + c1
    yk = ds.y0 + ds.wf * ds.K
    return bool(b > 0 and b + 2 * c2 * ds.y0 > 0 and b + 2 * c2 * yk > 0)


def energy_map_inverse(x, c):
    """g(x) = f^-1(x) for f(E) = c0 + (1+c1) E + c2 E^2 (increasing branch)."""
    c0, c1, c2 = c
    b = 1.0 + c1
    z = x - c0
    disc = b * b + 4.0 * c2 * z
    if np.real(disc) < 0:
        return np.inf if np.real(c2) < 0 else -np.inf
    return 2.0 * z / (b + np.sqrt(disc))


def edge_densities(H, wf):
    """Mean densities m_k of the fine bins and the edge densities d_k."""
    m = H / wf
    K = len(H)
    d = np.zeros(K + 1, dtype=m.dtype)
    d[0] = m[0]
    d[K] = m[K - 1]
    a, b = m[:-1], m[1:]
    pos = np.real(a * b) > 0
    den = np.where(pos, a + b, 1.0)
    d[1:K] = np.where(pos, 2.0 * a * b / den, 0.0)
    return m, d


def spline_parts(H, wf):
    m, d = edge_densities(H, wf)
    Ck = np.concatenate([[0.0 * H[0]], np.cumsum(H)])
    return m, d, Ck


def _locate(parts, wf, y0, y):
    K = len(parts[0])
    k = min(int(np.floor((np.real(y) - y0) / wf)), K - 1)
    return k, (y - (y0 + k * wf)) / wf


def density(H, wf, y0, y, parts=None):
    """rho at energy y (0 outside the fine range)."""
    m, d, _ = parts if parts is not None else spline_parts(H, wf)
    K = len(m)
    if np.real(y) < y0 or np.real(y) >= y0 + wf * K:
        return 0.0 * m[0]
    k, t = _locate((m, d), wf, y0, y)
    return d[k] * (1 - t) + d[k + 1] * t + 6.0 * (m[k] - 0.5 * (d[k] + d[k + 1])) * t * (1 - t)


def cumulative(H, wf, y0, y, parts=None):
    """C(y) = integral of rho from y_0 to y."""
    m, d, Ck = parts if parts is not None else spline_parts(H, wf)
    K = len(m)
    if np.real(y) < y0:
        return Ck[0]
    if np.real(y) >= y0 + wf * K:
        return Ck[K]
    k, t = _locate((m, d), wf, y0, y)
    integral = (d[k] * (t - 0.5 * t * t) + d[k + 1] * 0.5 * t * t
                + 6.0 * (m[k] - 0.5 * (d[k] + d[k + 1])) * (0.5 * t * t - t * t * t / 3.0))
    return Ck[k] + wf * integral


def rebin(ds, H, c):
    """Analysis-bin signal s_i = C(g(x_{i+1})) - C(g(x_i))."""
    parts = spline_parts(H, ds.wf)
    Cx = [cumulative(H, ds.wf, ds.y0, energy_map_inverse(x, c), parts) for x in ds.edges]
    return np.array([Cx[i + 1] - Cx[i] for i in range(ds.Nb)])


def backgrounds(ds, theta):
    B = np.zeros(ds.Nb, dtype=np.result_type(theta, np.float64))
    for b in ds.bkgs:
        r = _val(theta, b["rate"], 1.0)
        if b["shape"] is None:
            shape = 1.0
        else:
            shape = np.array([1.0 + _val(theta, i, 0.0) for i in b["shape"]])
        B = B + b["scale"] * r * b["template"] * shape
    return B
