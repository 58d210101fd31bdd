"""ctypes binding of libnufold (the C-ABI declared in include/nufold.h).

Argument marshalling only: every step of an evaluation runs in the library's
HIP kernels. Functions keep the C names; `Engine` is a thin convenience
wrapper. There is no fallback: if the shared library is missing the import of
any entry point raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

NF_OK, NF_WDOMAIN, NF_WNOCONV = 0, 1, 2
NF_EINVAL, NF_ESTATE, NF_ENOMEM, NF_EDEVICE, NF_EPARSE = -1, -2, -3, -4, -5
NF_M64, NF_M32 = 0, 1
NF_MAX_GRAPH_EVALS = 4096

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnufold.so")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u8p = C.POINTER(C.c_uint8)
_i32p = C.POINTER(C.c_int32)

# name: (restype, argtypes)
SIGNATURES = {
    "nf_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_char_p, C.c_int, C.c_void_p]),
    "nf_destroy": (None, [C.c_void_p]),
    "nf_last_error": (C.c_char_p, [C.c_void_p]),
    "nf_num_params": (C.c_int, [C.c_void_p]),
    "nf_num_datasets": (C.c_int, [C.c_void_p]),
    "nf_num_bins": (C.c_int, [C.c_void_p, C.c_int]),
    "nf_param_index": (C.c_int, [C.c_void_p, C.c_char_p]),
    "nf_set_events": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int]),
    "nf_dropped_events": (C.c_int64, [C.c_void_p, C.c_int]),
    "nf_set_data": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int]),
    "nf_eval_nll": (C.c_int, [C.c_void_p, _dp, _dp]),
    "nf_eval_nll_grad": (C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    "nf_eval_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "nf_eval_device_many": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "nf_eval_device_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "nf_expected": (C.c_int, [C.c_void_p, _dp, _dp]),
    "nf_set_option": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int64]),
    "nf_get_option": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int64)]),
    "nf_timing": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), _dp, _dp]),
}

NF_SURROGATE = 1


class FitOpts(C.Structure):
    _fields_ = [("edm_tol", C.c_double), ("max_iter", C.c_int), ("want_cov", C.c_int),
                ("warm_start", C.c_int), ("pad_", C.c_int)]


class FitResult(C.Structure):
    _fields_ = [("nll", C.c_double), ("edm", C.c_double), ("status", C.c_int), ("iters", C.c_int),
                ("evals", C.c_int), ("pad_", C.c_int), ("theta", C.c_void_p), ("cov", C.c_void_p)]


SIGNATURES["nf_fit"] = (C.c_int, [C.c_void_p, _dp, C.c_void_p, C.POINTER(FitOpts), C.POINTER(FitResult)])
SIGNATURES["nf_set_data_batch"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int])
SIGNATURES["nf_eval_batch"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
SIGNATURES["nf_fit_batch"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(FitOpts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p])

class BatchMember(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("B", C.c_int), ("pad_", C.c_int), ("start", C.c_void_p),
                ("fixed", C.c_void_p), ("data_idx", C.c_void_p), ("theta_out", C.c_void_p),
                ("nll_out", C.c_void_p), ("edm_out", C.c_void_p), ("status_out", C.c_void_p),
                ("iters_out", C.c_void_p), ("evals_out", C.c_void_p)]


SIGNATURES["nf_fit_batch_group"] = (C.c_int, [C.c_int, C.POINTER(BatchMember), C.POINTER(FitOpts)])
SIGNATURES["nf_set_surrogate"] = (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                            C.c_int, C.c_float])
SIGNATURES["nf_timing_overhead"] = (C.c_int, [C.c_void_p, C.c_int, _dp])
SIGNATURES["nf_autotune"] = (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p])
SIGNATURES["nf_expected_batch"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
SIGNATURES["nf_mlp_create"] = (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p])
SIGNATURES["nf_mlp_destroy"] = (None, [C.c_void_p])
SIGNATURES["nf_mlp_last_error"] = (C.c_char_p, [C.c_void_p])
SIGNATURES["nf_mlp_num_params"] = (C.c_int64, [C.c_void_p])
SIGNATURES["nf_mlp_set_params"] = (C.c_int, [C.c_void_p, C.c_void_p])
SIGNATURES["nf_mlp_get_params"] = (C.c_int, [C.c_void_p, C.c_void_p])
SIGNATURES["nf_mlp_forward"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int])
SIGNATURES["nf_mlp_grad"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int])
SIGNATURES["nf_mlp_train_step"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_float,
                                             C.POINTER(C.c_float), C.c_int])
SIGNATURES["nf_mlp_use_graphs"] = (C.c_int, [C.c_void_p, C.c_int])
SIGNATURES["nf_mlp_fit_inputs"] = (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.c_void_p])

_lib = None


def load():
    """Load libnufold.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime with the same SONAME as ROCm's
        # (libamdhip64.so.7). Loading torch first makes the engine bind to that
        # already-loaded runtime, so torch streams and device pointers are valid
        # in the engine; without torch the system ROCm runtime is used.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libnufold.so not built ({LIB_PATH}); run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class NufoldError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nufold error {code}: {msg}")
        self.code = code


def _err(ctx):
    m = load().nf_last_error(ctx)
    return m.decode() if m else ""


def _check(ctx, code, allow_warn=True):
    if code < 0 or (code > 0 and not allow_warn):
        raise NufoldError(code, _err(ctx))
    return code


def _ptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _is_cuda(t):
    return hasattr(t, "is_cuda") and t.is_cuda


class Engine:
    """One nf_ctx: model description, events, data; evaluations on the device."""

    def __init__(self, model, mode="m64", stream=None):
        text = model if isinstance(model, str) else json.dumps(model)
        self.mode = NF_M64 if mode in ("m64", NF_M64) else NF_M32
        h = C.c_void_p()
        code = load().nf_create(C.byref(h), text.encode(), self.mode,
                                C.c_void_p(stream) if stream else None)
        if code != NF_OK:
            raise NufoldError(code, _err(None))
        self.ctx = h
        self.P = load().nf_num_params(h)
        self.D = load().nf_num_datasets(h)
        self.nbins = [load().nf_num_bins(h, d) for d in range(self.D)]

    def close(self):
        if getattr(self, "ctx", None):
            load().nf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return _err(self.ctx)

    def param_index(self, name):
        return load().nf_param_index(self.ctx, name.encode())

    def set_option(self, key, value):
        _check(self.ctx, load().nf_set_option(self.ctx, key.encode(), int(value)))

    def get_option(self, key):
        v = C.c_int64()
        _check(self.ctx, load().nf_get_option(self.ctx, key.encode(), C.byref(v)))
        return int(v.value)

    def set_events(self, d, e_true, e_reco, source=None, weight=None):
        if _is_cuda(e_true):
            n = int(e_true.numel())
            ptrs = [t.data_ptr() if t is not None else None for t in (e_true, e_reco, source, weight)]
            return _check(self.ctx, load().nf_set_events(self.ctx, d, n, *ptrs, 1))
        et, pe = _ptr(e_true, np.float64)
        er, pr = _ptr(e_reco, np.float64)
        ps = pw = None
        if source is not None:
            src, ps = _ptr(source, np.uint8)
        if weight is not None:
            wt, pw = _ptr(weight, np.float32)
        return _check(self.ctx, load().nf_set_events(self.ctx, d, len(et), pe, pr, ps, pw, 0))

    def dropped(self, d):
        return load().nf_dropped_events(self.ctx, d)

    def set_data(self, d, counts):
        if _is_cuda(counts):
            return _check(self.ctx, load().nf_set_data(self.ctx, d, int(counts.numel()),
                                                       counts.data_ptr(), 1))
        c, p = _ptr(counts, np.float64)
        return _check(self.ctx, load().nf_set_data(self.ctx, d, len(c), p, 0))

    def eval_nll(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = C.c_double()
        code = _check(self.ctx, load().nf_eval_nll(self.ctx, th.ctypes.data_as(_dp), C.byref(out)))
        return out.value, code

    def eval_nll_grad(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        g = np.zeros(self.P)
        out = C.c_double()
        code = _check(self.ctx, load().nf_eval_nll_grad(self.ctx, th.ctypes.data_as(_dp), C.byref(out),
                                                        g.ctypes.data_as(_dp)))
        return out.value, g, code

    def expected(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        mu = np.zeros(sum(self.nbins))
        code = _check(self.ctx, load().nf_expected(self.ctx, th.ctypes.data_as(_dp), mu.ctypes.data_as(_dp)))
        out, o = [], 0
        for nb in self.nbins:
            out.append(mu[o:o + nb].copy())
            o += nb
        return out, code

    def eval_device(self, theta_ptr, out_ptr, status_ptr=None, want_grad=True):
        """Enqueue an evaluation on device pointers (ints); returns immediately."""
        return _check(self.ctx, load().nf_eval_device(self.ctx, C.c_void_p(theta_ptr), C.c_void_p(out_ptr),
                                                      C.c_void_p(status_ptr) if status_ptr else None,
                                                      1 if want_grad else 0))

    def eval_device_noalloc(self, theta_ptr, out_ptr, status_ptr=None, want_grad=True):
        """As eval_device, with the evaluation's scratch in the library's static
        per-GPU array (no device allocation); returns immediately."""
        return _check(self.ctx, load().nf_eval_device_noalloc(self.ctx, C.c_void_p(theta_ptr),
                                                              C.c_void_p(out_ptr),
                                                              C.c_void_p(status_ptr) if status_ptr else None,
                                                              1 if want_grad else 0))

    def eval_device_many(self, n, theta_ptr, out_ptr, status_ptr=None, want_grad=True):
        """Enqueue n evaluations (theta rows of P doubles, out rows of 1 + P)
        as one HIP graph launch; replays the cached graph when n, the
        pointers and want_grad repeat. Returns immediately."""
        return _check(self.ctx, load().nf_eval_device_many(self.ctx, int(n), C.c_void_p(theta_ptr),
                                                           C.c_void_p(out_ptr),
                                                           C.c_void_p(status_ptr) if status_ptr else None,
                                                           1 if want_grad else 0))

    def fit(self, start, fixed=None, edm_tol=1e-7, max_iter=1000, want_cov=False, warm_start=False):
        """Device L-BFGS fit from `start`; returns a dict (theta, nll, edm, status, iters,
        evals, cov, code)."""
        st = np.ascontiguousarray(start, dtype=np.float64)
        th = np.zeros(self.P)
        cov = np.zeros((self.P, self.P)) if want_cov else None
        fx = None
        if fixed is not None:
            fx = np.ascontiguousarray(np.asarray(fixed, dtype=bool).astype(np.uint8))
        opts = FitOpts(edm_tol, max_iter, 1 if want_cov else 0, NF_SURROGATE if warm_start else 0, 0)
        res = FitResult()
        res.theta = th.ctypes.data
        res.cov = cov.ctypes.data if cov is not None else None
        code = _check(self.ctx, load().nf_fit(self.ctx, st.ctypes.data_as(_dp),
                                              fx.ctypes.data if fx is not None else None,
                                              C.byref(opts), C.byref(res)))
        return dict(theta=th, nll=res.nll, edm=res.edm, status=res.status, iters=res.iters,
                    evals=res.evals, cov=cov, code=code)

    def set_data_batch(self, counts):
        """counts: nsets x (sum of analysis bins) observed counts."""
        c = np.ascontiguousarray(counts, dtype=np.float64)
        if c.ndim != 2 or c.shape[1] != sum(self.nbins):
            raise ValueError("counts must be nsets x total bins")
        return _check(self.ctx, load().nf_set_data_batch(self.ctx, c.shape[0], c.ctypes.data, 0))

    def eval_batch(self, theta, data_idx=None, want_grad=True):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        B = th.shape[0]
        nll = np.zeros(B)
        g = np.zeros((B, self.P)) if want_grad else None
        di = None if data_idx is None else np.ascontiguousarray(data_idx, dtype=np.int32)
        code = _check(self.ctx, load().nf_eval_batch(self.ctx, B, th.ctypes.data,
                                                     di.ctypes.data if di is not None else None,
                                                     nll.ctypes.data, g.ctypes.data if g is not None else None))
        return nll, g, code

    def fit_batch(self, start, fixed=None, data_idx=None, edm_tol=1e-7, max_iter=1000, warm_start=False):
        st = np.ascontiguousarray(start, dtype=np.float64)
        B = st.shape[0]
        th = np.zeros((B, self.P))
        nll, edm = np.zeros(B), np.zeros(B)
        status, iters, evals = (np.zeros(B, dtype=np.int32) for _ in range(3))
        fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=bool).astype(np.uint8))
        di = None if data_idx is None else np.ascontiguousarray(data_idx, dtype=np.int32)
        opts = FitOpts(edm_tol, max_iter, 0, NF_SURROGATE if warm_start else 0, 0)
        code = _check(self.ctx, load().nf_fit_batch(
            self.ctx, B, st.ctypes.data, fx.ctypes.data if fx is not None else None,
            di.ctypes.data if di is not None else None, C.byref(opts), th.ctypes.data, nll.ctypes.data,
            edm.ctypes.data, status.ctypes.data, iters.ctypes.data, evals.ctypes.data))
        return dict(theta=th, nll=nll, edm=edm, status=status, iters=iters, evals=evals, code=code)

    def set_surrogate(self, net, param_index, center, half, out_mean, out_std, x_prior, x_weight, starts,
                      iters=200, lr=0.02):
        """Attach a surrogate network (Mlp) for warm starts (nf_set_surrogate);
        net=None detaches."""
        if net is None:
            return _check(self.ctx, load().nf_set_surrogate(self.ctx, None, 0, None, None, None, None, None, None,
                                                            None, 0, None, 0, 0.0))
        self._sur = [np.ascontiguousarray(param_index, np.int32), np.ascontiguousarray(center, np.float64),
                     np.ascontiguousarray(half, np.float64), np.ascontiguousarray(out_mean, np.float32),
                     np.ascontiguousarray(out_std, np.float32), np.ascontiguousarray(x_prior, np.float32),
                     np.ascontiguousarray(x_weight, np.float32), np.ascontiguousarray(starts, np.float32), net]
        a = self._sur
        return _check(self.ctx, load().nf_set_surrogate(self.ctx, net.h, len(a[0]), *[x.ctypes.data for x in a[:7]],
                                                        a[7].shape[0], a[7].ctypes.data, int(iters), float(lr)))

    def timing_overhead(self, n=200):
        """Mean gap (us) between two back-to-back timing events on the stream."""
        us = C.c_double()
        _check(self.ctx, load().nf_timing_overhead(self.ctx, n, C.byref(us)))
        return us.value

    def autotune(self, theta, evals=50, batch=0):
        """Run the library's autotuner; returns ({option: value}, (us/eval, us/batched eval))."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        best = np.zeros(5, dtype=np.int64)
        us = np.zeros(2)
        _check(self.ctx, load().nf_autotune(self.ctx, th.ctypes.data, evals, batch, best.ctypes.data,
                                            us.ctypes.data))
        keys = ("chunk", "fold_block", "tail_threads", "batch_threads", "batch_fit_tile")
        return {k: int(v) for k, v in zip(keys, best)}, (float(us[0]), float(us[1]))

    def expected_batch(self, theta):
        """Expected counts for B parameter vectors: B x (all analysis bins)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        mu = np.zeros((th.shape[0], sum(self.nbins)))
        code = _check(self.ctx, load().nf_expected_batch(self.ctx, th.shape[0], th.ctypes.data, mu.ctypes.data))
        return mu, code

    def timing(self, reset=True):
        """(evaluations, summed fold ms, summed bin-stage ms) since the last reset."""
        n, f, t = C.c_int64(), C.c_double(), C.c_double()
        _check(self.ctx, load().nf_timing(self.ctx, 1 if reset else 0, C.byref(n), C.byref(f), C.byref(t)))
        return n.value, f.value, t.value


def fit_batch_group(members, edm_tol=1e-7, max_iter=1000, warm_start=False):
    """Batched fits of several engines advanced together (nf_fit_batch_group).
    members: list of (engine, start B x P, fixed or None, data_idx or None).
    Returns one result dict per member (as Engine.fit_batch) and the code."""
    keep, arr, outs = [], (BatchMember * len(members))(), []
    for k, (eng, start, fixed, didx) in enumerate(members):
        st = np.ascontiguousarray(start, dtype=np.float64)
        B = st.shape[0]
        fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=bool).astype(np.uint8))
        di = None if didx is None else np.ascontiguousarray(didx, dtype=np.int32)
        o = dict(theta=np.zeros((B, eng.P)), nll=np.zeros(B), edm=np.zeros(B),
                 status=np.zeros(B, np.int32), iters=np.zeros(B, np.int32), evals=np.zeros(B, np.int32))
        keep += [st, fx, di]
        m = arr[k]
        m.ctx, m.B = eng.ctx, B
        m.start = st.ctypes.data
        m.fixed = fx.ctypes.data if fx is not None else None
        m.data_idx = di.ctypes.data if di is not None else None
        m.theta_out, m.nll_out, m.edm_out = o["theta"].ctypes.data, o["nll"].ctypes.data, o["edm"].ctypes.data
        m.status_out, m.iters_out, m.evals_out = (o["status"].ctypes.data, o["iters"].ctypes.data,
                                                  o["evals"].ctypes.data)
        outs.append(o)
    opts = FitOpts(edm_tol, max_iter, 0, NF_SURROGATE if warm_start else 0, 0)
    code = load().nf_fit_batch_group(len(members), arr, C.byref(opts))
    if code < 0:
        msgs = [m for m in (_err(e.ctx) for e, *_ in members) if m]
        raise NufoldError(code, "; ".join(msgs))
    for o in outs:
        o["code"] = code
    return outs, code


def _mlp_err(h):
    m = load().nf_mlp_last_error(h)
    return m.decode() if m else ""


class Mlp:
    """One nf_mlp: dense GELU network on the matrix cores (BF16 in, FP32 out)."""

    def __init__(self, n_in, width, depth, n_out, max_batch, stream=None):
        h = C.c_void_p()
        code = load().nf_mlp_create(C.byref(h), n_in, width, depth, n_out, max_batch,
                                    C.c_void_p(stream) if stream else None)
        if code != NF_OK:
            raise NufoldError(code, _mlp_err(None))
        self.h = h
        self.n_in, self.width, self.depth, self.n_out, self.max_batch = n_in, width, depth, n_out, max_batch
        self.nparam = load().nf_mlp_num_params(h)

    def close(self):
        if getattr(self, "h", None):
            load().nf_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code < 0:
            raise NufoldError(code, _mlp_err(self.h))
        return code

    def layer_shapes(self):
        dims = [self.n_in] + [self.width] * self.depth + [self.n_out]
        return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.nparam
        self._check(load().nf_mlp_set_params(self.h, a.ctypes.data))

    def get_params(self):
        a = np.zeros(self.nparam, dtype=np.float32)
        self._check(load().nf_mlp_get_params(self.h, a.ctypes.data))
        return a

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], self.n_out), dtype=np.float32)
        self._check(load().nf_mlp_forward(self.h, x.shape[0], x.ctypes.data, y.ctypes.data, 0))
        return y

    def grad(self, x, dy, want_dx=True):
        x = np.ascontiguousarray(x, dtype=np.float32)
        dy = np.ascontiguousarray(dy, dtype=np.float32)
        g = np.zeros(self.nparam, dtype=np.float32)
        dx = np.zeros_like(x) if want_dx else None
        self._check(load().nf_mlp_grad(self.h, x.shape[0], x.ctypes.data, dy.ctypes.data, g.ctypes.data,
                                       dx.ctypes.data if want_dx else None, 0))
        return g, dx

    def use_graphs(self, on=True):
        """Training steps as replays of a captured graph (default) or as launches."""
        self._check(load().nf_mlp_use_graphs(self.h, 1 if on else 0))

    def train_step(self, x, t, lr, want_loss=True):
        """Host arrays, or device tensors (torch, float32, contiguous). Without
        want_loss a device-tensor step is enqueued and returns at once (None)."""
        loss = C.c_float()
        lp = C.byref(loss) if want_loss else None
        if _is_cuda(x):
            self._check(load().nf_mlp_train_step(self.h, x.shape[0], C.c_void_p(x.data_ptr()),
                                                 C.c_void_p(t.data_ptr()), lr, lp, 1))
        else:
            x = np.ascontiguousarray(x, dtype=np.float32)
            t = np.ascontiguousarray(t, dtype=np.float32)
            self._check(load().nf_mlp_train_step(self.h, x.shape[0], x.ctypes.data, t.ctypes.data, lr, lp, 0))
        return loss.value if want_loss else None

    def fit_inputs(self, x, nobs, out_mean, out_std, x_prior, x_weight, iters, lr):
        x = np.array(x, dtype=np.float32, order="C")
        args = [np.ascontiguousarray(a, dtype=np.float32) for a in (nobs, out_mean, out_std, x_prior, x_weight)]
        nll = np.zeros(x.shape[0], dtype=np.float32)
        self._check(load().nf_mlp_fit_inputs(self.h, x.shape[0], x.ctypes.data, *[a.ctypes.data for a in args],
                                             iters, lr, nll.ctypes.data))
        return x, nll
