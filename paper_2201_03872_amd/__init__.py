"""Python binding of libddamg, the gfx950 multi-rhs x multi-shift twisted-mass
DD-alpha-AMG library (C ABI in include/ddamg.h).

This module only marshals arguments: every step of the computation runs in
the library's HIP kernels.  Vectors are torch complex128 tensors on the GPU
(canonical layouts of the C ABI); PyTorch provides device memory and the
stream, nothing else.  If the compiled library is missing the import of the
native code fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libddamg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ddamg.h")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EDEVICE, EBREAKDOWN, ESTATE = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, FP16 = 0, 1, 2   # FP16: apply_sap only (FP16-stored right-hand sides)
PLAIN_FP64, MIXED = 0, 1
SMOOTHER_SAP, SMOOTHER_LEARNED = 0, 1


class DDAMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ddamg error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int * 4),
        ("kappa", ctypes.c_double),
        ("n_levels", ctypes.c_int),
        ("agg", (ctypes.c_int * 4) * 2),
        ("n_tv", ctypes.c_int * 2),
        ("sap_block", ctypes.c_int * 4),
        ("sap_cycles", ctypes.c_int),
        ("sap_mr_iters", ctypes.c_int),
        ("setup_rounds", ctypes.c_int),
        ("setup_coarse_iters", ctypes.c_int),
        ("setup_boot", ctypes.c_int),
        ("setup_fine_iters", ctypes.c_int),
        ("mu_setup", ctypes.c_double),
        ("coarse_mu_factor", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("r_m", ctypes.c_double),
        ("r_b", ctypes.c_double),
        ("outer_restart", ctypes.c_int),
        ("max_outer", ctypes.c_int),
        ("inner_iters", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("inner_fp16", ctypes.c_int),
        ("middle_restart", ctypes.c_int),
        ("middle_maxit", ctypes.c_int),
        ("bottom_maxit", ctypes.c_int),
        ("coarse_smooth_iters", ctypes.c_int),
        ("coarsest_block", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("smoother_cycles", ctypes.c_int),
        ("col_tile", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("max_active_cols", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("verbose", ctypes.c_int),
        ("csw", ctypes.c_double),
        ("sap_oddeven", ctypes.c_int),
        ("coarse_gamma5", ctypes.c_int),
        ("bottom_restart", ctypes.c_int),
        ("bottom_dr_k", ctypes.c_int),
        ("coarse_fp16", ctypes.c_int),
        ("transfer_fp16", ctypes.c_int),
    ]


class ColInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("converged", ctypes.c_int), ("true_rel_res", ctypes.c_double),
                ("err_vs_fp64", ctypes.c_double), ("fallbacks", ctypes.c_int)]


def _info(i):
    return dict(outer_iters=i.outer_iters, converged=bool(i.converged), true_rel_res=i.true_rel_res,
                err_vs_fp64=i.err_vs_fp64, fallbacks=i.fallbacks)


class Stats(ctypes.Structure):
    _fields_ = [
        ("setup_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double), ("outer_iters", ctypes.c_int),
        ("avg_middle_iters", ctypes.c_double), ("avg_bottom_iters", ctypes.c_double),
        ("n_middle_solves", ctypes.c_longlong), ("n_bottom_solves", ctypes.c_longlong),
        ("n_fine_ops", ctypes.c_longlong), ("n_sap_calls", ctypes.c_longlong), ("learned_fallbacks", ctypes.c_int),
        ("col_removals", ctypes.c_int), ("n_inner_iters", ctypes.c_longlong),
        ("n_fp16_restores", ctypes.c_longlong), ("sap_kernel_ms", ctypes.c_double),
        ("n_sap_kernels", ctypes.c_longlong), ("n_sap_kernel_tiles", ctypes.c_longlong),
        ("device_bytes", ctypes.c_longlong), ("device_bytes_peak", ctypes.c_longlong),
    ]


_lib = None


def header_symbols() -> list:
    """Names of every function declared in include/ddamg.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ddamg_\w+)\s*\(", txt)))


def load():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_03872_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp, ip = ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int)
    sig = {
        "ddamg_default_params": (None, [P(Params)]),
        "ddamg_setup": (ctypes.c_int, [P(Params), vp, ctypes.c_int, vp, vp, P(vp)]),
        "ddamg_set_test_vectors": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "ddamg_get_test_vectors": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "ddamg_apply_op": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, vp, vp]),
        "ddamg_apply_op_noalloc": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, vp, vp]),
        "ddamg_apply_op_nd": (ctypes.c_int, [vp, ctypes.c_int, dp, dp, ctypes.c_int, vp, vp]),
        "ddamg_solve_nd": (ctypes.c_int, [vp, dp, dp, ctypes.c_int, vp, vp, ctypes.c_int, vp]),
        "ddamg_apply_sap": (ctypes.c_int, [vp, ctypes.c_int, dp, ctypes.c_int, vp, vp]),
        "ddamg_restrict": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]),
        "ddamg_prolong": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]),
        "ddamg_get_coarse_op": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "ddamg_level_info": (ctypes.c_int, [vp, ctypes.c_int, ip, ip, ip]),
        "ddamg_solve": (ctypes.c_int, [vp, dp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, P(ColInfo)]),
        "ddamg_solve_batch": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), dp, vp, vp,
                                             ctypes.c_int, P(ColInfo)]),
        "ddamg_coarse_solve": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, vp, vp,
                                              ctypes.c_double, ctypes.c_int, ip]),
        "ddamg_get_stats": (ctypes.c_int, [vp, P(Stats)]),
        "ddamg_time_op": (ctypes.c_int, [vp] + [ctypes.c_int] * 5 + [dp]),
        "ddamg_set_tuning": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
        "ddamg_get_tuning": (ctypes.c_int, [vp, ctypes.c_int, ip]),
        "ddamg_autotune": (ctypes.c_int, [vp, ctypes.c_int, ip]),
        "ddamg_smoother_set_weights": (ctypes.c_int, [vp, vp, vp]),
        "ddamg_smoother_get_weights": (ctypes.c_int, [vp, vp, vp]),
        "ddamg_smoother_apply": (ctypes.c_int, [vp, ctypes.c_int, vp, vp]),
        "ddamg_load_smoother": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "ddamg_save_smoother": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "ddamg_ptc_layer": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]),
        "ddamg_ptc_weight_grad": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "ddamg_train_smoother": (ctypes.c_int, [vp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_int, ctypes.c_uint64, dp]),
        "ddamg_destroy": (None, [vp]),
        "ddamg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "ddamg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code, allow=(OK,)):
    if code not in allow:
        lib = load()
        raise DDAMGError(code, f"{lib.ddamg_strerror(code).decode()}: {lib.ddamg_last_error().decode()}")
    return code


def default_params(**kw) -> Params:
    p = Params()
    load().ddamg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("dims", "n_tv", "sap_block"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
        elif k == "agg":
            for l, a in enumerate(v):
                for i, x in enumerate(a):
                    p.agg[l][i] = int(x)
        else:
            setattr(p, k, v)
    return p


def _dptr(t) -> int:
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise TypeError("expected a contiguous complex128 CUDA tensor")
    return t.data_ptr()


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mu(mu) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Context:
    """One solver context: gauge field, internal layouts and MG hierarchy."""

    def __init__(self, params: Params, gauge, tv_init: Optional[Sequence[np.ndarray]] = None):
        import torch
        lib = load()
        self.params = params
        g = np.ascontiguousarray(np.asarray(gauge, dtype=np.complex128))
        self._tv = None
        tvp = None
        if tv_init is not None:
            self._tv = [np.ascontiguousarray(np.asarray(t, dtype=np.complex128)) for t in tv_init]
            arr = (ctypes.c_void_p * len(self._tv))(*[t.ctypes.data for t in self._tv])
            self._tv_arr = arr
            tvp = ctypes.cast(arr, ctypes.c_void_p)
        h = ctypes.c_void_p()
        torch.cuda.current_stream().synchronize()
        _check(lib.ddamg_setup(ctypes.byref(params), g.ctypes.data, 0, tvp, _stream_handle(), ctypes.byref(h)))
        self.h = h
        self.device = torch.device("cuda")

    def close(self):
        if getattr(self, "h", None):
            load().ddamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        V, d = ctypes.c_int(), ctypes.c_int()
        dims = (ctypes.c_int * 4)()
        _check(load().ddamg_level_info(self.h, level, ctypes.byref(V), ctypes.byref(d), dims))
        return V.value, d.value, tuple(dims)

    def _vec(self, level, ncol):
        import torch
        V, d, _ = self.level_info(level)
        shape = (ncol, V, 4, 3) if level == 0 else (ncol, V, d)
        return torch.empty(shape, dtype=torch.complex128, device=self.device)

    def apply_op(self, level, precision, mu, x):
        m, mp = _mu(mu)
        y = self._vec(level, x.shape[0])
        _check(load().ddamg_apply_op(self.h, level, precision, mp, x.shape[0], _dptr(x), _dptr(y)))
        return y

    def apply_op_noalloc(self, level, precision, mu, x, y):
        """The no-allocation form of apply_op: the caller provides y (same
        shape as x); the library allocates nothing."""
        m, mp = _mu(mu)
        _check(load().ddamg_apply_op_noalloc(self.h, level, precision, mp, x.shape[0], _dptr(x), _dptr(y)))
        return y

    def apply_op_nd(self, precision, mubar, epsbar, x):
        """Doublet operator on x: [n_pair][2][V][4][3] (or [2 n_pair][V][4][3])
        complex128 CUDA tensor."""
        m, mp = _mu(mubar)
        e, ep = _mu(epsbar)
        y = torch_empty_like(x)
        _check(load().ddamg_apply_op_nd(self.h, precision, mp, ep, len(m), _dptr(x), _dptr(y)))
        return y

    def solve_nd(self, mubar, epsbar, b, x0=None):
        """Doublet solves: b [n_pair][2][V][4][3] complex128 CUDA tensor.
        Returns (x, info per column, status)."""
        m, mp = _mu(mubar)
        e, ep = _mu(epsbar)
        x = x0.clone() if x0 is not None else torch_zeros_like(b)
        info = (ColInfo * (2 * len(m)))()
        st = _check(load().ddamg_solve_nd(self.h, mp, ep, len(m), _dptr(b), _dptr(x), int(x0 is not None),
                                          ctypes.cast(info, ctypes.c_void_p)), allow=(OK, NOT_CONVERGED))
        return x, [_info(i) for i in info], st

    def apply_sap(self, precision, mu, f):
        m, mp = _mu(mu)
        x = self._vec(0, f.shape[0])
        _check(load().ddamg_apply_sap(self.h, precision, mp, f.shape[0], _dptr(f), _dptr(x)))
        return x

    def restrict(self, level, precision, x):
        y = self._vec(level + 1, x.shape[0])
        _check(load().ddamg_restrict(self.h, level, precision, x.shape[0], _dptr(x), _dptr(y)))
        return y

    def prolong(self, level, precision, x):
        y = self._vec(level, x.shape[0])
        _check(load().ddamg_prolong(self.h, level, precision, x.shape[0], _dptr(x), _dptr(y)))
        return y

    def coarse_op(self, level) -> np.ndarray:
        V, d, _ = self.level_info(level)
        out = np.empty((V, 9, d, d), dtype=np.complex128)
        _check(load().ddamg_get_coarse_op(self.h, level, out.ctypes.data))
        return out

    def test_vectors(self, level) -> np.ndarray:
        V, d, _ = self.level_info(level)
        N = self.params.n_tv[level]
        out = np.empty((N, V, d), dtype=np.complex128)
        _check(load().ddamg_get_test_vectors(self.h, level, out.ctypes.data))
        return out

    def set_test_vectors(self, level, tv):
        a = np.ascontiguousarray(np.asarray(tv, dtype=np.complex128))
        _check(load().ddamg_set_test_vectors(self.h, level, a.ctypes.data))

    def solve(self, mu, b, x0=None):
        """b: [n_rhs][V][4][3] complex128 CUDA tensor; mu: n_shift shifts.
        Returns (x [n_rhs*n_shift][V][4][3], info list, status)."""
        import torch
        m, mp = _mu(mu)
        n_rhs = b.shape[0]
        ncol = n_rhs * len(m)
        x = x0.clone() if x0 is not None else torch.zeros((ncol,) + tuple(b.shape[1:]), dtype=torch.complex128,
                                                          device=self.device)
        info = (ColInfo * ncol)()
        st = _check(load().ddamg_solve(self.h, mp, len(m), _dptr(b), n_rhs, _dptr(x), int(x0 is not None), info),
                    allow=(OK, NOT_CONVERGED))
        return x, [_info(i) for i in info], st

    def solve_batch(self, systems, x0=None):
        """systems: list of (mus, b) with b a [n_rhs][V][4][3] complex128
        tensor (CUDA, or host memory: then the right-hand sides are gathered on
        the host and copied to the device once); all systems are solved in one
        simultaneous batch.  Returns (list of x [n_rhs*n_shift][V][4][3] per
        system, list of info lists, status)."""
        import torch
        n_rhs = [int(b.shape[0]) for _, b in systems]
        n_shift = [len(np.atleast_1d(m)) for m, _ in systems]
        mu = np.ascontiguousarray(np.concatenate([np.atleast_1d(np.asarray(m, dtype=np.float64)) for m, _ in systems]))
        b = torch.cat([torch.as_tensor(bb) for _, bb in systems]).contiguous()
        if not b.is_cuda:
            b = b.to(self.device)
        ncol = sum(r * k for r, k in zip(n_rhs, n_shift))
        x = x0.clone() if x0 is not None else torch.zeros((ncol,) + tuple(b.shape[1:]), dtype=torch.complex128,
                                                          device=self.device)
        info = (ColInfo * ncol)()
        ir, ik = (ctypes.c_int * len(systems))(*n_rhs), (ctypes.c_int * len(systems))(*n_shift)
        st = _check(load().ddamg_solve_batch(self.h, len(systems), ir, ik,
                                             mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _dptr(b), _dptr(x),
                                             int(x0 is not None), info), allow=(OK, NOT_CONVERGED))
        xs, infos, o = [], [], 0
        for r, k in zip(n_rhs, n_shift):
            xs.append(x[o:o + r * k])
            infos.append([_info(i) for i in info[o:o + r * k]])
            o += r * k
        return xs, infos, st

    def coarse_solve(self, level, precision, block, mu, b, tol, maxit):
        """(Block) GMRES on coarse level `level`: b [n_col][Vc][dof] complex128
        CUDA tensor, mu [n_col].  Returns (x, iterations per column)."""
        import torch
        m, mp = _mu(mu)
        x = torch.zeros_like(b)
        it = (ctypes.c_int * b.shape[0])()
        _check(load().ddamg_coarse_solve(self.h, level, precision, int(bool(block)), mp, b.shape[0], _dptr(b),
                                         _dptr(x), float(tol), int(maxit), it))
        return x, list(it)

    def stats(self) -> dict:
        s = Stats()
        _check(load().ddamg_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    KNOBS = {"dslash_sites_fp64": 0, "dslash_sites_fp32": 1, "fp32_links": 2, "coarse_mfma": 3,
             "sap_variant": 4,
             "dslash_order": 5, "walk_segments": 6, "fp16_rescale": 7, "time_sap": 8, "time_kernel": 8,
             "gram_one_reduction": 9}

    # ---- learned smoother ----
    def set_smoother_weights(self, w1, w2):
        a = np.ascontiguousarray(np.asarray(w1, dtype=np.complex128).reshape(9, 2, 1, 4, 4))
        b = np.ascontiguousarray(np.asarray(w2, dtype=np.complex128).reshape(9, 1, 2, 4, 4))
        _check(load().ddamg_smoother_set_weights(self.h, a.ctypes.data, b.ctypes.data))

    def smoother_weights(self):
        a = np.empty((9, 2, 1, 4, 4), dtype=np.complex128)
        b = np.empty((9, 1, 2, 4, 4), dtype=np.complex128)
        _check(load().ddamg_smoother_get_weights(self.h, a.ctypes.data, b.ctypes.data))
        return a, b

    def load_smoother(self, path):
        _check(load().ddamg_load_smoother(self.h, os.fsencode(path)))

    def save_smoother(self, path):
        _check(load().ddamg_save_smoother(self.h, os.fsencode(path)))

    def smoother_apply(self, x):
        y = self._vec(0, x.shape[0])
        _check(load().ddamg_smoother_apply(self.h, x.shape[0], _dptr(x), _dptr(y)))
        return y

    def ptc_layer(self, layer, adjoint, x):
        """x: [c_in][n_col][V][4][3] complex128 CUDA tensor."""
        import torch
        cout = {(1, 0): 2, (2, 0): 1, (1, 1): 1, (2, 1): 2}[(layer, int(bool(adjoint)))]
        out = torch.empty((cout,) + tuple(x.shape[1:]), dtype=torch.complex128, device=self.device)
        _check(load().ddamg_ptc_layer(self.h, layer, int(bool(adjoint)), x.shape[1], _dptr(x), _dptr(out)))
        return out

    def ptc_weight_grad(self, layer, x, gout):
        cin, cout = (1, 2) if layer == 1 else (2, 1)
        g = np.empty((9, cout, cin, 4, 4), dtype=np.complex128)
        _check(load().ddamg_ptc_weight_grad(self.h, layer, x.shape[1], _dptr(x), _dptr(gout), g.ctypes.data))
        return g

    def train_smoother(self, mus, steps, batch, lr, sap_sweeps=0, seed=1):
        m, mp = _mu(mus)
        hist = np.zeros(steps)
        _check(load().ddamg_train_smoother(self.h, mp, len(m), int(steps), int(batch), float(lr), int(sap_sweeps),
                                           int(seed),
                                           hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return hist

    def set_tuning(self, knob, value):
        _check(load().ddamg_set_tuning(self.h, self.KNOBS.get(knob, knob), int(value)))

    def get_tuning(self, knob) -> int:
        v = ctypes.c_int()
        _check(load().ddamg_get_tuning(self.h, self.KNOBS.get(knob, knob), ctypes.byref(v)))
        return v.value

    def autotune(self, n_col) -> dict:
        vals = (ctypes.c_int * len(self.KNOBS))()
        _check(load().ddamg_autotune(self.h, int(n_col), vals))
        return {k: vals[i] for k, i in self.KNOBS.items()}

    def time_op(self, op, level, precision, n_col, n_iter) -> float:
        sec = ctypes.c_double()
        _check(load().ddamg_time_op(self.h, op, level, precision, n_col, n_iter, ctypes.byref(sec)))
        return sec.value


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)


def torch_zeros_like(t):
    import torch
    return torch.zeros_like(t)


def params_for_workload(w, **overrides) -> Params:
    """ddamg_params of a synthetic workload description (see synthetic.Workload)."""
    kw = dict(dims=w.dims, kappa=w.kappa, n_levels=w.n_levels, sap_block=w.sap_block,
              mu_setup=float(min(w.mus)))
    if w.n_levels > 1:
        agg = [list(a) for a in w.agg] + [[1, 1, 1, 1]] * (2 - len(w.agg))
        n_tv = list(w.n_tv) + [8] * (2 - len(w.n_tv))
        kw.update(agg=agg, n_tv=n_tv)
    kw.update(overrides)
    return default_params(**kw)
