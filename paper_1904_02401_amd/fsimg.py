"""ctypes binding of the fsimg C ABI (include/fsimg.h, include/fsimg_newton.h).

Argument marshalling only: every function forwards to the entry point of the
same name in libfsimg.so, which runs all numerical work in HIP kernels on the
GPU.  Device vectors are passed as torch tensors (or raw integer device
addresses); streams as torch.cuda.Stream, raw hipStream_t integers, or None
(the current torch stream).  There is no CPU fallback: if the library is
missing, importing this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsimg.so")

FSIMG_OK, FSIMG_ERR_ARG, FSIMG_ERR_OOM, FSIMG_ERR_HIP, FSIMG_ERR_SINGULAR = 0, 1, 2, 3, 4
FSIMG_ERR_NOCONV, FSIMG_ERR_NONFINITE, FSIMG_ERR_BUDGET, FSIMG_ERR_STATE = 5, 6, 7, 8
FSIMG_FP64, FSIMG_MIXED = 0, 1
FSIMG_VANKA_GATHER, FSIMG_VANKA_PARITY, FSIMG_VANKA_GREEDY = 0, 1, 2
FSIMG_WEIGHT_PLAIN, FSIMG_WEIGHT_MULT = 0, 1
FSIMG_TUNE_SPMV_ROWS, FSIMG_TUNE_VANKA_PPW = 0, 1
FSIMG_PATCH_ELEMENT, FSIMG_PATCH_BLOCK = 0, 1
FSIMG_SMOOTHER_VANKA, FSIMG_SMOOTHER_ILU = 0, 1

_STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_HIP", 4: "ERR_SINGULAR",
                 5: "ERR_NOCONV", 6: "ERR_NONFINITE", 7: "ERR_BUDGET", 8: "ERR_STATE"}


class FsimgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fsimg {_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class fsimg_level_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("block", ctypes.c_int), ("cells", ctypes.c_int * 3),
                ("nrows", ctypes.c_int64), ("nnzb", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("dirichlet", ctypes.c_void_p),
                ("cell_class", ctypes.c_void_p)]


class fsimg_opts(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("rtol", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("vanka_schedule", ctypes.c_int),
                ("vanka_weighting", ctypes.c_int), ("profile", ctypes.c_int),
                ("graphs", ctypes.c_int), ("vanka_patches", ctypes.c_int),
                ("smoother", ctypes.c_int), ("omega_ilu", ctypes.c_double),
                ("krylov_lookahead", ctypes.c_int), ("small_level_kib", ctypes.c_int)]


FSIMG_HIST = 64


class fsimg_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("vanka_ms", ctypes.c_double), ("vanka_launches", ctypes.c_int),
                ("spmv_ms", ctypes.c_double), ("spmv_launches", ctypes.c_int),
                ("restrict_ms", ctypes.c_double), ("restrict_launches", ctypes.c_int),
                ("prolong_ms", ctypes.c_double), ("prolong_launches", ctypes.c_int),
                ("setup_ms", ctypes.c_double), ("factor_ms", ctypes.c_double),
                ("bytes_moved", ctypes.c_double), ("nhist", ctypes.c_int),
                ("res_hist", ctypes.c_double * FSIMG_HIST)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "res_hist"}
        d["res_hist"] = [self.res_hist[i] for i in range(self.nhist)]
        return d


class fsimg_request(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int), ("mom", ctypes.POINTER(fsimg_level_desc)),
                ("ale", ctypes.POINTER(fsimg_level_desc)), ("b_mom", ctypes.c_void_p),
                ("b_ale", ctypes.c_void_p), ("node_solid", ctypes.c_void_p),
                ("time_steps", ctypes.c_int), ("newton_steps", ctypes.c_void_p),
                ("k", ctypes.c_double), ("theta", ctypes.c_double), ("arrival", ctypes.c_double),
                ("n_states", ctypes.c_int), ("state_vals", ctypes.POINTER(ctypes.c_void_p)),
                ("n_rhs", ctypes.c_int), ("rhs_mom", ctypes.POINTER(ctypes.c_void_p))]


class fsimg_level_info(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("n", ctypes.c_int64), ("nnzb", ctypes.c_int64),
                ("npatch", ctypes.c_int64), ("np", ctypes.c_int), ("ncolours", ctypes.c_int),
                ("bytes", ctypes.c_size_t), ("factor_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fsimg_phys(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("rho_f", "nu_f", "rho_s", "mu_s", "lambda_s", "k",
                                                "theta", "alpha0")]


class fsimg_fsi_level(ctypes.Structure):
    _fields_ = [("coords", ctypes.c_void_p * 3), ("cell_solid", ctypes.c_void_p),
                ("node_coords", ctypes.c_void_p)]


def _fill_geometry(arr, levels, keep):
    """levels: per level (coords per axis, cell_solid[, node_coords or None])"""
    for l, lv in enumerate(levels):
        coords, solid = lv[0], lv[1]
        xyz = lv[2] if len(lv) > 2 else None
        cs = [np.ascontiguousarray(c, dtype=np.float64) for c in coords]
        sd = np.ascontiguousarray(solid, dtype=np.uint8)
        keep += cs + [sd]
        for a in range(3):
            arr[l].coords[a] = cs[a].ctypes.data if a < len(cs) else None
        arr[l].cell_solid = sd.ctypes.data
        if xyz is not None:
            xa = np.ascontiguousarray(xyz, dtype=np.float64)
            keep.append(xa)
            arr[l].node_coords = xa.ctypes.data
        else:
            arr[l].node_coords = None


class fsimg_newton_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_steps", ctypes.c_int),
                ("gamma", ctypes.c_double), ("max_halvings", ctypes.c_int), ("lin_rtol", ctypes.c_double),
                ("ale_rtol", ctypes.c_double)]


class fsimg_newton_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int), ("jacobians", ctypes.c_int),
                ("halvings", ctypes.c_int), ("lin_iters_mom", ctypes.c_int),
                ("lin_iters_ale", ctypes.c_int), ("res0", ctypes.c_double), ("res", ctypes.c_double),
                ("res_hist", ctypes.c_double * 32), ("omega_hist", ctypes.c_double * 32),
                ("ms_total", ctypes.c_double), ("ms_residual", ctypes.c_double),
                ("ms_jacobian", ctypes.c_double), ("ms_factor", ctypes.c_double),
                ("ms_solve", ctypes.c_double)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n not in ("res_hist", "omega_hist")}
        d["res_hist"] = [self.res_hist[i] for i in range(min(self.steps + 1, 32))]
        d["omega_hist"] = [self.omega_hist[i] for i in range(min(self.steps, 32))]
        return d


class fsimg_newton_request(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int), ("mom", ctypes.c_void_p), ("ale", ctypes.c_void_p),
                ("geom", ctypes.c_void_p), ("phys", fsimg_phys), ("x", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("x_old", ctypes.c_void_p), ("u_old", ctypes.c_void_p),
                ("time_steps", ctypes.c_int), ("newton", fsimg_newton_opts), ("arrival", ctypes.c_double)]


# entry point -> argument types
_P, _I, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "fsimg_default_opts": (None, [ctypes.POINTER(fsimg_opts)]),
    "fsimg_ctx_create": (_I, [_I, _SZ, ctypes.POINTER(_P)]),
    "fsimg_ctx_destroy": (None, [_P]),
    "fsimg_ctx_bytes_in_use": (_SZ, [_P]),
    "fsimg_hier_footprint": (_I, [ctypes.POINTER(fsimg_level_desc), _I, ctypes.POINTER(fsimg_opts),
                                  ctypes.POINTER(_SZ)]),
    "fsimg_hier_create": (_I, [_P, ctypes.POINTER(fsimg_level_desc), _I, ctypes.POINTER(fsimg_opts),
                               _P, ctypes.POINTER(_P)]),
    "fsimg_hier_destroy": (None, [_P]),
    "fsimg_hier_info": (_I, [_P, _I, ctypes.POINTER(fsimg_level_info)]),
    "fsimg_hier_update_values": (_I, [_P, _I, _P, _I, _P]),
    "fsimg_hier_set_profile": (_I, [_P, _I]),
    "fsimg_factor": (_I, [_P, _P]),
    "fsimg_solve": (_I, [_P, _P, _P, ctypes.POINTER(fsimg_stats), _P]),
    "fsimg_solve_noalloc": (_I, [_P, _P, _P, ctypes.POINTER(fsimg_stats), _P]),
    "fsimg_solve_batch": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                               ctypes.POINTER(fsimg_stats), _P]),
    "fsimg_deform_update": (_I, [_I64, _I, _P, _D, _D, _P, _I, _I, _P, _P, _P, _P]),
    "fsimg_level_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "fsimg_level_residual": (_I, [_P, _I, _I, _P, _P, _P, _P]),
    "fsimg_vanka_step": (_I, [_P, _I, _I, _P, _P, _P]),
    "fsimg_ilu_step": (_I, [_P, _I, _I, _P, _P, _P]),
    "fsimg_ilu_factors": (_I, [_P, _I, _P]),
    "fsimg_restrict": (_I, [_P, _I, _I, _P, _P, _P]),
    "fsimg_prolong_add": (_I, [_P, _I, _I, _P, _P, _P]),
    "fsimg_coarse_solve": (_I, [_P, _P, _P, _P]),
    "fsimg_vcycle": (_I, [_P, _I, _P, _P, _P]),
    "fsimg_patch_inverse": (_I, [_P, _I, _I64, _P, ctypes.POINTER(_I64), _P]),
    "fsimg_server_create": (_I, [_P, ctypes.POINTER(fsimg_opts), _I, ctypes.POINTER(_P)]),
    "fsimg_server_destroy": (None, [_P]),
    "fsimg_server_clock": (_D, [_P]),
    "fsimg_server_submit": (_I, [_P, ctypes.POINTER(fsimg_request), ctypes.POINTER(_I64)]),
    "fsimg_server_step": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), _P]),
    "fsimg_server_poll": (_I, [_P, _P, _P, _P, _I, ctypes.POINTER(_I)]),
    "fsimg_server_result": (_I, [_P, _I64, _P, _P]),
    "fsimg_server_request_status": (_I, [_P, _I64, ctypes.POINTER(_I)]),
    "fsimg_server_release": (_I, [_P, _I64]),
    "fsimg_hier_tune": (_I, [_P, _I, _P]),
    "fsimg_server_set_order": (_I, [_P, _I]),
    "fsimg_tune_schedule": (_I, [_P, ctypes.POINTER(fsimg_level_desc), _I, ctypes.POINTER(fsimg_opts), _I,
                                 ctypes.POINTER(_D), ctypes.POINTER(_I), _P]),
    "fsimg_tune_set": (_I, [_P, _I, _I, _I, _I64, _I]),
    "fsimg_tune_get": (_I, [_P, _I, _I, _I, _I64, ctypes.POINTER(_I)]),
    "fsimg_tune_save": (_I, [_P, ctypes.c_char_p]),
    "fsimg_tune_load": (_I, [_P, ctypes.c_char_p]),
    "fsimg_last_error": (ctypes.c_char_p, []),
    "fsimg_fsi_create": (_I, [_P, _P, ctypes.POINTER(fsimg_fsi_level), ctypes.POINTER(fsimg_phys),
                              ctypes.POINTER(_P)]),
    "fsimg_fsi_destroy": (None, [_P]),
    "fsimg_fsi_residual": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "fsimg_fsi_jacobian": (_I, [_P, _P, _P, _P, _P, _P]),
    "fsimg_default_newton_opts": (None, [ctypes.POINTER(fsimg_newton_opts)]),
    "fsimg_fsi_newton": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(fsimg_newton_opts),
                              ctypes.POINTER(fsimg_newton_stats), _P]),
    "fsimg_fsi_drop_jacobian": (_I, [_P]),
    "fsimg_fsi_time_step": (_I, [_P, _P, _P, _P, _P, _P, _P, _I64, _D, ctypes.POINTER(fsimg_newton_opts),
                                 ctypes.POINTER(fsimg_newton_stats), _P]),
    "fsimg_fsi_force": (_I, [_P, _P, _P, _P, _P, _P, _I64, ctypes.POINTER(_D), _P]),
    "fsimg_server_submit_newton": (_I, [_P, ctypes.POINTER(fsimg_newton_request), ctypes.POINTER(_I64)]),
    "fsimg_server_newton_stats": (_I, [_P, _I64, ctypes.POINTER(fsimg_newton_stats)]),
    "fsimg_fsi_set_profile": (_I, [_P, _I]),
    "fsimg_fsi_profile": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_D),
                               ctypes.POINTER(_I)]),
}
EXPORTED = tuple(_SIGS)

_lib = None


def load(path: str = LIB_PATH):
    """Load libfsimg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise FsimgError(FSIMG_ERR_STATE, f"{path} not built: run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != FSIMG_OK:
        raise FsimgError(status, load().fsimg_last_error().decode())


def _dev(t, dtype=None, numel=None):
    """device address of a tensor (or an int address / None).  dtype: the
    torch dtype the kernels read (checked when given); numel: the number of
    elements they read (the tensor must hold at least that many)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected a {dtype} tensor, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"expected at least {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _f64():
    import torch
    return torch.float64


def _i64():
    import torch
    return torch.int64


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ---------------------------------------------------------------- helpers
def fsimg_default_opts(**overrides) -> fsimg_opts:
    o = fsimg_opts()
    load().fsimg_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class LevelDescs:
    """Host-side descriptor array for a list of levels; keeps the numpy
    buffers alive for the duration of a call."""

    def __init__(self, levels):
        self._keep = []
        self.levels = levels
        n = len(levels)
        self.arr = (fsimg_level_desc * n)()
        for i, lv in enumerate(levels):
            d = self.arr[i]
            d.dim, d.block = int(lv["dim"]), int(lv["block"])
            cells = list(lv["cells"]) + [1] * (3 - len(lv["cells"]))
            for a in range(3):
                d.cells[a] = int(cells[a])
            rp = np.ascontiguousarray(lv["rowptr"], dtype=np.int32)
            ci = np.ascontiguousarray(lv["colind"], dtype=np.int32)
            va = np.ascontiguousarray(lv["vals"], dtype=np.float64)
            di = np.ascontiguousarray(lv["dirichlet"], dtype=np.uint8)
            cc = lv.get("cell_class")
            cc = None if cc is None else np.ascontiguousarray(cc, dtype=np.uint8)
            self._keep += [rp, ci, va, di, cc]
            d.nrows = rp.shape[0] - 1
            d.nnzb = ci.shape[0]
            d.rowptr, d.colind = rp.ctypes.data, ci.ctypes.data
            d.vals, d.dirichlet = va.ctypes.data, di.ctypes.data
            d.cell_class = None if cc is None else cc.ctypes.data
        self.n = n


# ------------------------------------------------------------- entry points
def fsimg_ctx_create(device: int = 0, hbm_budget_bytes: int = 0):
    out = ctypes.c_void_p()
    _check(load().fsimg_ctx_create(device, hbm_budget_bytes, ctypes.byref(out)))
    return out.value


def fsimg_ctx_destroy(ctx):
    load().fsimg_ctx_destroy(ctx)


def fsimg_ctx_bytes_in_use(ctx) -> int:
    return load().fsimg_ctx_bytes_in_use(ctx)


def fsimg_hier_footprint(levels, opts) -> int:
    d = LevelDescs(levels)
    out = ctypes.c_size_t()
    _check(load().fsimg_hier_footprint(d.arr, d.n, ctypes.byref(opts), ctypes.byref(out)))
    return out.value


def fsimg_hier_create(ctx, levels, opts, stream=None):
    d = LevelDescs(levels)
    out = ctypes.c_void_p()
    _check(load().fsimg_hier_create(ctx, d.arr, d.n, ctypes.byref(opts), _stream(stream),
                                    ctypes.byref(out)))
    return out.value


def fsimg_hier_destroy(h):
    load().fsimg_hier_destroy(h)


def fsimg_hier_info(h, level: int) -> dict:
    info = fsimg_level_info()
    _check(load().fsimg_hier_info(h, level, ctypes.byref(info)))
    return info.as_dict()


def fsimg_hier_update_values(h, level: int, vals, stream=None):
    if isinstance(vals, np.ndarray):
        v = np.ascontiguousarray(vals, dtype=np.float64)
        _check(load().fsimg_hier_update_values(h, level, v.ctypes.data, 0, _stream(stream)))
    else:
        _check(load().fsimg_hier_update_values(h, level, _dev(vals), 1, _stream(stream)))


def fsimg_hier_set_profile(h, on: int):
    _check(load().fsimg_hier_set_profile(h, int(on)))


def fsimg_factor(h, stream=None):
    _check(load().fsimg_factor(h, _stream(stream)))


def fsimg_solve(h, b, x, stream=None, raise_on_noconv: bool = True) -> dict:
    st = fsimg_stats()
    rc = load().fsimg_solve(h, _dev(b), _dev(x), ctypes.byref(st), _stream(stream))
    if rc != FSIMG_OK and (raise_on_noconv or rc != FSIMG_ERR_NOCONV):
        _check(rc)
    return st.as_dict()


def fsimg_solve_noalloc(h, b, x, stream=None, raise_on_noconv: bool = True) -> dict:
    st = fsimg_stats()
    rc = load().fsimg_solve_noalloc(h, _dev(b), _dev(x), ctypes.byref(st), _stream(stream))
    if rc != FSIMG_OK and (raise_on_noconv or rc != FSIMG_ERR_NOCONV):
        _check(rc)
    return st.as_dict()


def fsimg_solve_batch(hiers, bs, xs, stream=None, raise_on_noconv: bool = True) -> list:
    """Solve len(hiers) independent systems in one batched solve; returns the
    per-instance stats."""
    n = len(hiers)
    H = (ctypes.c_void_p * n)(*hiers)
    B = (ctypes.c_void_p * n)(*[_dev(t) for t in bs])
    X = (ctypes.c_void_p * n)(*[_dev(t) for t in xs])
    st = (fsimg_stats * n)()
    rc = load().fsimg_solve_batch(n, H, B, X, st, _stream(stream))
    if rc != FSIMG_OK and (raise_on_noconv or rc != FSIMG_ERR_NOCONV):
        _check(rc)
    return [s.as_dict() for s in st]


def fsimg_deform_update(nnodes: int, dim: int, mask, k: float, theta: float, v_new, v_stride: int,
                        v_offset: int, u_old, v_old, u_new, stream=None):
    _check(load().fsimg_deform_update(nnodes, dim, _dev(mask), k, theta, _dev(v_new), v_stride,
                                      v_offset, _dev(u_old), _dev(v_old), _dev(u_new),
                                      _stream(stream)))


def fsimg_level_apply(h, level, precision, x, y, stream=None):
    _check(load().fsimg_level_apply(h, level, precision, _dev(x), _dev(y), _stream(stream)))


def fsimg_level_residual(h, level, precision, b, x, d, stream=None):
    _check(load().fsimg_level_residual(h, level, precision, _dev(b), _dev(x), _dev(d),
                                       _stream(stream)))


def fsimg_vanka_step(h, level, precision, b, x, stream=None):
    _check(load().fsimg_vanka_step(h, level, precision, _dev(b), _dev(x), _stream(stream)))


def fsimg_ilu_step(h, level, precision, b, x, stream=None):
    _check(load().fsimg_ilu_step(h, level, precision, _dev(b), _dev(x), _stream(stream)))


def fsimg_ilu_factors(h, level: int, nnzb: int, b: int) -> np.ndarray:
    """The FP64 ILU factors of a level, [nnzb, b, b] in the matrix's layout."""
    out = np.empty(nnzb * b * b, dtype=np.float64)
    _check(load().fsimg_ilu_factors(h, level, out.ctypes.data))
    return out.reshape(nnzb, b, b)


def fsimg_restrict(h, level, precision, rf, rc, stream=None):
    _check(load().fsimg_restrict(h, level, precision, _dev(rf), _dev(rc), _stream(stream)))


def fsimg_prolong_add(h, level, precision, xc, xf, stream=None):
    _check(load().fsimg_prolong_add(h, level, precision, _dev(xc), _dev(xf), _stream(stream)))


def fsimg_coarse_solve(h, r, x, stream=None):
    _check(load().fsimg_coarse_solve(h, _dev(r), _dev(x), _stream(stream)))


def fsimg_vcycle(h, precision, r, z, stream=None):
    _check(load().fsimg_vcycle(h, precision, _dev(r), _dev(z), _stream(stream)))


def fsimg_patch_inverse(h, level: int, patch: int, stream=None):
    info = fsimg_hier_info(h, level)
    npp = info["np"]
    out = np.empty((npp, npp), dtype=np.float64)
    elem = ctypes.c_int64()
    _check(load().fsimg_patch_inverse(h, level, patch, out.ctypes.data, ctypes.byref(elem),
                                      _stream(stream)))
    return out, elem.value


# ------------------------------------------------------------------ serving
class RequestData:
    """Host data of one simulation request: momentum / ALE level descriptors,
    further momentum states (per state, one value array per level, same
    pattern), momentum right-hand sides (the first is b_mom), the ALE
    right-hand side and the interface/solid node mask.  The arrays must stay
    alive until the request completes; one RequestData may back many
    requests."""

    def __init__(self, mom_levels, ale_levels, b_mom, b_ale, node_solid, k, theta,
                 states=(), rhs=()):
        self.mom = LevelDescs(mom_levels)
        self.ale = LevelDescs(ale_levels)
        self.b_mom = np.ascontiguousarray(b_mom, dtype=np.float64)
        self.b_ale = np.ascontiguousarray(b_ale, dtype=np.float64)
        self.node_solid = np.ascontiguousarray(node_solid, dtype=np.uint8)
        self.k, self.theta = float(k), float(theta)
        self.nlev = self.mom.n
        self.states = [[np.ascontiguousarray(v, dtype=np.float64) for v in st] for st in states]
        for st in self.states:
            if len(st) != self.nlev:
                raise ValueError("every state needs one value array per level")
        self.rhs = [np.ascontiguousarray(b, dtype=np.float64) for b in rhs]
        flat = [v.ctypes.data for st in self.states for v in st]
        self.state_ptrs = (ctypes.c_void_p * max(len(flat), 1))(*flat)
        self.rhs_ptrs = (ctypes.c_void_p * max(len(self.rhs), 1))(*[b.ctypes.data for b in self.rhs])


def fsimg_server_create(ctx, opts, max_active: int = 0):
    out = ctypes.c_void_p()
    _check(load().fsimg_server_create(ctx, ctypes.byref(opts), max_active, ctypes.byref(out)))
    return out.value


def fsimg_server_destroy(srv):
    load().fsimg_server_destroy(srv)


def fsimg_server_clock(srv) -> float:
    return load().fsimg_server_clock(srv)


def fsimg_server_submit(srv, data: RequestData, newton_steps, arrival: float) -> int:
    ns = np.ascontiguousarray(newton_steps, dtype=np.int32)
    req = fsimg_request(nlev=data.nlev, mom=data.mom.arr, ale=data.ale.arr,
                        b_mom=data.b_mom.ctypes.data, b_ale=data.b_ale.ctypes.data,
                        node_solid=data.node_solid.ctypes.data, time_steps=len(ns),
                        newton_steps=ns.ctypes.data, k=data.k, theta=data.theta, arrival=arrival,
                        n_states=1 + len(data.states), state_vals=data.state_ptrs,
                        n_rhs=1 + len(data.rhs), rhs_mom=data.rhs_ptrs)
    rid = ctypes.c_int64()
    _check(load().fsimg_server_submit(srv, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def fsimg_server_step(srv, stream=None):
    a, q = ctypes.c_int(), ctypes.c_int()
    _check(load().fsimg_server_step(srv, ctypes.byref(a), ctypes.byref(q), _stream(stream)))
    return a.value, q.value


def fsimg_server_poll(srv, max_n: int = 1024):
    ids = np.zeros(max_n, dtype=np.int64)
    adm = np.zeros(max_n)
    fin = np.zeros(max_n)
    c = ctypes.c_int()
    _check(load().fsimg_server_poll(srv, ids.ctypes.data, adm.ctypes.data, fin.ctypes.data, max_n,
                                    ctypes.byref(c)))
    n = c.value
    return ids[:n], adm[:n], fin[:n]


def fsimg_server_result(srv, rid: int, n_mom: int, n_ale: int):
    xm = np.zeros(n_mom)
    xa = np.zeros(n_ale)
    _check(load().fsimg_server_result(srv, rid, xm.ctypes.data, xa.ctypes.data))
    return xm, xa


def fsimg_server_request_status(srv, rid: int) -> int:
    st = ctypes.c_int()
    _check(load().fsimg_server_request_status(srv, rid, ctypes.byref(st)))
    return st.value


def fsimg_server_release(srv, rid: int):
    _check(load().fsimg_server_release(srv, rid))


def fsimg_hier_tune(h, force: bool = False, stream=None):
    _check(load().fsimg_hier_tune(h, 1 if force else 0, _stream(stream)))


def fsimg_server_set_order(srv, order: int):
    """0: first fit in arrival order; 1: least work first"""
    _check(load().fsimg_server_set_order(srv, order))


def fsimg_tune_schedule(ctx, levels, opts, reps: int = 5, stream=None):
    """(ms per V-cycle for GATHER, PARITY, GREEDY (-1: not applicable), the
    fastest schedule)"""
    d = LevelDescs(levels)
    ms = (ctypes.c_double * 3)()
    best = ctypes.c_int()
    _check(load().fsimg_tune_schedule(ctx, d.arr, d.n, ctypes.byref(opts), reps, ms, ctypes.byref(best),
                                      _stream(stream)))
    return list(ms), best.value


def fsimg_tune_set(ctx, kind: int, key: int, word: int, size: int, value: int):
    _check(load().fsimg_tune_set(ctx, kind, key, word, size, value))


def fsimg_tune_get(ctx, kind: int, key: int, word: int, size: int) -> int:
    v = ctypes.c_int()
    _check(load().fsimg_tune_get(ctx, kind, key, word, size, ctypes.byref(v)))
    return v.value


def fsimg_tune_save(ctx, path: str):
    _check(load().fsimg_tune_save(ctx, os.fsencode(path)))


def fsimg_tune_load(ctx, path: str):
    _check(load().fsimg_tune_load(ctx, os.fsencode(path)))


# ------------------------------------------------------------ Newton loop
def fsimg_phys_of(params: dict) -> fsimg_phys:
    return fsimg_phys(**{n: float(params[n]) for n, _ in fsimg_phys._fields_})


def fsimg_fsi_create(mom, ale, levels, params: dict):
    """levels: per multigrid level (coords per axis, cell_solid uint8[, node
    positions [nnodes, dim] or None]) of the momentum hierarchy; params: the
    fsimg_phys fields."""
    keep = []
    arr = (fsimg_fsi_level * len(levels))()
    _fill_geometry(arr, levels, keep)
    out = ctypes.c_void_p()
    _check(load().fsimg_fsi_create(mom, ale, arr, ctypes.byref(fsimg_phys_of(params)),
                                   ctypes.byref(out)))
    info = fsimg_hier_info(mom, 0)
    _FSI_SIZES[out.value] = (info["n"], info["nrows"] * len(levels[0][0]))
    return out.value


# finest-level lengths of x = (p, v) and u per Newton object (the kernels read
# that many FP64 entries of every state vector)
_FSI_SIZES = {}


def _state(f, x, u, x_old, u_old):
    nx, nu = _FSI_SIZES.get(f, (None, None))
    f64 = _f64()
    return (_dev(x, f64, nx), _dev(u, f64, nu), _dev(x_old, f64, nx), _dev(u_old, f64, nu))


def fsimg_fsi_destroy(f):
    _FSI_SIZES.pop(f, None)
    load().fsimg_fsi_destroy(f)


def fsimg_fsi_residual(f, x, u, x_old, u_old, res, stream=None):
    _check(load().fsimg_fsi_residual(f, *_state(f, x, u, x_old, u_old),
                                     _dev(res, _f64(), _FSI_SIZES.get(f, (None,))[0]), _stream(stream)))


def fsimg_fsi_jacobian(f, x, u, x_old, u_old, stream=None):
    _check(load().fsimg_fsi_jacobian(f, *_state(f, x, u, x_old, u_old), _stream(stream)))


def fsimg_default_newton_opts(**overrides) -> fsimg_newton_opts:
    o = fsimg_newton_opts()
    load().fsimg_default_newton_opts(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def fsimg_fsi_newton(f, x, u, x_old, u_old, opts=None, stream=None, raise_on_noconv: bool = True) -> dict:
    st = fsimg_newton_stats()
    o = opts if opts is not None else fsimg_default_newton_opts()
    rc = load().fsimg_fsi_newton(f, *_state(f, x, u, x_old, u_old), ctypes.byref(o),
                                 ctypes.byref(st), _stream(stream))
    if rc != FSIMG_OK and (raise_on_noconv or rc != FSIMG_ERR_NOCONV):
        _check(rc)
    return st.as_dict()


def fsimg_fsi_drop_jacobian(f):
    _check(load().fsimg_fsi_drop_jacobian(f))


def fsimg_fsi_time_step(f, x, u, x_old, u_old, rows=None, vals=None, scale: float = 1.0, opts=None,
                        stream=None, raise_on_noconv: bool = True) -> dict:
    """rows (int64) and vals (float64): device tensors of the held rows of x
    and their unscaled values, or None."""
    st = fsimg_newton_stats()
    o = opts if opts is not None else fsimg_default_newton_opts()
    n = 0 if rows is None else int(rows.numel())
    rc = load().fsimg_fsi_time_step(f, *_state(f, x, u, x_old, u_old),
                                    _dev(rows, _i64()) if n else None,
                                    _dev(vals, _f64(), n) if n else None, n,
                                    float(scale), ctypes.byref(o), ctypes.byref(st), _stream(stream))
    if rc != FSIMG_OK and (raise_on_noconv or rc != FSIMG_ERR_NOCONV):
        _check(rc)
    return st.as_dict()


def fsimg_fsi_force(f, x, u, x_old, u_old, nodes, dim: int, stream=None):
    """nodes: int64 device tensor; returns [dim] floats (drag, lift[, z])."""
    out = (_D * 3)()
    _check(load().fsimg_fsi_force(f, *_state(f, x, u, x_old, u_old), _dev(nodes, _i64()),
                                  int(nodes.numel()), out, _stream(stream)))
    return [out[j] for j in range(dim)]


def fsimg_fsi_set_profile(f, on: int):
    _check(load().fsimg_fsi_set_profile(f, on))


def fsimg_fsi_profile(f) -> dict:
    jm, rm = ctypes.c_double(), ctypes.c_double()
    jn, rn = ctypes.c_int(), ctypes.c_int()
    _check(load().fsimg_fsi_profile(f, ctypes.byref(jm), ctypes.byref(jn), ctypes.byref(rm),
                                    ctypes.byref(rn)))
    return dict(jac_ms=jm.value, jac_launches=jn.value, res_ms=rm.value, res_launches=rn.value)


class NewtonRequestData:
    """Host data of one Newton serving request: momentum / ALE level
    descriptors, the momentum levels' geometry (coordinates per axis,
    cell_solid), material parameters and the initial state (x, u) with its
    t_{n-1} state.  The arrays must stay alive until the request completes."""

    def __init__(self, mom_levels, ale_levels, geometry, params, x, u, x_old, u_old):
        self.mom = LevelDescs(mom_levels)
        self.ale = LevelDescs(ale_levels)
        self.nlev = self.mom.n
        self._keep = []
        self.geom = (fsimg_fsi_level * self.nlev)()
        _fill_geometry(self.geom, geometry, self._keep)
        self.phys = fsimg_phys_of(params)
        self.vecs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, u, x_old, u_old)]


def fsimg_server_submit_newton(srv, data: NewtonRequestData, time_steps: int, opts=None,
                               arrival: float = 0.0) -> int:
    o = opts if opts is not None else fsimg_default_newton_opts()
    x, u, xo, uo = data.vecs
    req = fsimg_newton_request(nlev=data.nlev, mom=ctypes.cast(data.mom.arr, ctypes.c_void_p),
                               ale=ctypes.cast(data.ale.arr, ctypes.c_void_p),
                               geom=ctypes.cast(data.geom, ctypes.c_void_p), phys=data.phys,
                               x=x.ctypes.data, u=u.ctypes.data, x_old=xo.ctypes.data,
                               u_old=uo.ctypes.data, time_steps=int(time_steps), newton=o,
                               arrival=float(arrival))
    rid = ctypes.c_int64()
    _check(load().fsimg_server_submit_newton(srv, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def fsimg_server_newton_stats(srv, rid: int) -> dict:
    st = fsimg_newton_stats()
    _check(load().fsimg_server_newton_stats(srv, rid, ctypes.byref(st)))
    d = {n: getattr(st, n) for n, _ in st._fields_ if n not in ("res_hist", "omega_hist")}
    return d
