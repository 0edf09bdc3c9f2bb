"""Python binding of the gfx950 NMF library (``libnmf_mi355x.so``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory and the current HIP stream.  If
the library has not been built the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# NMF_LIB names another build of the same library (the host-sanitizer build
# the CPU tests make); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("NMF_LIB") or os.path.join(_PKG, "libnmf_mi355x.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "nmf_mi355x.h")

NMF_OK = 0
NMF_ERR_ARG, NMF_ERR_SHAPE, NMF_ERR_NONFINITE, NMF_ERR_NEGATIVE = -1, -2, -3, -4
NMF_ERR_DIVERGED, NMF_ERR_HIP, NMF_ERR_NOMEM, NMF_ERR_UNSUPPORTED = -5, -6, -7, -8
NMF_WARN_NONMONOTONE, NMF_WARN_MAXITER = 1, 2

PREC = {"fp32": 0, "bf16x3": 1}
F_VALIDATE_DATA, F_CLIP_NEGATIVE, F_NORMALIZE_H = 1, 2, 4
F_BINARY_WEIGHTS, F_MASKED_GRAM, F_WARM_START, F_ASYNC, F_AUTOTUNE = 8, 16, 32, 64, 128
RS_WARM_FALLBACK = 1 << 8  # report status bit: a warm start fell back to the cold start

MAT_W, MAT_H, MAT_C = 0, 1, 2


class NmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("k", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("tol", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_int32), ("floor_eps", ctypes.c_float),
        ("split", ctypes.c_int32), ("waves", ctypes.c_int32), ("pipeline", ctypes.c_int32),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("iters_run", ctypes.c_int32),
        ("status_flags", ctypes.c_int32), ("objective", ctypes.c_double),
        ("objective_rel", ctypes.c_double), ("elapsed_ms", ctypes.c_float),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "struct_size"}


_vp, _i64, _i32, _u64, _dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p
_SIGS = {
    "nmf_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "nmf_destroy": (ctypes.c_int, [_vp]),
    "nmf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "nmf_last_error": (ctypes.c_char_p, []),
    "nmf_params_default": (None, [ctypes.POINTER(Params)]),
    "nmf_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "nmf_init_uniform": (ctypes.c_int, [_vp, _u64, _i32, _i64, _i64, _vp, _vp]),
    "nmf_objective": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i32, _i32, _dp, _vp]),
    "nmf_build_basis": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, ctypes.POINTER(Params), _vp, _vp,
                                       _vp, _vp, _dp, ctypes.POINTER(Report), _vp]),
    "nmf_project": (ctypes.c_int, [_vp, _vp, _i64, _i64, _vp, _vp, _i64, ctypes.POINTER(Params),
                                   _vp, _vp, _vp, ctypes.POINTER(Report), _vp]),
    "nmf_project_ragged": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _vp,
                                          ctypes.POINTER(Params), _vp, _vp, _vp,
                                          ctypes.POINTER(Report), _vp]),
    "nmf_device_clock_khz": (ctypes.c_double, [_vp]),
    "nmf_warm_fallbacks": (ctypes.c_int64, [_vp]),
    "nmf_frame_iters": (ctypes.c_int64, [_vp, _vp, _i64]),
    "nmf_frame_visits": (ctypes.c_int64, [_vp, _vp, _i64]),
    "nmf_subtract": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _vp]),
    "nmf_warmstart_param_count": (ctypes.c_int64, [_i32]),
    "nmf_warmstart_init": (ctypes.c_int, [_vp, _vp, _i32, _u64, _vp]),
    "nmf_warmstart_pool": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "nmf_warmstart_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32,
                                          ctypes.c_float, _i32, _vp, _dp, _vp]),
    "nmf_warmstart_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32,
                                           _i32, ctypes.c_float, _u64, _dp, _vp]),
    "nmf_warmstart_infer": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp]),
    "nmf_closest_frames": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp, _vp, _i64, _i64, _vp,
                                          _vp, _vp]),
    "nmf_closest_frames_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp, _vp, _i64,
                                                  _i64, _vp, _vp]),
    "nmf_best_factor": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64,
                                       ctypes.c_float, ctypes.c_float, _vp, _vp]),
    "nmf_build_basis_sequential": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, ctypes.POINTER(Params),
                                                  _vp, _vp, _dp, ctypes.POINTER(Report), _vp]),
    "nmf_autotune_report": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "nmf_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "nmf_profile_get": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]),
}

_lib = None
_lock = threading.Lock()


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions the public header declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"HIP library not built ({LIB_PATH}); run __graft_entry__.build()")
            l = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(l, name)
                fn.restype = res
                fn.argtypes = args
            _lib = l
    return _lib


def _check(status: int) -> int:
    if status < 0:
        msg = lib().nmf_last_error().decode(errors="replace")
        raise NmfError(status, msg)
    return status


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, dtype=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(device):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class Handle:
    """Owns a library handle (device workspace) on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().nmf_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().nmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return int(lib().nmf_workspace_bytes(self.h))


_handles: dict[int, Handle] = {}


def default_handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def make_params(k, iters, precision="fp32", seed=0, flags=0, eps=1e-30, split=0, tol=0.0,
                check_every=0, waves=0, pipeline=0) -> Params:
    p = Params()
    lib().nmf_params_default(ctypes.byref(p))
    p.k = int(k)
    p.max_iter = int(iters)
    p.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    p.seed = int(seed)
    p.flags = int(flags)
    p.floor_eps = float(eps)
    p.split = int(split)
    p.tol = float(tol)
    p.check_every = int(check_every)
    p.waves = int(waves)
    p.pipeline = int(pipeline)
    return p


def _new_report() -> Report:
    r = Report()
    r.struct_size = ctypes.sizeof(Report)
    return r


# ---------------------------------------------------------------------------

def init_uniform(seed: int, matrix_id: int, rows: int, cols: int, device: int = 0, handle=None):
    torch = _torch()
    h = handle or default_handle(device)
    out = torch.empty((rows, cols), dtype=torch.float32, device=f"cuda:{device}")
    _check(lib().nmf_init_uniform(h.h, seed, matrix_id, rows, cols, _dev_ptr(out, "out"),
                                  _stream(device)))
    return out


def objective(V, M, W, H, precision="fp32", handle=None) -> float:
    torch = _torch()
    dev = V.device.index or 0
    h = handle or default_handle(dev)
    n, p = V.shape
    k = W.shape[1]
    out = ctypes.c_double()
    f32 = torch.float32
    _check(lib().nmf_objective(h.h, _dev_ptr(V, "V", f32), _dev_ptr(M, "M", f32),
                               _dev_ptr(W, "W", f32), _dev_ptr(H, "H", f32), n, p, k,
                               PREC[precision], ctypes.addressof(out), _stream(dev)))
    return out.value


def build_basis(V, M, k, iters, *, precision="fp32", W_init=None, H_init=None, seed=0, flags=0,
                eps=1e-30, split=0, tol=0.0, check_every=0, waves=0, pipeline=0, warm=False,
                handle=None):
    """Basis construction (Eq. 3 iterated).  Returns (W, H, J history, report).
    ``warm=True``: (W_init, H_init) is a warm start kept only if its cost is
    not above the seeded cold start's."""
    if warm:
        flags |= F_WARM_START
    torch = _torch()
    dev = V.device.index or 0
    h = handle or default_handle(dev)
    n, p = V.shape
    f32 = torch.float32
    W = torch.empty((n, k), dtype=f32, device=V.device)
    H = torch.empty((k, p), dtype=f32, device=V.device)
    hist = np.zeros(iters + 1, np.float64)
    prm = make_params(k, iters, precision, seed, flags, eps, split, tol, check_every, waves,
                      pipeline)
    rep = _new_report()
    st = _check(lib().nmf_build_basis(
        h.h, _dev_ptr(V, "V", f32), _dev_ptr(M, "M", f32), n, p, ctypes.byref(prm),
        _dev_ptr(W_init, "W_init", f32), _dev_ptr(H_init, "H_init", f32), _dev_ptr(W, "W_out"),
        _dev_ptr(H, "H_out"), hist.ctypes.data, ctypes.byref(rep), _stream(dev)))
    info = rep.as_dict()
    info["status"] = st
    return W, H, hist[: rep.iters_run + 1], info


def project(H, T, MT, iters, *, C_init=None, precision="fp32", seed=0, flags=0, eps=1e-30,
            split=0, want_objective=False, gram=False, warm=False, tol=0.0, check_every=0,
            handle=None):
    """Target modelling: per-frame coefficients with the basis fixed
    (``gram=True``: through per-frame masked Gram matrices; ``warm=True``:
    C_init is a warm start with per-frame fallback to the cold start;
    ``tol``/``check_every``: per-frame stop rule of the Gram form, see
    frame_iters())."""
    if gram:
        flags |= F_MASKED_GRAM
    if warm:
        flags |= F_WARM_START
    torch = _torch()
    dev = H.device.index or 0
    h = handle or default_handle(dev)
    k, p = H.shape
    f = T.shape[0]
    f32 = torch.float32
    C = torch.empty((f, k), dtype=f32, device=H.device)
    obj = torch.empty(f, dtype=torch.float64, device=H.device) if want_objective else None
    prm = make_params(k, iters, precision, seed, flags, eps, split, tol, check_every)
    rep = _new_report()
    _check(lib().nmf_project(h.h, _dev_ptr(H, "H", f32), k, p, _dev_ptr(T, "T", f32),
                             _dev_ptr(MT, "M_T", f32), f, ctypes.byref(prm),
                             _dev_ptr(C_init, "C_init", f32), _dev_ptr(C, "C_out"),
                             _dev_ptr(obj, "obj_out"), ctypes.byref(rep), _stream(dev)))
    return (C, obj, rep.as_dict()) if want_objective else (C, rep.as_dict())


def subtract(H, C, T, MT, scale=None, want_model=True, handle=None):
    """Model PSF and residual frames (NaN at masked pixels)."""
    torch = _torch()
    dev = H.device.index or 0
    h = handle or default_handle(dev)
    k, p = H.shape
    f = T.shape[0]
    f32 = torch.float32
    resid = torch.empty((f, p), dtype=f32, device=H.device)
    model = torch.empty((f, p), dtype=f32, device=H.device) if want_model else None
    _check(lib().nmf_subtract(h.h, _dev_ptr(H, "H", f32), _dev_ptr(C, "C", f32),
                              _dev_ptr(T, "T", f32), _dev_ptr(MT, "M_T", f32), f, k, p,
                              _dev_ptr(scale, "scale", f32), _dev_ptr(model, "model_out"),
                              _dev_ptr(resid, "resid_out"), _stream(dev)))
    return model, resid


def closest_frames(V, M, T, MT, n_sel, want_dist=False, handle=None):
    """Reference selection: per target frame, the indices (int32, f x n_sel)
    of the n_sel library frames closest in the masked Euclidean norm, by
    increasing distance (ties by index); optionally the f x n FP64
    distances."""
    torch = _torch()
    dev = V.device.index or 0
    h = handle or default_handle(dev)
    n, p = V.shape
    f = T.shape[0]
    f32 = torch.float32
    idx = torch.empty((f, n_sel), dtype=torch.int32, device=V.device)
    dist = torch.empty((f, n), dtype=torch.float64, device=V.device) if want_dist else None
    _check(lib().nmf_closest_frames(h.h, _dev_ptr(V, "V", f32), _dev_ptr(M, "M", f32), n, p,
                                    _dev_ptr(T, "T", f32), _dev_ptr(MT, "M_T", f32), f, n_sel,
                                    _dev_ptr(dist, "dist_out"), _dev_ptr(idx, "idx_out"),
                                    _stream(dev)))
    return (idx, dist) if want_dist else idx


def closest_frames_noalloc(V, M, T, MT, n_sel, idx_out=None, handle=None):
    """The same selection through the allocation-free entry point (every
    intermediate in the library's fixed per-device scratch array); the
    caller may pass the output tensor."""
    torch = _torch()
    dev = V.device.index or 0
    h = handle or default_handle(dev)
    n, p = V.shape
    f = T.shape[0]
    f32 = torch.float32
    idx = idx_out if idx_out is not None else torch.empty((f, n_sel), dtype=torch.int32,
                                                          device=V.device)
    _check(lib().nmf_closest_frames_noalloc(h.h, _dev_ptr(V, "V", f32), _dev_ptr(M, "M", f32), n,
                                            p, _dev_ptr(T, "T", f32), _dev_ptr(MT, "M_T", f32), f,
                                            n_sel, _dev_ptr(idx, "idx_out", torch.int32),
                                            _stream(dev)))
    return idx


def best_factor(H, C, T, MT, region=None, s_lo=0.0, s_hi=float("inf"), handle=None):
    """Per-frame scale of the model PSF minimising the residual variance
    over the valid pixels (inside ``region`` when given), clamped."""
    torch = _torch()
    dev = H.device.index or 0
    h = handle or default_handle(dev)
    k, p = H.shape
    f = T.shape[0]
    f32 = torch.float32
    out = torch.empty(f, dtype=f32, device=H.device)
    _check(lib().nmf_best_factor(h.h, _dev_ptr(H, "H", f32), _dev_ptr(C, "C", f32),
                                 _dev_ptr(T, "T", f32), _dev_ptr(MT, "M_T", f32),
                                 _dev_ptr(region, "region", f32), f, k, p, s_lo, s_hi,
                                 _dev_ptr(out, "scale_out"), _stream(dev)))
    return out


def build_basis_sequential(V, M, k, iters, *, precision="fp32", seed=0, flags=0, eps=1e-30,
                           tol=0.0, check_every=0, handle=None):
    """Component-by-component basis construction: stages 1..k, each
    ``iters`` iterations from the previous components plus a new one.
    Returns (W, H, objective after each stage, report)."""
    torch = _torch()
    dev = V.device.index or 0
    h = handle or default_handle(dev)
    n, p = V.shape
    f32 = torch.float32
    W = torch.empty((n, k), dtype=f32, device=V.device)
    H = torch.empty((k, p), dtype=f32, device=V.device)
    stages = np.zeros(k, np.float64)
    prm = make_params(k, iters, precision, seed, flags, eps, 0, tol, check_every)
    rep = _new_report()
    st = _check(lib().nmf_build_basis_sequential(
        h.h, _dev_ptr(V, "V", f32), _dev_ptr(M, "M", f32), n, p, ctypes.byref(prm),
        _dev_ptr(W, "W_out"), _dev_ptr(H, "H_out"), stages.ctypes.data, ctypes.byref(rep),
        _stream(dev)))
    info = rep.as_dict()
    info["status"] = st
    return W, H, stages, info


def profile_enable(handle: Handle, on: bool = True):
    """Live kernel timing (HIP events around each launch) on or off."""
    _check(lib().nmf_profile_enable(handle.h, 1 if on else 0))


def profile_get(handle: Handle, kernel_class: int):
    """(launch count, summed device ms) of one kernel class."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().nmf_profile_get(handle.h, kernel_class, ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def project_ragged(H, offsets, pix, val, wt, iters, *, C_init=None, seed=0, flags=0, eps=1e-30,
                   want_ticks=False, warm=False, precision="fp32", tol=0.0, check_every=0,
                   handle=None):
    """Projection of CSR frames (one persistent launch, masked Gram form).
    offsets: int64 (f+1), pix: int32, val/wt: float32 (wt may be None)."""
    if warm:
        flags |= F_WARM_START
    torch = _torch()
    dev = H.device.index or 0
    h = handle or default_handle(dev)
    k, p = H.shape
    f = offsets.shape[0] - 1
    nnz = pix.shape[0]
    C = torch.empty((f, k), dtype=torch.float32, device=H.device)
    ticks = torch.zeros(2 * f, dtype=torch.int64, device=H.device) if want_ticks else None
    prm = make_params(k, iters, precision, seed, flags, eps, 0, tol, check_every)
    rep = _new_report()
    _check(lib().nmf_project_ragged(
        h.h, _dev_ptr(H, "H", torch.float32), k, p, f, _dev_ptr(offsets, "offsets", torch.int64),
        nnz, _dev_ptr(pix, "pix", torch.int32), _dev_ptr(val, "val", torch.float32),
        _dev_ptr(wt, "wt", torch.float32), ctypes.byref(prm), _dev_ptr(C_init, "C_init", torch.float32),
        _dev_ptr(C, "C_out"), _dev_ptr(ticks, "frame_ticks"), ctypes.byref(rep), _stream(dev)))
    return (C, ticks, rep.as_dict()) if want_ticks else (C, rep.as_dict())


def warm_fallbacks(handle=None, device=0) -> int:
    """Frames of the last warm-started projection that fell back to the cold
    start (-1 if none ran on the handle)."""
    h = handle or default_handle(device)
    return int(lib().nmf_warm_fallbacks(h.h))


def frame_iters(handle=None, device=0):
    """Iterations per frame of the last masked-Gram projection with a stop
    rule on the handle (int32 numpy array; None if it had none)."""
    import numpy as np
    h = handle or default_handle(device)
    n = _check(int(lib().nmf_frame_iters(h.h, None, 0)))
    if n == 0:
        return None
    buf = np.zeros(n, np.int32)
    _check(int(lib().nmf_frame_iters(h.h, buf.ctypes.data, n)))
    return buf


def frame_visits(handle=None, device=0):
    """How many times the last masked-Gram projection on the handle took each
    frame from its queue (int32 numpy array; None if none ran)."""
    import numpy as np
    h = handle or default_handle(device)
    n = _check(int(lib().nmf_frame_visits(h.h, None, 0)))
    if n == 0:
        return None
    buf = np.zeros(n, np.int32)
    _check(int(lib().nmf_frame_visits(h.h, buf.ctypes.data, n)))
    return buf


def device_clock_khz(handle=None, device=0) -> float:
    h = handle or default_handle(device)
    return float(lib().nmf_device_clock_khz(h.h))


# ---------------------------------------------------------------------------
# learned warm start
# ---------------------------------------------------------------------------
WS_IN, WS_HIDDEN = 1024, 512
WS_PREC = {"fp32": 0, "bf16x3": 1, "bf16": 2}
WS_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def ws_shapes(k):
    return [(WS_IN, WS_HIDDEN), (WS_HIDDEN,), (WS_HIDDEN, WS_HIDDEN), (WS_HIDDEN,), (WS_HIDDEN, k), (k,)]


def ws_param_count(k):
    return int(lib().nmf_warmstart_param_count(k))


def ws_state_from_params(params, k, device="cuda:0"):
    """Pack host parameters (dict of arrays) into a device state with zero
    Adam moments."""
    torch = _torch()
    flat = np.concatenate([np.asarray(params[n], np.float64).reshape(-1) for n in WS_NAMES])
    assert flat.size == ws_param_count(k)
    st = np.zeros(3 * flat.size, np.float32)
    st[: flat.size] = flat
    return torch.from_numpy(st).to(device)


def ws_unpack(vec, k):
    """Split a parameter-sized vector (state prefix or gradients) by name."""
    v = vec.detach().cpu().numpy().astype(np.float64) if hasattr(vec, "detach") else np.asarray(vec)
    out, o = {}, 0
    for n, shp in zip(WS_NAMES, ws_shapes(k)):
        c = int(np.prod(shp))
        out[n] = v[o:o + c].reshape(shp)
        o += c
    return out


def ws_init(k, seed=0, handle=None, device=0):
    torch = _torch()
    h = handle or default_handle(device)
    st = torch.empty(3 * ws_param_count(k), dtype=torch.float32, device=f"cuda:{device}")
    _check(lib().nmf_warmstart_init(h.h, st.data_ptr(), k, seed, _stream(device)))
    return st


def ws_pool(T, MT, ny, nx, handle=None):
    torch = _torch()
    dev = T.device.index or 0
    h = handle or default_handle(dev)
    f = T.shape[0]
    X = torch.empty((f, WS_IN), dtype=torch.float32, device=T.device)
    s = torch.empty(f, dtype=torch.float32, device=T.device)
    _check(lib().nmf_warmstart_pool(h.h, _dev_ptr(T, "T", torch.float32), _dev_ptr(MT, "M_T", torch.float32),
                                    f, ny, nx, X.data_ptr(), s.data_ptr(), _stream(dev)))
    return X, s


def ws_step(state, X, s, cstar, G, k, precision="fp32", lr=0.0, step=1, want_grads=False,
            handle=None):
    torch = _torch()
    dev = state.device.index or 0
    h = handle or default_handle(dev)
    b = X.shape[0]
    grads = torch.empty(ws_param_count(k), dtype=torch.float32, device=state.device) if want_grads else None
    loss = ctypes.c_double()
    f32 = torch.float32
    _check(lib().nmf_warmstart_step(h.h, _dev_ptr(state, "state", f32), _dev_ptr(X, "X", f32),
                                    _dev_ptr(s, "s", f32), _dev_ptr(cstar, "c_star", f32),
                                    _dev_ptr(G, "G", f32), b, k, WS_PREC[precision], lr, step,
                                    _dev_ptr(grads, "grads"), ctypes.addressof(loss), _stream(dev)))
    return (loss.value, grads) if want_grads else loss.value


def ws_train(state, X, s, cstar, G, k, epochs, batch, lr, seed=0, precision="fp32", handle=None):
    torch = _torch()
    dev = state.device.index or 0
    h = handle or default_handle(dev)
    hist = np.zeros(max(epochs, 1), np.float64)
    f32 = torch.float32
    _check(lib().nmf_warmstart_train(h.h, _dev_ptr(state, "state", f32), _dev_ptr(X, "X", f32),
                                     _dev_ptr(s, "s", f32), _dev_ptr(cstar, "c_star", f32),
                                     _dev_ptr(G, "G", f32), X.shape[0], k, WS_PREC[precision],
                                     epochs, batch, lr, seed, hist.ctypes.data, _stream(dev)))
    return hist[:epochs]


def ws_infer(state, X, s, k, precision="fp32", handle=None):
    torch = _torch()
    dev = state.device.index or 0
    h = handle or default_handle(dev)
    f = X.shape[0]
    C = torch.empty((f, k), dtype=torch.float32, device=state.device)
    f32 = torch.float32
    _check(lib().nmf_warmstart_infer(h.h, _dev_ptr(state, "state", f32), _dev_ptr(X, "X", f32),
                                     _dev_ptr(s, "s", f32), f, k, WS_PREC[precision], C.data_ptr(),
                                     _stream(dev)))
    return C


def autotune_report(handle: Handle) -> str:
    buf = ctypes.create_string_buffer(8192)
    _check(lib().nmf_autotune_report(handle.h, buf, 8192))
    return buf.value.decode()
