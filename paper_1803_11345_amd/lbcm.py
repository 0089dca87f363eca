"""Thin ctypes binding of liblbcm.so (declared in include/lbcm.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in the library's HIP
kernels.  PyTorch supplies device memory (an optional workspace tensor) and the HIP stream.
The functions carry the C names; ``Lattice`` bundles a handle with its workspace.

There is no fallback: if liblbcm.so has not been built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbcm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbcm.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(HERE), "include", "lbcm_net.h")]

LBCM_OK, LBCM_EINVAL, LBCM_ENOMEM, LBCM_EHIP, LBCM_EDIVERGED, LBCM_ESTATE = 0, -1, -2, -3, -4, -5
LBCM_BC_PERIODIC, LBCM_BC_WALLS = 0, 1
LBCM_FP64, LBCM_FP32, LBCM_FP16_SHIFTED, LBCM_BF16_SHIFTED = 0, 1, 2, 3
PRECISIONS = {"fp64": LBCM_FP64, "fp32": LBCM_FP32, "fp16s": LBCM_FP16_SHIFTED, "bf16s": LBCM_BF16_SHIFTED}
_ERRNAMES = {LBCM_EINVAL: "LBCM_EINVAL", LBCM_ENOMEM: "LBCM_ENOMEM", LBCM_EHIP: "LBCM_EHIP",
             LBCM_EDIVERGED: "LBCM_EDIVERGED", LBCM_ESTATE: "LBCM_ESTATE"}


class LbcmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class lbcm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("a", ctypes.c_double), ("gamma", ctypes.c_double), ("mobility", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double),
        ("omega3", ctypes.c_double), ("force_x", ctypes.c_double), ("force_y", ctypes.c_double),
        ("wall_vx_bottom", ctypes.c_double), ("wall_vx_top", ctypes.c_double), ("wall_gradient", ctypes.c_double),
        ("k8_variant", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32), ("tile_wx", ctypes.c_int32),
        ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class lbcm_diagnostics(ctypes.Structure):
    _fields_ = [
        ("sum_phi", ctypes.c_double), ("sum_abs_phi", ctypes.c_double), ("sum_rho", ctypes.c_double),
        ("sum_jx", ctypes.c_double), ("sum_jy", ctypes.c_double), ("max_u", ctypes.c_double),
        ("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64), ("max_du", ctypes.c_double),
    ]


def make_params(nx, ny, *, bc_y=0, precision="fp32", a=0.04, gamma=0.08, mobility=0.1, Gamma=1.0,
                nu_l=1 / 6, nu_g=1 / 6, omega3=1.0, force_x=0.0, force_y=0.0, wall_vx_bottom=0.0,
                wall_vx_top=0.0, wall_gradient=0.0, k8_variant=0,
                check_every=0, tile_rows=0, tile_wx=0, stream=None, workspace=None, workspace_bytes=0):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return lbcm_params(nx=nx, ny=ny, bc_y=bc_y, precision=precision, a=a, gamma=gamma,
                       mobility=mobility, Gamma=Gamma, nu_l=nu_l, nu_g=nu_g, omega3=omega3,
                       force_x=force_x, force_y=force_y, wall_vx_bottom=wall_vx_bottom,
                       wall_vx_top=wall_vx_top, wall_gradient=wall_gradient, k8_variant=k8_variant,
                       check_every=check_every, tile_rows=tile_rows, tile_wx=tile_wx,
                       stream=stream, workspace=workspace, workspace_bytes=workspace_bytes)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p


def load():
    """Load liblbcm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1803_11345_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lbcm_params)
    lib.lbcm_workspace_size.argtypes = [P]
    lib.lbcm_workspace_size.restype = ctypes.c_size_t
    lib.lbcm_create.argtypes = [P, ctypes.POINTER(_H)]
    lib.lbcm_init.argtypes = [_H, _D, _D, _D, _D]
    lib.lbcm_init_device.argtypes = [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.lbcm_step.argtypes = [_H, ctypes.c_int64]
    lib.lbcm_fields.argtypes = [_H, _D, _D, _D, _D, _D]
    lib.lbcm_fields_device.argtypes = [_H] + [ctypes.c_void_p] * 5
    lib.lbcm_populations.argtypes = [_H, _D, _D]
    lib.lbcm_diag.argtypes = [_H, ctypes.POINTER(lbcm_diagnostics)]
    lib.lbcm_stream_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    lib.lbcm_diag_state.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(lbcm_diagnostics)]
    lib.lbcm_state_size.argtypes = [_H]
    lib.lbcm_state_size.restype = ctypes.c_size_t
    lib.lbcm_get_state.argtypes = [_H, ctypes.c_void_p, ctypes.c_size_t]
    lib.lbcm_set_state.argtypes = [_H, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64]
    lib.lbcm_destroy.argtypes = [_H]
    lib.lbcm_last_error.argtypes = [_H]
    lib.lbcm_last_error.restype = ctypes.c_char_p
    I32 = ctypes.c_int32
    PI = ctypes.POINTER(ctypes.c_int32)
    lib.lbcm_autotune.argtypes = [_H, ctypes.c_int]
    lib.lbcm_tile_shape.argtypes = [_H, PI, PI]
    lib.lbcm_tile_rows_per_wave.argtypes = [_H, PI]
    lib.lbcm_info.argtypes = [_H, P]
    lib.lbcm_copy_state.argtypes = [_H, _H, ctypes.c_int64]
    lib.lbcm_step_count.argtypes = [_H]
    lib.lbcm_step_count.restype = ctypes.c_int64
    lib.lbcm_batch_create.argtypes = [P, I32, ctypes.POINTER(_H)]
    lib.lbcm_batch_box.argtypes = [_H, I32]
    lib.lbcm_batch_box.restype = _H
    lib.lbcm_batch_step.argtypes = [_H, ctypes.c_int64]
    lib.lbcm_batch_step_looped.argtypes = [_H, ctypes.c_int64]
    lib.lbcm_batch_step_looped_streams.argtypes = [_H, ctypes.c_int64, ctypes.c_int32]
    lib.lbcm_batch_autotune.argtypes = [_H, I32]
    lib.lbcm_batch_set_graph.argtypes = [_H, I32]
    lib.lbcm_batch_set_order.argtypes = [_H, I32]
    lib.lbcm_batch_set_persistent.argtypes = [_H, I32]
    lib.lbcm_batch_info.argtypes = [_H, PI, PI, PI, PI, PI]
    lib.lbcm_batch_destroy.argtypes = [_H]
    lib.lbcm_batch_last_error.argtypes = [_H]
    lib.lbcm_batch_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def declared_functions() -> list[str]:
    """Names of the entry points declared in include/lbcm.h and include/lbcm_net.h."""
    text = "\n".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|size_t|const char \*|lbcm_handle \*)\s*\**\s*(lbcm_\w+)\s*\(",
                                 text, re.M)))


def _check(h, rc):
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_last_error(h))
    return rc


def _dptr(a):
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError("expected a C-contiguous float64 numpy array")
    return a.ctypes.data_as(_D)


def _tptr(t):
    if t is None:
        return None
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- C entry points

def lbcm_workspace_size(params: lbcm_params) -> int:
    return load().lbcm_workspace_size(ctypes.byref(params))


def lbcm_create(params: lbcm_params):
    h = _H()
    rc = load().lbcm_create(ctypes.byref(params), ctypes.byref(h))
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_last_error(None))
    return h


def lbcm_init(h, phi0, rho0=None, ux0=None, uy0=None):
    return _check(h, load().lbcm_init(h, _dptr(phi0), _dptr(rho0), _dptr(ux0), _dptr(uy0)))


def lbcm_init_device(h, phi0, rho0=None, ux0=None, uy0=None):
    return _check(h, load().lbcm_init_device(h, _tptr(phi0), _tptr(rho0), _tptr(ux0), _tptr(uy0)))


def lbcm_step(h, nsteps: int = 1):
    return _check(h, load().lbcm_step(h, int(nsteps)))


def lbcm_fields(h, phi=None, rho=None, ux=None, uy=None, p0=None):
    return _check(h, load().lbcm_fields(h, _dptr(phi), _dptr(rho), _dptr(ux), _dptr(uy), _dptr(p0)))


def lbcm_fields_device(h, phi=None, rho=None, ux=None, uy=None, p0=None):
    return _check(h, load().lbcm_fields_device(h, _tptr(phi), _tptr(rho), _tptr(ux), _tptr(uy), _tptr(p0)))


def lbcm_populations(h, f=None, g=None):
    return _check(h, load().lbcm_populations(h, _dptr(f), _dptr(g)))


def lbcm_diag(h) -> dict:
    d = lbcm_diagnostics()
    _check(h, load().lbcm_diag(h, ctypes.byref(d)))
    return {name: getattr(d, name) for name, _ in lbcm_diagnostics._fields_}


def lbcm_stream_probe(src, dst, n: int, planes: int = 18, reps: int = 20, stream=None) -> float:
    """Milliseconds per launch of the library's streaming reference (src, dst: CUDA tensors of
    planes * n float32)."""
    ms = ctypes.c_float()
    rc = load().lbcm_stream_probe(src.data_ptr(), dst.data_ptr(), int(n), int(planes), int(reps), stream,
                                  ctypes.byref(ms))
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_last_error(None))
    return ms.value


def lbcm_diag_state(params: lbcm_params, f, g, f_prev=None, step: int = 0) -> dict:
    """Diagnostics of a state in caller device memory (f, g, f_prev: CUDA tensors or raw device
    addresses); allocation-free."""
    def addr(t):
        if t is None or isinstance(t, int):
            return t
        if not t.is_cuda or not t.is_contiguous():
            raise TypeError("expected a contiguous CUDA tensor")
        return t.data_ptr()

    d = lbcm_diagnostics()
    rc = load().lbcm_diag_state(ctypes.byref(params), addr(f), addr(g), addr(f_prev), int(step), ctypes.byref(d))
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_last_error(None))
    return {name: getattr(d, name) for name, _ in lbcm_diagnostics._fields_}


def lbcm_state_size(h) -> int:
    return load().lbcm_state_size(h)


def lbcm_get_state(h, buf: np.ndarray):
    return _check(h, load().lbcm_get_state(h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))


def lbcm_set_state(h, buf: np.ndarray, step: int = 0):
    return _check(h, load().lbcm_set_state(h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes, int(step)))


def lbcm_destroy(h):
    return _check(None, load().lbcm_destroy(h))


def lbcm_last_error(h) -> str:
    m = load().lbcm_last_error(h)
    return m.decode() if m else ""


def lbcm_autotune(h, trials: int = 5):
    return _check(h, load().lbcm_autotune(h, int(trials)))


def lbcm_info(h) -> lbcm_params:
    p = lbcm_params()
    _check(h, load().lbcm_info(h, ctypes.byref(p)))
    return p


def lbcm_copy_state(dst, src, step: int):
    _check(dst, load().lbcm_copy_state(dst, src, step))


def lbcm_step_count(h) -> int:
    return load().lbcm_step_count(h)


def lbcm_tile_shape(h):
    wx, rows = ctypes.c_int32(), ctypes.c_int32()
    _check(h, load().lbcm_tile_shape(h, ctypes.byref(wx), ctypes.byref(rows)))
    return wx.value, rows.value


def lbcm_tile_rows_per_wave(h):
    rpw = ctypes.c_int32()
    _check(h, load().lbcm_tile_rows_per_wave(h, ctypes.byref(rpw)))
    return rpw.value


def _bcheck(b, rc):
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_batch_last_error(b))
    return rc


def lbcm_batch_create(params_list):
    arr = (lbcm_params * len(params_list))(*params_list)
    b = _H()
    rc = load().lbcm_batch_create(arr, len(params_list), ctypes.byref(b))
    if rc != LBCM_OK:
        raise LbcmError(rc, lbcm_batch_last_error(None))
    return b


def lbcm_batch_box(b, i: int):
    h = load().lbcm_batch_box(b, int(i))
    if not h:
        raise IndexError(i)
    return _H(h)


def lbcm_batch_step(b, nsteps: int = 1):
    return _bcheck(b, load().lbcm_batch_step(b, int(nsteps)))


def lbcm_batch_step_looped(b, nsteps: int = 1):
    return _bcheck(b, load().lbcm_batch_step_looped(b, int(nsteps)))


def lbcm_batch_step_looped_streams(b, nsteps: int = 1, nstreams: int = 4):
    return _bcheck(b, load().lbcm_batch_step_looped_streams(b, int(nsteps), int(nstreams)))


def lbcm_batch_autotune(b, trials: int = 5):
    return _bcheck(b, load().lbcm_batch_autotune(b, int(trials)))


def lbcm_batch_set_graph(b, enable: bool):
    return _bcheck(b, load().lbcm_batch_set_graph(b, int(bool(enable))))


def lbcm_batch_set_persistent(b, mode: int):
    return _bcheck(b, load().lbcm_batch_set_persistent(b, int(mode)))


def lbcm_batch_set_order(b, order: int):
    return _bcheck(b, load().lbcm_batch_set_order(b, int(order)))


def lbcm_batch_info(b, nboxes: int) -> dict:
    waves, order, ntiles = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    wx = (ctypes.c_int32 * nboxes)()
    rows = (ctypes.c_int32 * nboxes)()
    _bcheck(b, load().lbcm_batch_info(b, ctypes.byref(waves), ctypes.byref(order), ctypes.byref(ntiles), wx, rows))
    return {"waves": waves.value, "order": order.value, "ntiles": ntiles.value, "wx": list(wx), "rows": list(rows)}


def lbcm_batch_destroy(b):
    return _bcheck(None, load().lbcm_batch_destroy(b))


def lbcm_batch_last_error(b) -> str:
    m = load().lbcm_batch_last_error(b)
    return m.decode() if m else ""


# ---------------------------------------------------------------- convenience wrappers

class _View:
    """Host-side operations on one lattice handle (own or inside a batch)."""

    h = None
    nx = ny = 0

    def init(self, phi0, rho0=None, ux0=None, uy0=None):
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (phi0, rho0, ux0, uy0)]
        for a in arr:
            if a is not None and a.shape != (self.ny, self.nx):
                raise ValueError(f"planes must have shape {(self.ny, self.nx)}")
        lbcm_init(self.h, *arr)
        return self

    def step(self, n=1):
        lbcm_step(self.h, n)
        return self

    def fields(self) -> dict:
        out = {k: np.empty((self.ny, self.nx)) for k in ("phi", "rho", "ux", "uy", "p0")}
        lbcm_fields(self.h, out["phi"], out["rho"], out["ux"], out["uy"], out["p0"])
        return out

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((9, self.ny, self.nx))
        lbcm_populations(self.h, f, g)
        return f, g

    def diag(self) -> dict:
        return lbcm_diag(self.h)

    def get_state(self) -> np.ndarray:
        buf = np.empty(lbcm_state_size(self.h), dtype=np.uint8)
        lbcm_get_state(self.h, buf)
        return buf

    def set_state(self, buf, step=0):
        lbcm_set_state(self.h, np.ascontiguousarray(buf, dtype=np.uint8), step)

    def autotune(self, trials=5):
        lbcm_autotune(self.h, trials)
        return lbcm_tile_shape(self.h)

    def tile_shape(self):
        return lbcm_tile_shape(self.h)

    def rows_per_wave(self):
        return lbcm_tile_rows_per_wave(self.h)


class Batch:
    """An ensemble of boxes advanced by one launch per step.  ``boxes`` is a list of dicts of
    make_params keywords (nx, ny and any physics); precision and stream are shared."""

    class Box(_View):
        def __init__(self, h, nx, ny):
            self.h, self.nx, self.ny = h, nx, ny

    def __init__(self, boxes, *, precision="fp32", stream=None):
        import torch

        # a stream of its own (the null stream cannot be captured into a graph)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        plist = [make_params(precision=precision, stream=self.stream.cuda_stream, **kw) for kw in boxes]
        self.b = lbcm_batch_create(plist)
        self.boxes = [Batch.Box(lbcm_batch_box(self.b, i), p.nx, p.ny) for i, p in enumerate(plist)]

    def __len__(self):
        return len(self.boxes)

    def __getitem__(self, i):
        return self.boxes[i]

    def step(self, n=1):
        lbcm_batch_step(self.b, n)
        return self

    def step_looped(self, n=1):
        lbcm_batch_step_looped(self.b, n)
        return self

    def step_looped_streams(self, n=1, nstreams=4):
        lbcm_batch_step_looped_streams(self.b, n, nstreams)
        return self

    def autotune(self, trials=5):
        lbcm_batch_autotune(self.b, trials)
        return self.info()

    def set_graph(self, enable):
        lbcm_batch_set_graph(self.b, enable)

    def set_order(self, order):
        lbcm_batch_set_order(self.b, order)

    def set_persistent(self, mode):
        lbcm_batch_set_persistent(self.b, mode)

    def info(self):
        return lbcm_batch_info(self.b, len(self.boxes))

    def close(self):
        if self.b is not None:
            lbcm_batch_destroy(self.b)
            self.b = None
            self.boxes = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice(_View):
    """One lattice on the current CUDA device.  The workspace is a torch uint8 tensor and work
    is queued on ``stream`` (default: torch's current stream)."""

    def __init__(self, nx, ny, *, stream=None, own_workspace=True, **kw):
        import torch

        self.nx, self.ny = nx, ny
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.params = make_params(nx, ny, stream=self.stream.cuda_stream, **kw)
        self.workspace = None
        if own_workspace:
            nbytes = lbcm_workspace_size(self.params)
            if nbytes == 0:
                raise LbcmError(LBCM_EINVAL, "invalid parameters")
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self.params.workspace = self.workspace.data_ptr()
            self.params.workspace_bytes = nbytes
        self.h = lbcm_create(self.params)

    def close(self):
        if self.h is not None:
            lbcm_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
