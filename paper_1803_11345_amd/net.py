"""Thin ctypes binding of the surrogate network and the hybrid driver (include/lbcm_net.h).

Argument marshalling only: the forward and backward passes, the optimiser, the state packing and
the hybrid's error checks run in the library's HIP kernels; PyTorch supplies device memory and
the stream.  The functions carry the C names; ``Surrogate`` and ``Hybrid`` bundle a handle.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import inputs, lbcm
from .lbcm import LBCM_OK, LbcmError

_H = ctypes.c_void_p
_F = ctypes.POINTER(ctypes.c_float)
_V = ctypes.c_void_p
_bound = False


class lbcm_hybrid_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("jumps", ctypes.c_int64), ("lb_steps_run", ctypes.c_int64),
                ("checks", ctypes.c_int64), ("failed_checks", ctypes.c_int64), ("last_error", ctypes.c_double),
                ("max_error", ctypes.c_double), ("last_velocity_error", ctypes.c_double),
                ("max_accepted_error", ctypes.c_double), ("max_accepted_velocity_error", ctypes.c_double),
                ("audits", ctypes.c_int64), ("failed_audits", ctypes.c_int64),
                ("max_audited_error", ctypes.c_double), ("max_audited_velocity_error", ctypes.c_double)]


def load():
    global _bound
    lib = lbcm.load()
    if _bound:
        return lib
    I32, D = ctypes.c_int32, ctypes.c_double
    lib.lbcm_net_create.argtypes = [I32, I32, I32, I32, I32, _V, ctypes.POINTER(_H)]
    lib.lbcm_net_param_count.argtypes = [_H]
    lib.lbcm_net_param_count.restype = ctypes.c_size_t
    lib.lbcm_net_set_output_scale.argtypes = [_H, _F]
    lib.lbcm_net_set_params.argtypes = [_H, _F, ctypes.c_size_t]
    lib.lbcm_net_get_params.argtypes = [_H, _F, ctypes.c_size_t]
    lib.lbcm_net_get_grads.argtypes = [_H, _F, ctypes.c_size_t]
    lib.lbcm_net_forward.argtypes = [_H, _V, _V]
    lib.lbcm_net_forward_planes.argtypes = [_H, _V, _V, _V, _V, D, D, _V, _V, _V, _V]
    lib.lbcm_net_state_from_planes.argtypes = [_H, _V, _V, _V, _V, D, D, _V]
    lib.lbcm_net_gather_states.argtypes = [_H, _V, ctypes.c_int64, ctypes.POINTER(I32), I32, D, D, _V]
    lib.lbcm_net_backward.argtypes = [_H, _V, _F]
    lib.lbcm_net_adam.argtypes = [_H, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int64]
    lib.lbcm_net_destroy.argtypes = [_H]
    lib.lbcm_net_last_error.argtypes = [_H]
    lib.lbcm_net_last_error.restype = ctypes.c_char_p
    lib.lbcm_hybrid_create.argtypes = [_H, _H, I32, I32, D, D, D, D, ctypes.POINTER(_H)]
    lib.lbcm_hybrid_advance.argtypes = [_H, ctypes.c_int64]
    lib.lbcm_hybrid_get_stats.argtypes = [_H, ctypes.POINTER(lbcm_hybrid_stats)]
    lib.lbcm_hybrid_set_audit.argtypes = [_H, ctypes.c_int32]
    lib.lbcm_hybrid_destroy.argtypes = [_H]
    lib.lbcm_hybrid_last_error.argtypes = [_H]
    lib.lbcm_hybrid_last_error.restype = ctypes.c_char_p
    _bound = True
    return lib


def _msg(m):
    return m.decode() if m else ""


def _nchk(n, rc):
    if rc != LBCM_OK:
        raise LbcmError(rc, _msg(load().lbcm_net_last_error(n)))


def _hchk(h, rc):
    if rc != LBCM_OK:
        raise LbcmError(rc, _msg(load().lbcm_hybrid_last_error(h)))


def _dev(t, dtype):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return _V(t.data_ptr())


def _host_f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != (n,):
        raise ValueError(f"expected {n} parameters")
    return a


# ---------------------------------------------------------------- C entry points

def lbcm_net_create(batch, height, width, channels, layers, stream):
    h = _H()
    rc = load().lbcm_net_create(batch, height, width, channels, layers, stream, ctypes.byref(h))
    _nchk(None, rc)
    return h


def lbcm_net_param_count(n) -> int:
    return load().lbcm_net_param_count(n)


STATE_C = 4  # (phi, v_x, v_y, rho)


def lbcm_net_set_output_scale(n, alpha):
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    if a.shape != (STATE_C,):
        raise ValueError(f"expected {STATE_C} output scales")
    _nchk(n, load().lbcm_net_set_output_scale(n, a.ctypes.data_as(_F)))


def lbcm_net_set_params(n, params):
    a = _host_f32(params, lbcm_net_param_count(n))
    _nchk(n, load().lbcm_net_set_params(n, a.ctypes.data_as(_F), a.size))


def lbcm_net_get_params(n) -> np.ndarray:
    a = np.empty(lbcm_net_param_count(n), dtype=np.float32)
    _nchk(n, load().lbcm_net_get_params(n, a.ctypes.data_as(_F), a.size))
    return a


def lbcm_net_get_grads(n) -> np.ndarray:
    a = np.empty(lbcm_net_param_count(n), dtype=np.float32)
    _nchk(n, load().lbcm_net_get_grads(n, a.ctypes.data_as(_F), a.size))
    return a


def lbcm_net_forward(n, state, out=None):
    import torch

    _nchk(n, load().lbcm_net_forward(n, _dev(state, torch.float32), None if out is None else _dev(out, torch.float32)))


def lbcm_net_forward_planes(n, phi, ux, uy, rho, u_scale, rho_scale, phi_out, ux_out, uy_out, rho_out):
    import torch

    d = torch.float64
    _nchk(n, load().lbcm_net_forward_planes(n, _dev(phi, d), _dev(ux, d), _dev(uy, d), _dev(rho, d), u_scale, rho_scale,
                                            _dev(phi_out, d), _dev(ux_out, d), _dev(uy_out, d), _dev(rho_out, d)))


def lbcm_net_state_from_planes(n, phi, ux, uy, rho, u_scale, rho_scale, state):
    import torch

    d = torch.float64
    _nchk(n, load().lbcm_net_state_from_planes(n, _dev(phi, d), _dev(ux, d), _dev(uy, d), _dev(rho, d), u_scale,
                                               rho_scale, _dev(state, torch.float32)))


def lbcm_net_gather_states(n, frames, frame_index, symmetry, u_scale, rho_scale, state):
    """frames: contiguous FP64 CUDA tensor [4, nframes, H, W]; frame_index: one int per sample."""
    import torch

    if frames.dim() != 4 or frames.shape[0] != 4:
        raise ValueError("frames must have the shape [4, nframes, H, W]")
    idx = np.ascontiguousarray(frame_index, dtype=np.int32)
    _nchk(n, load().lbcm_net_gather_states(n, _dev(frames, torch.float64), frames.shape[1],
                                           idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(symmetry), u_scale,
                                           rho_scale, _dev(state, torch.float32)))


def lbcm_net_backward(n, target, want_loss=True):
    import torch

    loss = ctypes.c_float()
    _nchk(n, load().lbcm_net_backward(n, _dev(target, torch.float32), ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def lbcm_net_adam(n, lr, beta1, beta2, eps, t):
    _nchk(n, load().lbcm_net_adam(n, lr, beta1, beta2, eps, t))


def lbcm_net_destroy(n):
    _nchk(None, load().lbcm_net_destroy(n))


def lbcm_net_last_error(n) -> str:
    return _msg(load().lbcm_net_last_error(n))


def lbcm_hybrid_create(lattice, net, steps_per_jump, jumps_per_check, u_scale, rho_scale, threshold,
                       velocity_threshold=0.0):
    h = _H()
    rc = load().lbcm_hybrid_create(lattice, net, steps_per_jump, jumps_per_check, u_scale, rho_scale, threshold,
                                   velocity_threshold, ctypes.byref(h))
    _hchk(None, rc)
    return h


def lbcm_hybrid_advance(h, windows):
    _hchk(h, load().lbcm_hybrid_advance(h, windows))


def lbcm_hybrid_set_audit(h, every: int):
    return _hchk(h, load().lbcm_hybrid_set_audit(h, int(every)))


def lbcm_hybrid_get_stats(h) -> dict:
    s = lbcm_hybrid_stats()
    _hchk(h, load().lbcm_hybrid_get_stats(h, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in lbcm_hybrid_stats._fields_}


def lbcm_hybrid_destroy(h):
    _hchk(None, load().lbcm_hybrid_destroy(h))


def lbcm_hybrid_last_error(h) -> str:
    return _msg(load().lbcm_hybrid_last_error(h))


# ---------------------------------------------------------------- convenience wrappers

def layer_shapes(channels: int, layers: int):
    """(c_in, c_out, bias entries) of each layer in the parameter vector."""
    out = []
    for l in range(layers):
        cin = STATE_C if l == 0 else channels
        cout = STATE_C if l == layers - 1 else channels
        out.append((cin, cout, 32 if l == layers - 1 else channels))
    return out


def initial_params(channels: int, layers: int, seed: int = 1) -> np.ndarray:
    """He-uniform weights, zero biases, and a zero last layer (the network starts as the identity
    map state -> state)."""
    shapes = []
    for l, (ci, co, nb) in enumerate(layer_shapes(channels, layers)):
        shapes.append((9 * ci, 9 * ci * co, l == layers - 1))
        shapes.append((1, nb, True))
    return inputs.he_uniform(seed, shapes).astype(np.float32)


class Surrogate:
    """A network for ``batch`` boxes of height x width on the current CUDA device."""

    def __init__(self, batch, height, width, *, channels=64, layers=6, stream=None):
        import torch

        self.batch, self.height, self.width = batch, height, width
        self.channels, self.layers = channels, layers
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = lbcm_net_create(batch, height, width, channels, layers, self.stream.cuda_stream)
        self.nparams = lbcm_net_param_count(self.h)
        self.t = 0
        self.alpha = (1.0,) * STATE_C

    def set_params(self, p):
        lbcm_net_set_params(self.h, p)
        self.t = 0

    def set_output_scale(self, alpha):
        lbcm_net_set_output_scale(self.h, alpha)
        self.alpha = tuple(float(a) for a in alpha)

    def params(self):
        return lbcm_net_get_params(self.h)

    def grads(self):
        return lbcm_net_get_grads(self.h)

    def forward(self, state, out=None):
        lbcm_net_forward(self.h, state, out)
        return out

    def forward_planes(self, phi, ux, uy, rho, u_scale, rho_scale, phi_out, ux_out, uy_out, rho_out):
        lbcm_net_forward_planes(self.h, phi, ux, uy, rho, u_scale, rho_scale, phi_out, ux_out, uy_out, rho_out)

    def state_from_planes(self, phi, ux, uy, rho, u_scale, rho_scale, state):
        lbcm_net_state_from_planes(self.h, phi, ux, uy, rho, u_scale, rho_scale, state)

    def gather_states(self, frames, frame_index, symmetry, u_scale, rho_scale, state):
        if len(frame_index) != self.batch:
            raise ValueError(f"expected {self.batch} frame indices")
        lbcm_net_gather_states(self.h, frames, frame_index, symmetry, u_scale, rho_scale, state)

    def backward(self, target, want_loss=True):
        return lbcm_net_backward(self.h, target, want_loss)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        lbcm_net_adam(self.h, lr, beta1, beta2, eps, self.t)

    def close(self):
        if self.h is not None:
            lbcm_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hybrid:
    """Surrogate jumps on a periodic lattice with a lattice Boltzmann check every
    ``jumps_per_check`` jumps (see lbcm_hybrid_create)."""

    def __init__(self, lattice, net: Surrogate, *, steps_per_jump=16, jumps_per_check=8, u_scale=1.0, rho_scale=1.0,
                 threshold=1e-2, velocity_threshold=0.0, audit_every=0):
        self.lattice, self.net = lattice, net
        self.span = steps_per_jump * jumps_per_check
        self.h = lbcm_hybrid_create(lattice.h, net.h, steps_per_jump, jumps_per_check, u_scale, rho_scale, threshold,
                                    velocity_threshold)
        if audit_every:
            lbcm_hybrid_set_audit(self.h, audit_every)

    def advance(self, windows=1):
        lbcm_hybrid_advance(self.h, windows)
        return self

    def stats(self):
        return lbcm_hybrid_get_stats(self.h)

    def close(self):
        if self.h is not None:
            lbcm_hybrid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
