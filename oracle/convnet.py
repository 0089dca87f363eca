"""FP64 CPU oracle of the learned surrogate's convolutional network.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module; the product path never imports it.  It shares no code with the HIP kernels.

The network is not part of the paper's method: it is a learned shortcut over K steps of it,
trained on trajectories of the method.  Its definition, written out here in plain numpy:

  state s of shape [B, H, W, 4] (phi, v_x / u_scale, v_y / u_scale, (rho - 1) / rho_scale) on
  periodic boxes;
  tap t = 0..8 reads the input at (y + dy_t, x + dx_t) with dy_t = t // 3 - 1, dx_t = t % 3 - 1,
  indices taken modulo the box (circular padding);
  layer l:  z_l[p] = b_l + sum_t a_l[p + d_t] @ W_l[t]       (W_l[t] of shape [c_in, c_out])
  a_0 = s,  a_{l+1} = max(z_l, 0) for l < L - 1,  out = s + alpha * z_{L-1};
  loss = mean over pixels and the 4 channels of ((out - target) / alpha)^2,
with alpha a fixed per-channel output scale (the typical size of the state's change).

Layer 0 maps 4 -> C channels, the hidden layers C -> C and the last C -> 4.  The flat parameter
vector holds, layer after layer, W_l[t][ci][co] and then the bias padded to the kernels' output
width (C for hidden layers, 32 for the last; the padding entries carry no meaning and get zero
gradient).

With ``emulate_bf16`` the oracle rounds to bfloat16 (round to nearest even) exactly the operands
that the MFMA kernels hold in bfloat16: the weights of layers 1 .. L-1, each hidden activation,
the gradient of the output and each hidden gradient.  The first layer (state and weights) and
everything else (biases, the residual add, sums) stay FP64, as the kernels keep them in FP32.

Adam follows Kingma and Ba, "Adam: A method for stochastic optimization" (ICLR 2015), Algorithm 1,
with the bias corrections applied to the moments.
"""
from __future__ import annotations

import numpy as np

STATE_C = 4
LAST_BIAS_PAD = 32


def taps():
    """(dy, dx) of the nine taps, t = 3 (dy + 1) + (dx + 1)."""
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def layer_shapes(C: int, L: int):
    """(c_in, c_out, bias entries) of each layer."""
    out = []
    for l in range(L):
        cin = STATE_C if l == 0 else C
        cout = STATE_C if l == L - 1 else C
        out.append((cin, cout, LAST_BIAS_PAD if l == L - 1 else C))
    return out


def param_count(C: int, L: int) -> int:
    return sum(9 * ci * co + nb for ci, co, nb in layer_shapes(C, L))


def unpack(params: np.ndarray, C: int, L: int):
    """Flat vector -> list of (W [9, c_in, c_out], b [c_out])."""
    params = np.asarray(params, dtype=np.float64)
    assert params.shape == (param_count(C, L),)
    out, o = [], 0
    for ci, co, nb in layer_shapes(C, L):
        W = params[o:o + 9 * ci * co].reshape(9, ci, co)
        o += 9 * ci * co
        b = params[o:o + co]
        o += nb
        out.append((W, b))
    return out


def pack(layers, C: int, L: int) -> np.ndarray:
    """Inverse of ``unpack``: bias padding entries are written as zero."""
    parts = []
    for (W, b), (ci, co, nb) in zip(layers, layer_shapes(C, L)):
        parts.append(np.asarray(W, dtype=np.float64).reshape(-1))
        bb = np.zeros(nb)
        bb[:co] = b
        parts.append(bb)
    return np.concatenate(parts)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (8 significand bits, round to nearest, ties to even), via float32,
    returned as float64.  Inputs are finite."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shifted(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """r[:, y, x] = a[:, (y + dy) mod H, (x + dx) mod W]."""
    return np.roll(a, shift=(-dy, -dx), axis=(1, 2))


def conv(a: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One layer: z[p] = b + sum_t a[p + d_t] @ W[t]."""
    z = np.broadcast_to(b, a.shape[:3] + (W.shape[2],)).copy()
    for t, (dy, dx) in enumerate(taps()):
        z += shifted(a, dy, dx) @ W[t]
    return z


def forward(params, state, C: int, L: int, emulate_bf16: bool = False, alpha=(1.0,) * STATE_C):
    """Returns (out, cache); cache holds what ``backward`` needs."""
    rnd = bf16 if emulate_bf16 else (lambda v: v)
    s = np.asarray(state, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    layers = [(W if l == 0 else rnd(W), b) for l, (W, b) in enumerate(unpack(params, C, L))]
    acts = [s]
    z = None
    for l, (W, b) in enumerate(layers):
        z = conv(acts[l], W, b)
        if l < L - 1:
            acts.append(rnd(np.maximum(z, 0.0)))
    out = s + alpha * z
    return out, {"acts": acts, "layers": layers, "out": out, "emulate": emulate_bf16, "alpha": alpha}


def loss(out, target, alpha=(1.0,) * STATE_C) -> float:
    return float(np.mean(((np.asarray(out) - np.asarray(target)) / np.asarray(alpha, dtype=np.float64)) ** 2))


def backward(cache, target, C: int, L: int):
    """Gradient of ``loss`` with respect to the flat parameter vector, and the loss."""
    rnd = bf16 if cache["emulate"] else (lambda v: v)
    out, acts, layers, alpha = cache["out"], cache["acts"], cache["layers"], cache["alpha"]
    target = np.asarray(target, dtype=np.float64)
    g = rnd(2.0 * (out - target) / alpha / out.size)  # d loss / d z_{L-1}
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        a = acts[l]
        W, _ = layers[l]
        dW = np.empty_like(W)
        for t, (dy, dx) in enumerate(taps()):
            dW[t] = np.einsum("bhwi,bhwo->io", shifted(a, dy, dx), g)
        grads[l] = (dW, g.sum(axis=(0, 1, 2)))
        if l == 0:
            break
        da = np.zeros_like(a)
        for t, (dy, dx) in enumerate(taps()):
            da += shifted(g, -dy, -dx) @ W[t].T
        g = rnd(da * (a > 0))
    return pack(grads, C, L), loss(out, target, alpha)


def adam(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
