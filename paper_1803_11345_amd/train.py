"""Training data and training loop of the learned surrogate.

The data are trajectories of the lattice Boltzmann step itself (liblbcm.so), recorded every K
steps as FP64 device planes (phi, v_x, v_y): spinodal decomposition from small random phi and the
coalescence of two droplets.  Training pairs are (state, state K steps later) of one trajectory.
The forward pass, backward pass and Adam update are the library's kernels (net.Surrogate); torch
only gathers minibatches and applies the symmetries of the square lattice to them.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, lbcm
from .net import Surrogate

# free-energy and transport constants of the surrogate's workload: those of the spinodal
# decomposition runs (a, gamma, mobility, equal viscosities)
PHYSICS = dict(a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)


def spinodal_phi(n: int, seed: int) -> np.ndarray:
    return inputs.spinodal(n, n, seed=seed, amplitude=0.05)


def coalescence_phi(n: int, case) -> np.ndarray:
    r1, r2, gap = case
    return inputs.two_droplets(n, n, r1, r2, gap, inputs.interface_width(PHYSICS["a"], PHYSICS["gamma"]))


def record(phi0: np.ndarray, frames, start: int, count: int, K: int, warm: int = 0, stream=None):
    """Run the FP32 lattice from phi0 (v = 0), skip ``warm`` steps, then store ``count`` states
    K steps apart into frames[:, start:start + count] (frames: FP64 CUDA tensor [3, N, n, n])."""
    n = phi0.shape[0]
    lat = lbcm.Lattice(n, n, precision="fp32", stream=stream, **PHYSICS)
    lat.init(phi0)
    if warm:
        lat.step(warm)
    for i in range(count):
        if i:
            lat.step(K)
        lbcm.lbcm_fields_device(lat.h, frames[0, start + i], None, frames[1, start + i], frames[2, start + i], None)
    lat.close()


def build_dataset(n: int, K: int, runs, frames_per_run: int, device="cuda"):
    """runs: list of (phi0, warm steps).  Returns (frames [3, N, n, n] FP64, pairs [M, 2])."""
    import torch

    N = len(runs) * frames_per_run
    frames = torch.empty(3, N, n, n, dtype=torch.float64, device=device)
    pairs = []
    for r, (phi0, warm) in enumerate(runs):
        s = r * frames_per_run
        record(phi0, frames, s, frames_per_run, K, warm)
        pairs += [(s + i, s + i + 1) for i in range(frames_per_run - 1)]
    torch.cuda.synchronize()
    return frames, np.asarray(pairs, dtype=np.int64)


def velocity_scale(frames) -> float:
    """RMS of the velocity over the data set (the network sees v / u_scale)."""
    import torch

    return float(torch.sqrt((frames[1] ** 2 + frames[2] ** 2).mean() / 2).item())


def output_scale(frames, pairs, u_scale: float, sample: int = 256, seed: int = 3):
    """Per-channel RMS of the change over one pair (phi, v_x / u_scale, v_y / u_scale), on up to
    ``sample`` pairs: the network's output scale, so that each channel's residual is O(1)."""
    import torch

    idx = (inputs.splitmix64(seed, min(sample, len(pairs))) % np.uint64(len(pairs))).astype(np.int64)
    sel = torch.from_numpy(pairs[idx]).to(frames.device)
    d = frames[:, sel[:, 1]] - frames[:, sel[:, 0]]
    rms = torch.sqrt((d ** 2).mean(dim=(1, 2, 3))).cpu().numpy()
    rms[1:] /= u_scale
    return tuple(float(max(r, 1e-12)) for r in rms)


def dihedral(planes, k: int):
    """Element k (0..7) of the symmetry group of the square lattice applied to (phi, vx, vy)
    planes of shape [B, n, n]: optional transpose, then optional flips of y and of x."""
    phi, vx, vy = planes
    if k & 4:
        phi, vx, vy = phi.transpose(1, 2), vy.transpose(1, 2), vx.transpose(1, 2)
    if k & 2:
        phi, vx, vy = phi.flip(1), vx.flip(1), -vy.flip(1)
    if k & 1:
        phi, vx, vy = phi.flip(2), -vx.flip(2), vy.flip(2)
    return [p.contiguous() for p in (phi, vx, vy)]


def lr_at(it: int, iters: int, lr: float, warmup: int = 100, floor: float = 0.02) -> float:
    """Linear warm-up, then cosine decay to floor * lr."""
    if it < warmup:
        return lr * (it + 1) / warmup
    q = (it - warmup) / max(1, iters - warmup)
    return lr * (floor + (1 - floor) * 0.5 * (1 + math.cos(math.pi * q)))


def train(model: Surrogate, frames, pairs, u_scale: float, iters: int, lr: float = 1e-3, seed: int = 5,
          log_every: int = 100, augment: bool = True, log=None):
    """Adam on minibatches of model.batch pairs drawn with SplitMix64(seed).  Returns the list of
    (iteration, loss) logged and the seconds spent."""
    import torch

    B, n = model.batch, model.height
    xin = torch.empty(B, n, n, 3, dtype=torch.float32, device=frames.device)
    tgt = torch.empty_like(xin)
    draws = (inputs.splitmix64(seed, iters * (B + 1)) % np.uint64(len(pairs) * 8)).astype(np.int64)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        d = draws[it * (B + 1):(it + 1) * (B + 1)]
        sel = torch.from_numpy(pairs[d[:B] // 8]).to(frames.device)
        k = int(d[B] % 8) if augment else 0
        a = dihedral([frames[c].index_select(0, sel[:, 0]) for c in range(3)], k)
        b = dihedral([frames[c].index_select(0, sel[:, 1]) for c in range(3)], k)
        model.state_from_planes(a[0], a[1], a[2], u_scale, xin)
        model.state_from_planes(b[0], b[1], b[2], u_scale, tgt)
        model.forward(xin)
        want = log_every and (it % log_every == 0 or it == iters - 1)
        loss = model.backward(tgt, want_loss=bool(want))
        model.adam(lr_at(it, iters, lr))
        if want:
            hist.append((it, loss))
            if log:
                log(f"iter {it} loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def jump_errors(model: Surrogate, frames, pairs, u_scale: float):
    """Relative phi L2 error of one surrogate jump and of persistence (phi unchanged) on each
    pair; model has batch 1.  Returns two arrays."""
    import torch

    n = model.height
    outs = [torch.empty(n, n, dtype=torch.float64, device=frames.device) for _ in range(3)]
    e_net, e_keep = [], []
    for i0, i1 in pairs:
        model.forward_planes(frames[0, i0], frames[1, i0], frames[2, i0], u_scale, *outs)
        ref = frames[0, i1]
        nr = torch.linalg.vector_norm(ref).item()
        e_net.append(torch.linalg.vector_norm(outs[0] - ref).item() / nr)
        e_keep.append(torch.linalg.vector_norm(frames[0, i0] - ref).item() / nr)
    return np.asarray(e_net), np.asarray(e_keep)
