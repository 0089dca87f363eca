"""Training data and training loop of the learned surrogate.

The data are trajectories of the lattice Boltzmann step itself (liblbcm.so), recorded every K
steps as FP64 device planes (phi, v_x, v_y, rho): spinodal decomposition from small random phi and
the coalescence of two droplets.  Training pairs are (state, state K steps later) of one trajectory.
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
    K steps apart into frames[:, start:start + count] (frames: FP64 CUDA tensor [4, N, n, n] of
    phi, v_x, v_y, rho)."""
    n = phi0.shape[0]
    lat = lbcm.Lattice(n, n, precision="fp32", stream=stream, **PHYSICS)
    lat.init(phi0)
    if warm:
        lat.step(warm)
    for i in range(count):
        if i:
            lat.step(K)
        lbcm.lbcm_fields_device(lat.h, frames[0, start + i], frames[3, start + i], frames[1, start + i],
                                frames[2, start + i], None)
    lat.close()


def build_dataset(n: int, K: int, runs, frames_per_run: int, device="cuda"):
    """runs: list of (phi0, warm steps).  Returns (frames [4, N, n, n] FP64, pairs [M, 2])."""
    import torch

    N = len(runs) * frames_per_run
    frames = torch.empty(4, N, n, n, dtype=torch.float64, device=device)
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


def density_scale(frames) -> float:
    """RMS of rho - 1 over the data set (the network sees (rho - 1) / rho_scale)."""
    import torch

    return float(torch.sqrt(((frames[3] - 1.0) ** 2).mean()).item())


def output_scale(frames, pairs, u_scale: float, rho_scale: float, sample: int = 256, seed: int = 3):
    """Per-channel RMS of the change over one pair (phi, v_x / u_scale, v_y / u_scale,
    rho / rho_scale), on up to ``sample`` pairs: the network's output scale, so that each channel's
    residual is O(1)."""
    import torch

    idx = (inputs.splitmix64(seed, min(sample, len(pairs))) % np.uint64(len(pairs))).astype(np.int64)
    sel = torch.from_numpy(pairs[idx]).to(frames.device)
    d = frames[:, sel[:, 1]] - frames[:, sel[:, 0]]
    rms = torch.sqrt((d ** 2).mean(dim=(1, 2, 3))).cpu().numpy()
    rms[1:3] /= u_scale
    rms[3] /= rho_scale
    return tuple(float(max(r, 1e-12)) for r in rms)


def lr_at(it: int, iters: int, lr: float, warmup: int = 100, floor: float = 0.02) -> float:
    """Linear warm-up, then cosine decay to floor * lr."""
    if it < warmup:
        return lr * (it + 1) / warmup
    q = (it - warmup) / max(1, iters - warmup)
    return lr * (floor + (1 - floor) * 0.5 * (1 + math.cos(math.pi * q)))


def train(model: Surrogate, frames, pairs, u_scale: float, rho_scale: float, iters: int, lr: float = 1e-3, seed: int = 5,
          log_every: int = 100, augment: bool = True, noise: float = 0.0, pushforward: int = 0,
          frames_per_run: int = 0, log=None):
    """Adam on minibatches of model.batch pairs drawn with SplitMix64(seed).  With ``noise`` > 0
    the input state (not the target) gets Gaussian noise of noise * alpha_c per channel.  With
    ``pushforward`` = m > 0, iteration i first advances the input by i % (m + 1) jumps of the
    network itself (no gradient through them) and takes the target that many jumps further on, so
    that the network learns to correct the errors of its own rollouts (the pushforward trick of
    Brandstetter, Worrall and Welling, ICLR 2022); pairs then index frames of runs of
    ``frames_per_run`` consecutive frames.  Returns the list of (iteration, loss) logged and the
    seconds spent."""
    import torch

    B, n = model.batch, model.height
    xin = torch.empty(B, n, n, 4, dtype=torch.float32, device=frames.device)
    tgt = torch.empty_like(xin)
    gen = torch.Generator(device=frames.device)
    gen.manual_seed(seed)
    sigma = torch.tensor([noise * a for a in model.alpha], dtype=torch.float32, device=frames.device)
    draws = (inputs.splitmix64(seed, iters * (B + 1)) % np.uint64(len(pairs) * 8)).astype(np.int64)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        d = draws[it * (B + 1):(it + 1) * (B + 1)]
        sel = pairs[d[:B] // 8].copy()
        m = it % (pushforward + 1) if pushforward else 0
        if m:
            # keep start + m + 1 inside the run: pull starts back where needed
            fpr = frames_per_run
            room = fpr - 1 - (sel[:, 0] % fpr)
            shift = np.maximum(0, m + 1 - room)
            sel[:, 0] -= shift
            sel[:, 1] = sel[:, 0] + m + 1
        k = int(d[B] % 8) if augment else 0  # one of the 8 symmetries of the square for the batch
        model.gather_states(frames, sel[:, 0], k, u_scale, rho_scale, xin)
        model.gather_states(frames, sel[:, 1], k, u_scale, rho_scale, tgt)
        if noise > 0:
            xin.add_(torch.randn(xin.shape, generator=gen, device=xin.device) * sigma)
        for _ in range(m):  # the network's own rollout, no gradient through it
            model.forward(xin, xin)
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


def jump_errors(model: Surrogate, frames, pairs, u_scale: float, rho_scale: float):
    """Relative L2 errors of one surrogate jump and of persistence (state unchanged) on each pair,
    for phi and for v; model has batch 1.  Returns a dict of arrays."""
    import torch

    n = model.height
    outs = [torch.empty(n, n, dtype=torch.float64, device=frames.device) for _ in range(4)]
    err = {k: [] for k in ("phi_net", "phi_keep", "v_net", "v_keep")}
    nrm = lambda t: torch.linalg.vector_norm(t).item()
    for i0, i1 in pairs:
        model.forward_planes(*[frames[c, i0] for c in range(4)], u_scale, rho_scale, *outs)
        ref = frames[0, i1]
        err["phi_net"].append(nrm(outs[0] - ref) / nrm(ref))
        err["phi_keep"].append(nrm(frames[0, i0] - ref) / nrm(ref))
        vref = nrm(frames[1:3, i1])
        err["v_net"].append(nrm(torch.stack(outs[1:3]) - frames[1:3, i1]) / vref)
        err["v_keep"].append(nrm(frames[1:3, i0] - frames[1:3, i1]) / vref)
    return {k: np.asarray(v) for k, v in err.items()}


def dataset_runs(n: int, spinodal_seeds, coalescence):
    """(phi0, warm-up steps) of the training or evaluation runs: spinodal decomposition from the
    given seeds and two-droplet coalescence for the given (r1, r2, gap) cases."""
    return [(spinodal_phi(n, s), 0) for s in spinodal_seeds] + [(coalescence_phi(n, c), 0) for c in coalescence]


def fit(n: int, K: int, runs, frames_per_run: int, *, channels=64, layers=6, batch=8, iters=2000, lr=1e-3,
        seed=1, noise=0.0, pushforward=0, log=None):
    """Record the runs, derive the scales, train a fresh network.  Returns (model, info); the
    data tensors are released."""
    import torch

    t0 = time.perf_counter()
    frames, pairs = build_dataset(n, K, runs, frames_per_run)
    t_data = time.perf_counter() - t0
    us = velocity_scale(frames)
    rs = density_scale(frames)
    alpha = output_scale(frames, pairs, us, rs)
    model = Surrogate(batch, n, n, channels=channels, layers=layers)
    from .net import initial_params

    model.set_params(initial_params(channels, layers, seed=seed))
    model.set_output_scale(alpha)
    hist, secs = train(model, frames, pairs, us, rs, iters, lr=lr, log_every=max(1, iters // 10), noise=noise,
                       pushforward=pushforward, frames_per_run=frames_per_run, log=log)
    del frames
    torch.cuda.empty_cache()
    info = {"pairs": int(len(pairs)), "record_s": round(t_data, 2), "train_s": round(secs, 2), "iters": iters,
            "batch": batch, "ms_per_iter": round(secs / iters * 1e3, 3), "u_scale": us, "rho_scale": rs,
            "alpha": [float(a) for a in alpha], "noise": noise, "pushforward": pushforward, "loss_first": hist[0][1],
            "loss_last": hist[-1][1]}
    return model, info


def single_box(model: Surrogate, stream=None) -> Surrogate:
    """A batch-1 copy of a trained network (same parameters and output scale)."""
    m = Surrogate(1, model.height, model.width, channels=model.channels, layers=model.layers, stream=stream)
    m.set_params(model.params())
    m.set_output_scale(model.alpha)
    return m


def hybrid_vs_lb(model1: Surrogate, phi0, u_scale: float, rho_scale: float, windows: int, *, K=16, J=8, threshold=1e-2,
                 velocity_threshold=0.25, audit_every=0):
    """Advance phi0 by `windows` hybrid windows and by the same number of plain FP32 lattice steps
    from the same start; returns wall-clock rates, the hybrid's check (and audit) statistics and
    the trajectory error of the hybrid against plain lattice Boltzmann at equal simulated time:
    the relative L2 difference of the final phi and of its structure factor (the measure that
    stays meaningful where the dynamics amplify small differences, as in spinodal coarsening)."""
    import torch

    from . import analysis
    from .net import Hybrid

    n = phi0.shape[0]
    kw = dict(steps_per_jump=K, jumps_per_check=J, u_scale=u_scale, rho_scale=rho_scale, threshold=threshold,
              velocity_threshold=velocity_threshold, audit_every=audit_every)
    lat = lbcm.Lattice(n, n, precision="fp32", **PHYSICS)
    lat.init(phi0)
    hy = Hybrid(lat, model1, **kw)
    hy.advance(1)  # warm-up window (first launches)
    lat.init(phi0)
    hy.close()
    hy = Hybrid(lat, model1, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hy.advance(windows)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    st = hy.stats()
    hy.close()
    phi_h = lat.fields()["phi"]
    ref = lbcm.Lattice(n, n, precision="fp32", **PHYSICS)
    ref.init(phi0)
    ref.step(32)
    ref.init(phi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.step(st["steps"])
    torch.cuda.synchronize()
    t_lb = time.perf_counter() - t0
    phi_lb = ref.fields()["phi"]
    lat.close()
    ref.close()
    out = {"steps": st["steps"], "hybrid_steps_per_s": round(st["steps"] / t_h, 1),
           "lb_steps_per_s": round(st["steps"] / t_lb, 1), "speedup": round(t_lb / t_h, 3),
           "accepted_jumps": st["jumps"], "lb_steps_run": st["lb_steps_run"], "checks": st["checks"],
           "failed_checks": st["failed_checks"],
           "max_accepted_phi_error": st["max_accepted_error"],
           "max_accepted_velocity_error": st["max_accepted_velocity_error"],
           "final_phi_rel_l2_vs_lb": analysis.rel_l2(phi_h, phi_lb),
           "final_sk_rel_l2_vs_lb": analysis.sk_rel_l2(phi_h, phi_lb)}
    if audit_every:
        out.update({"audit_every": audit_every, "audits": st["audits"], "failed_audits": st["failed_audits"],
                    "max_audited_phi_error": st["max_audited_error"],
                    "max_audited_velocity_error": st["max_audited_velocity_error"]})
    return out


def restart_control(phi0, steps: int, span: int) -> dict:
    """The cost of the hybrid's equilibrium restarts alone: plain FP32 lattice Boltzmann that is
    re-initialised every `span` steps from the equilibrium populations of its own fields (phi, v,
    rho), as an accepted hybrid window's check does, against the same run without restarts, after
    `steps` steps: the relative L2 difference of phi and of its structure factor."""
    import torch

    from . import analysis

    n = phi0.shape[0]
    a = lbcm.Lattice(n, n, precision="fp32", **PHYSICS).init(phi0)
    b = lbcm.Lattice(n, n, precision="fp32", **PHYSICS).init(phi0)
    planes = [torch.empty(n, n, dtype=torch.float64, device="cuda") for _ in range(4)]  # phi, rho, v_x, v_y
    done = 0
    while done < steps:
        k = min(span, steps - done)
        a.step(k)
        done += k
        if done < steps:
            lbcm.lbcm_fields_device(a.h, planes[0], planes[1], planes[2], planes[3], None)
            lbcm.lbcm_init_device(a.h, *planes)
    b.step(steps)
    pa, pb = a.fields()["phi"], b.fields()["phi"]
    a.close()
    b.close()
    return {"steps": steps, "restart_every": span, "phi_rel_l2_vs_lb": analysis.rel_l2(pa, pb),
            "sk_rel_l2_vs_lb": analysis.sk_rel_l2(pa, pb)}
