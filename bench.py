"""Throughput of the fused lattice Boltzmann step on one MI355X.

Workload: 4096 x 4096 periodic spinodal decomposition (phi0 i.i.d. uniform in [-0.05, 0.05]
from SplitMix64 seed 1, rho = 1, v = 0, a = 0.04, gamma = 0.08, M = 0.1, Gamma = 1,
nu = 0.05 in both phases), FP32 populations.  One step = one launch of the fused step kernel,
which updates both population sets of every node (one LUP per node).

Timing: W warm-up steps, then 5 blocks of K steps, each between HIP events on the stream the
kernel runs on with the device synchronised on both sides; the line reports the median block
(and the mean and every block).  The untimed device-copy probe runs right before the warm-up, so
the GPU is busy when the warm-up starts: after any idle gap the first ~60 steps run up to 5 %
(FP32) and 8 % (16-bit) slower while the clocks come back up, whatever the state.

Prints one JSON line: MLUPS of the median timed block,
the HBM roofline of the step kernel (144 algorithmic bytes per LUP: 9 f + 9 g read, 9 f + 9 g
written, 4 bytes each) beside a plain device copy, and the FP64 CPU oracle timed on a bounded
sample on the host cores (all threads and one), plus the 64 x 64 droplet in full.  Further legs
in the same line: reduced-precision storage (throughput, and phi / sum-phi / structure-factor
errors against an FP64 GPU run at 2000 and 20000 steps), the 512-box ensemble, the learned
surrogate, and the two cache-resident correctness configurations.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BASELINE_METRIC = "MLUPS & % of HBM peak (D2Q9 f+g); surrogate speedup at φ L2 err ≤1e-2"
# bytes moved per lattice update (read + write of both sets): FP64 / FP32 planes, or 16-bit f and
# g_1..g_8 with g_0 kept in FP32
BYTES_PER_LUP = {"fp64": 288, "fp32": 144, "fp16s": 76, "bf16s": 76}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f32 (f16 storage)", "bf16s": "f32 (bf16 storage)"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--precision", default="fp32", choices=sorted(BYTES_PER_LUP))
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-wx", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=5, help="timed blocks of --steps steps (the median is reported)")
    ap.add_argument("--cpu-steps", type=int, default=16,
                    help="oracle steps in the CPU sample, timed as two halves (0 = skip)")
    ap.add_argument("--cpu-single-steps", type=int, default=1,
                    help="oracle steps of the single-thread CPU sample (0 = skip it)")
    ap.add_argument("--copy-probe", action="store_true", default=True,
                    help="time a plain device copy beside the step (the default)")
    ap.add_argument("--no-copy-probe", dest="copy_probe", action="store_false")
    ap.add_argument("--acc-steps", type=int, default=2000,
                    help="steps of the reduced-precision accuracy comparison (0 = skip the report)")
    ap.add_argument("--acc-long-steps", type=int, default=20000,
                    help="the same comparison continued to this many steps, with the structure factor "
                         "(0 = stop at --acc-steps)")
    ap.add_argument("--small-steps", type=int, default=2000,
                    help="steps of the cache-resident 64x64 and 4x256 cases (0 = skip them)")
    ap.add_argument("--ens-boxes", type=int, default=512, help="boxes of the ensemble leg (0 = skip it)")
    ap.add_argument("--ens-steps", type=int, default=5000, help="batched steps of the ensemble leg")
    ap.add_argument("--ens-looped-steps", type=int, default=40, help="looped steps timed for comparison")
    ap.add_argument("--ens-persistent-steps", type=int, default=400,
                    help="steps timed with each persistent schedule (0 = skip them)")
    ap.add_argument("--sur-iters", type=int, default=2000, help="training iterations of the surrogate leg (0 = skip it)")
    ap.add_argument("--sur-windows", type=int, default=40, help="hybrid windows (8 jumps of 16 steps) timed per case")
    ap.add_argument("--sur-kernels", type=int, default=0,
                    help="only a short kernel workload of the surrogate (for counter runs): this many jumps and "
                         "training iterations on seeded data, with progress lines; every other leg is skipped")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n: int, steps: int, single_steps: int, small_steps: int) -> dict:
    """The FP64 oracle on the host: the 4096^2 workload on all threads given by OMP_NUM_THREADS
    (a bounded sample of steps, timed as two halves run in place, so that the spread shows the
    per-step cost is constant), on one thread, and the 64 x 64 static droplet run in full."""
    import numpy as np

    import oracle
    from paper_1803_11345_amd import inputs

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    phys = dict(a=0.04, gamma=0.08, mobility=0.1, Gamma=1.0, nu_l=0.05, nu_g=0.05)

    def timed(nx, ny, phi, parts, nthreads, **kw):
        q = dict(phys)
        q.update(kw)
        p = oracle.Params(nx, ny, nthreads=nthreads, **q)
        f, g = oracle.init(p, phi)
        secs = []
        for k in parts:
            t0 = time.perf_counter()
            oracle.run(p, f, g, k, inplace=True)
            secs.append(time.perf_counter() - t0)
        assert np.isfinite(f).all()
        return nx * ny * sum(parts) / sum(secs) / 1e6, secs

    phi0 = inputs.spinodal(n, n, seed=1)
    half = max(1, steps // 2)
    v, secs = timed(n, n, phi0, (half, half), threads)
    out = {"value": round(v, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"FP64 oracle (gcc -O3, OpenMP), {n}x{n} spinodal (same initial state), {2 * half} steps "
                     f"after initialisation, {sum(secs):.1f} s on {threads} OpenMP threads; halves "
                     f"{n * n * half / secs[0] / 1e6:.2f} and {n * n * half / secs[1] / 1e6:.2f} MLUPS"}
    if single_steps > 0:
        v1, s1 = timed(n, n, phi0, (single_steps,), 1)
        out["single_thread"] = {"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                                "sample": f"the same, {single_steps} step(s), {sum(s1):.1f} s on one thread"}
    if small_steps > 0:
        w = inputs.interface_width(0.04, 0.08)
        vs, ss = timed(64, 64, inputs.droplet(64, 64, 16, w), (small_steps,), threads, nu_l=1 / 6, nu_g=1 / 6)
        out["droplet64"] = {"value": round(vs, 3), "unit": "MLUPS", "cores": threads,
                            "sample": f"64x64 static droplet (R = 16, nu = 1/6), {small_steps} steps, {sum(ss):.2f} s"}
    return out


def copy_probe(nbytes: int = 1 << 31, reps: int = 20) -> float:
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * nbytes / sec / 1e9


def stream_probe(n: int) -> float:
    """GB/s of the library's streaming reference: 18 planes of n^2 floats read and written, one
    element per lane (the step kernel's access pattern without shifts, halos and arithmetic)."""
    import torch

    from paper_1803_11345_amd import lbcm

    N = n * n
    a = torch.zeros(18 * N, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = lbcm.lbcm_stream_probe(a, b, N, 18, 20, torch.cuda.current_stream().cuda_stream)
    del a, b
    return 2 * 18 * N * 4 / ms / 1e6


def measured_traffic(n, precision, args, sec_per_step):
    """HBM traffic of the step kernel from the committed rocprofv3 counter record of this
    workload, as GB/s at the live step time; None when no record exists, the tiles differ from
    the defaults it was taken with, or the kernel source has changed since."""
    from paper_1803_11345_amd import profile_summary

    path = os.path.join(ROOT, "profiles", f"k_step_spinodal{n}_{precision}_traffic.json")
    if args.tile_rows or args.tile_wx or not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("source_sha256") != profile_summary.source_digest() or rec.get("nodes") != n * n:
        return None, None
    return rec["traffic_bytes_per_launch"] / sec_per_step / 1e9, rec["traffic_bytes_per_launch"]


def make_lattice(lbcm, n, precision, args):
    return lbcm.Lattice(n, n, precision=precision, tile_rows=args.tile_rows, tile_wx=args.tile_wx,
                        a=0.04, gamma=0.08, mobility=0.1, Gamma=1.0, nu_l=0.05, nu_g=0.05)


def time_blocks(lat, steps, warmup, blocks):
    """Seconds per step of each of `blocks` blocks of `steps` launches, each between HIP events on
    the lattice's stream with the device synchronised before and after, after `warmup` untimed
    steps."""
    import torch

    lat.step(warmup)
    torch.cuda.synchronize()
    out = []
    for _ in range(blocks):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / 1e3 / steps)
    return out


def median(v):
    import statistics

    return statistics.median(v)


# secondary legs (not the headline line) warm up long enough to pass the clock ramp after idle gaps
LEG_WARMUP = 200


def precision_report(lbcm, phi0, n, args, fp32_sec):
    """Reduced-precision storage against the plain FP32 step: throughput, speedup, and the error
    against an FP64 GPU run of the same workload after acc_steps steps (phi L2, sum phi drift) and
    after acc_long_steps (the same, and the radially averaged structure factor, which the chaotic
    growth of round-off leaves comparable where phi itself is not)."""
    import numpy as np

    from paper_1803_11345_amd import analysis

    marks = [args.acc_steps] + ([args.acc_long_steps] if args.acc_long_steps > args.acc_steps else [])
    phis, drift = {}, {}
    for prec in ("fp64", "fp32", "fp16s", "bf16s"):
        lat = make_lattice(lbcm, n, prec, args).init(phi0)
        d0 = lat.diag()
        done = 0
        for mark in marks:
            lat.step(mark - done)
            done = mark
            phis[prec, mark] = lat.fields()["phi"]
            d1 = lat.diag()
            drift[prec, mark] = abs(d1["sum_phi"] - d0["sum_phi"]) / d0["sum_abs_phi"]
        lat.close()

    def errors(prec, mark):
        ref = phis["fp64", mark]
        e = {"phi_rel_l2": float(np.linalg.norm(phis[prec, mark] - ref) / np.linalg.norm(ref)),
             "sum_phi_drift": drift[prec, mark]}
        if mark != args.acc_steps:
            e["sk_rel_l2"] = analysis.sk_rel_l2(phis[prec, mark], ref)
        return e

    a = args.acc_steps
    out = {"acc_steps": a, "reference": "fp64 GPU run, same initial state",
           "fp64_sum_phi_drift": drift["fp64", a], "fp32": errors("fp32", a)}
    if len(marks) > 1:
        out["long"] = {"steps": marks[1], "fp64_sum_phi_drift": drift["fp64", marks[1]],
                       **{prec: errors(prec, marks[1]) for prec in ("fp32", "fp16s", "bf16s")}}
    for prec in ("fp16s", "bf16s"):
        lat = make_lattice(lbcm, n, prec, args).init(phi0)
        sec = median(time_blocks(lat, args.steps, max(args.warmup, LEG_WARMUP), args.blocks))
        lat.close()
        out[prec] = {"value": round(n * n / sec / 1e6, 1), "unit": "MLUPS",
                     "speedup_vs_fp32": round(fp32_sec / sec, 3),
                     "hbm_gbs_alg": round(BYTES_PER_LUP[prec] * n * n / sec / 1e9, 1), **errors(prec, a)}
    return out


def small_report(lbcm, steps, warmup):
    """MLUPS of the two correctness configurations, whose data stay in the caches (launch
    latency, not HBM, bounds them): the 64 x 64 static droplet in FP64 and the 4 x 256 layered
    channel (walls, body force, viscosity ratio 1000) in FP32."""
    from paper_1803_11345_amd import inputs

    w = inputs.interface_width(0.04, 0.08)
    cases = {
        "droplet64_fp64": (64, 64, inputs.droplet(64, 64, 16, w),
                           dict(precision="fp64", a=0.04, gamma=0.08, mobility=0.1, nu_l=1 / 6, nu_g=1 / 6)),
        "channel4x256_fp32": (4, 256, inputs.layered(4, 256, w),
                              dict(precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.1, nu_g=100.0,
                                   bc_y=lbcm.LBCM_BC_WALLS, force_x=1e-6)),
    }
    out = {"note": "cache-resident: MLUPS only, no HBM fraction"}
    for name, (nx, ny, phi, kw) in cases.items():
        lat = lbcm.Lattice(nx, ny, **kw).init(phi)
        sec = median(time_blocks(lat, steps, max(warmup, LEG_WARMUP), 5))
        lat.close()
        out[name] = {"value": round(nx * ny / sec / 1e6, 1), "unit": "MLUPS", "us_per_step": round(sec * 1e6, 2)}
    return out


def ensemble_report(lbcm, args) -> dict:
    """Ensemble of independent boxes (sides 64..1024, droplets or layered channels, viscosity
    ratio 1..1000, FP16-shifted storage) advanced by one launch per step under a hipGraph with
    autotuned tiles, against the same steps as single-box launches (on the batch's stream, and
    dealt over 4 and 8 streams), and against one persistent launch per call (grid barrier per
    step, and per-tile dataflow)."""
    import torch

    from paper_1803_11345_amd import inputs

    spec = inputs.ensemble(args.ens_boxes, seed=7)
    nodes = sum(p["nx"] * p["ny"] for p, _ in spec)
    bt = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    for box, (_, phi0) in zip(bt, spec):
        box.init(phi0)
    del spec
    t0 = time.perf_counter()
    info = bt.autotune(trials=10)
    tune_s = time.perf_counter() - t0

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bt.stream)
        fn(steps)
        e1.record(bt.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    timed(bt.step, 20)
    sec = timed(bt.step, args.ens_steps)
    timed(bt.step_looped, 2)
    sec_loop = timed(bt.step_looped, args.ens_looped_steps)
    # the same single-box launches over several streams (boxes of one step may then overlap)
    loop_streams = {}
    for ns in (4, 8):
        timed(lambda k: bt.step_looped_streams(k, ns), 2)
        sl = timed(lambda k: bt.step_looped_streams(k, ns), args.ens_looped_steps)
        loop_streams[str(ns)] = round(nodes * args.ens_looped_steps / sl / 1e6, 1)
    persistent = {}
    if args.ens_persistent_steps > 0:
        for mode, name in ((1, "barrier_per_step"), (2, "dataflow")):
            bt.set_persistent(mode)
            timed(bt.step, 10)
            sp = timed(bt.step, args.ens_persistent_steps)
            persistent[name] = {"value": round(nodes * args.ens_persistent_steps / sp / 1e6, 1), "unit": "MLUPS",
                                "steps": args.ens_persistent_steps}
        bt.set_persistent(0)
    nonfinite = sum(box.diag()["nonfinite"] for box in bt)
    mlups = nodes * args.ens_steps / sec / 1e6
    mlups_loop = nodes * args.ens_looped_steps / sec_loop / 1e6
    bt.close()
    return {"boxes": args.ens_boxes, "nodes": nodes, "precision": "fp16s", "steps": args.ens_steps,
            "value": round(mlups, 1), "unit": "MLUPS", "hbm_gbs_alg": round(mlups * 76 / 1e3, 1),
            "looped_single_box_mlups": round(mlups_loop, 1),
            "looped_single_box_over_streams_mlups": loop_streams,
            "speedup_vs_looped_over_streams": round(mlups / max(loop_streams.values()), 3),
            "persistent_launch": persistent,
            "speedup_vs_looped": round(mlups / mlups_loop, 3), "graph": True,
            "tuned": {"waves": info["waves"], "order": ["box order", "largest first", "one XCD per box"][info["order"]],
                      "tiles": info["ntiles"], "autotune_s": round(tune_s, 2)},
            "nonfinite_nodes": int(nonfinite)}


def surrogate_report(lbcm, args) -> dict:
    """Learned surrogate on 256 x 256 periodic boxes: record LB trajectories (spinodal
    decomposition and two-droplet coalescence), train the 6-layer 64-channel network on the GPU
    with the library's kernels, then compare one jump with persistence on held-out runs and time
    the hybrid (surrogate jumps of K = 16 steps, a lattice check of the last of every 8 jumps,
    fallback above a phi error of 1e-2) against the plain FP32 step on the same box."""
    import numpy as np
    import torch

    from paper_1803_11345_amd import inputs
    from paper_1803_11345_amd import train as T

    n, K = 256, 16
    cases = inputs.coalescence_cases(12, seed=11)
    model, info = T.fit(n, K, T.dataset_runs(n, (101, 102, 103, 104), cases[:8]), 400, iters=args.sur_iters)
    m1 = T.single_box(model)
    model.close()
    us, rs = info["u_scale"], info["rho_scale"]
    # one jump against persistence on held-out runs
    frames, pairs = T.build_dataset(n, K, T.dataset_runs(n, (105,), cases[8:9]), 400)
    gains = {}
    for name, sl in (("spinodal", slice(10, 399)), ("coalescence", slice(409, 798))):
        e = T.jump_errors(m1, frames, pairs[sl], us, rs)
        gains[name] = {k: {"mean": float(v.mean()), "max": float(v.max())} for k, v in e.items()}
    # time of one jump (FP64 planes in and out, as the hybrid runs it)
    outs = [torch.empty(n, n, dtype=torch.float64, device="cuda") for _ in range(4)]
    ins = [frames[c, 0] for c in range(4)]
    for _ in range(LEG_WARMUP):
        m1.forward_planes(*ins, us, rs, *outs)
    torch.cuda.synchronize()
    jump_blocks = []  # five blocks of 100 jumps, the median reported (as the headline's blocks)
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(100):
            m1.forward_planes(*ins, us, rs, *outs)
        e1.record()
        torch.cuda.synchronize()
        jump_blocks.append(e0.elapsed_time(e1) * 1e3 / 100)
    jump_us = median(jump_blocks)
    del frames, ins
    torch.cuda.empty_cache()
    # padded MFMA work of one jump: layers 1..L-2 are 64 -> 64, the last 64 -> 16 computed
    # channels (4 real) in the fused inference path
    flops = 2 * n * n * 9 * 64 * (4 * 64 + 16)
    hybrid, audited, identity, restart = {}, {}, {}, {}
    from paper_1803_11345_amd.net import Surrogate

    m0 = Surrogate(1, n, n, channels=64, layers=6)  # control: the zero network is the identity map
    m0.set_params(np.zeros(m0.nparams, dtype=np.float32))
    m0.set_output_scale(m1.alpha)
    for name, phi0 in (("spinodal", T.spinodal_phi(n, 106)), ("coalescence", T.coalescence_phi(n, cases[9]))):
        hybrid[name] = T.hybrid_vs_lb(m1, phi0, us, rs, args.sur_windows)
        audited[name] = T.hybrid_vs_lb(m1, phi0, us, rs, args.sur_windows, audit_every=4)
        identity[name] = T.hybrid_vs_lb(m0, phi0, us, rs, args.sur_windows, threshold=float("inf"),
                                        velocity_threshold=0.0)
        restart[name] = T.restart_control(phi0, hybrid[name]["steps"], 8 * K)
    m0.close()
    m1.close()
    return {"box": f"{n}x{n} periodic", "network": "3x3 conv x6, 64 channels, first layer FP32 MFMA, "
            "others BF16 MFMA with FP32 accumulation", "steps_per_jump": K, "jumps_per_check": 8,
            "threshold_phi_rel_l2": 1e-2, "threshold_velocity_rel_l2": 0.25, "train": info, "one_jump_rel_l2": gains,
            "jump_us": round(jump_us, 2), "jump_us_blocks": [round(b, 2) for b in jump_blocks],
            "jump_mfma_tflops": round(flops / jump_us / 1e6, 1),
            "hybrid": hybrid,
            "speedup_vs_lb": round(float(np.mean([h["speedup"] for h in hybrid.values()])), 3),
            "speedup_at_error": {k: {"speedup": h["speedup"], "final_phi_rel_l2_vs_lb": round(h["final_phi_rel_l2_vs_lb"], 5),
                                     "final_sk_rel_l2_vs_lb": round(h["final_sk_rel_l2_vs_lb"], 5)}
                                 for k, h in hybrid.items()},
            "hybrid_audit_every_4_windows": audited,
            "controls": {"identity_network_no_threshold": identity,
                         "plain_lb_with_equilibrium_restart_every_window": restart}}


def surrogate_kernels(n_iter: int) -> dict:
    """The surrogate's kernels alone, on seeded data (no lattice runs): n_iter inference jumps of
    the 6-layer 64-channel network on one 256^2 box from FP64 planes, and n_iter training
    iterations (forward, backward, Adam) at batch 8.  Prints a line per phase (stderr)."""
    import numpy as np
    import torch

    from paper_1803_11345_amd import inputs
    from paper_1803_11345_amd.net import Surrogate, initial_params

    n = 256
    p = initial_params(64, 6, seed=1)
    m1 = Surrogate(1, n, n, channels=64, layers=6)
    m1.set_params(p)
    planes = [torch.from_numpy(inputs.uniform(10 + c, n * n).reshape(n, n) * 0.1).cuda() for c in range(4)]
    outs = [torch.empty(n, n, dtype=torch.float64, device="cuda") for _ in range(4)]
    print(f"surrogate kernels: {n_iter} jumps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_iter):
        m1.forward_planes(*planes, 1.0, 1.0, *outs)
    torch.cuda.synchronize()
    jump = (time.perf_counter() - t0) / n_iter
    m1.close()
    m8 = Surrogate(8, n, n, channels=64, layers=6)
    m8.set_params(p)
    x = torch.from_numpy((inputs.uniform(20, 8 * n * n * 4).reshape(8, n, n, 4) * 0.1).astype(np.float32)).cuda()
    y = torch.from_numpy((inputs.uniform(21, 8 * n * n * 4).reshape(8, n, n, 4) * 0.1).astype(np.float32)).cuda()
    print(f"surrogate kernels: {n_iter} training iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_iter):
        m8.forward(x)
        m8.backward(y, want_loss=False)
        m8.adam(1e-4)
    torch.cuda.synchronize()
    it = (time.perf_counter() - t0) / n_iter
    m8.close()
    print("surrogate kernels: done", file=sys.stderr, flush=True)
    return {"jumps": n_iter, "jump_us_wall": round(jump * 1e6, 2), "iterations": n_iter,
            "iteration_ms_wall": round(it * 1e3, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU slab decomposition is a design note, not code", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1803_11345_amd import inputs, lbcm

    torch.cuda.set_device(0)
    if args.sur_kernels > 0:
        print(json.dumps({"surrogate_kernels": surrogate_kernels(args.sur_kernels)}), flush=True)
        return
    n = args.n
    phi0 = inputs.spinodal(n, n, seed=1)
    lat = make_lattice(lbcm, n, args.precision, args).init(phi0)
    copy_gbs = copy_probe() if args.copy_probe else None  # untimed; keeps the GPU busy up to the warm-up
    stream_gbs = stream_probe(n) if args.copy_probe else None
    wall0 = time.perf_counter()
    block_sec = time_blocks(lat, args.steps, args.warmup, args.blocks)
    wall = time.perf_counter() - wall0
    sec_per_step = median(block_sec)
    nodes = n * n
    mlups = nodes / sec_per_step / 1e6
    d = lat.diag()
    assert d["nonfinite"] == 0, "non-finite state after the timed steps"
    achieved = BYTES_PER_LUP[args.precision] * nodes / sec_per_step / 1e9
    traffic, traffic_bytes = measured_traffic(n, args.precision, args, sec_per_step)
    out = {
        "metric": BASELINE_METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_step * 1e3, 5),
        "timing": {"blocks": args.blocks, "steps_per_block": args.steps, "reported": "median block",
                   "block_ms_per_step": [round(b * 1e3, 5) for b in block_sec],
                   "mean_ms_per_step": round(sum(block_sec) / len(block_sec) * 1e3, 5),
                   "mean_mlups": round(nodes / (sum(block_sec) / len(block_sec)) / 1e6, 1)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"spinodal decomposition {n}x{n} periodic D2Q9 f+g, "
                               f"phi0 U[-0.05,0.05] seed 1, a=0.04 gamma=0.08 M=0.1 nu=0.05, "
                               f"{args.precision} populations",
                   "nx": n, "ny": n, "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic, 1),
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": "k_step", "bytes_per_lup": BYTES_PER_LUP[args.precision]},
        "wall_s_warmup_and_timed": round(wall, 3),
        "sum_phi_drift": abs(d["sum_phi"] - float(np.sum(phi0))) / float(np.sum(np.abs(phi0))),
    }
    lat.close()
    if args.acc_steps > 0 and args.precision == "fp32":
        out["reduced_precision"] = precision_report(lbcm, phi0, n, args, sec_per_step)
    if args.ens_boxes > 0 and args.precision == "fp32":
        out["ensemble"] = ensemble_report(lbcm, args)
    if args.sur_iters > 0 and args.precision == "fp32":
        out["surrogate"] = surrogate_report(lbcm, args)
    if args.small_steps > 0 and args.precision == "fp32":
        out["cache_resident"] = small_report(lbcm, args.small_steps, args.warmup)
    if copy_gbs is not None:
        out["roofline"]["copy_probe_gbs"] = round(copy_gbs, 1)
        out["roofline"]["copy_probe"] = "torch device copy of 2 GiB (reads + writes)"
        out["roofline"]["stream_probe_gbs"] = round(stream_gbs, 1)
        out["roofline"]["stream_probe"] = ("lbcm_stream_probe: 18 planes of the lattice's size read and written, one "
                                           "FP32 element per lane, non-temporal stores")
        out["roofline"]["frac_of_stream_probe"] = round(achieved / stream_gbs, 4)
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_steps, args.cpu_single_steps,
                                           args.small_steps if args.precision == "fp32" else 0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
