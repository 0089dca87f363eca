"""GPU tests of the ensemble path: one launch per step over every tile of every box.  The
per-node arithmetic does not depend on the tile a node falls in, so every box of a batch must
match, bit for bit, the same box stepped as a single lattice (which the parity tests tie to the
oracle)."""
import numpy as np
import pytest

from paper_1803_11345_amd import inputs, lbcm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def say(*a):
    print(*a, flush=True)


BOXES = [
    dict(nx=64, ny=64, nu_l=0.1, nu_g=0.01),
    dict(nx=100, ny=37, bc_y=1, nu_l=0.1, nu_g=1.0, force_x=1e-5),
    dict(nx=33, ny=17, nu_l=0.1, nu_g=0.05, force_y=2e-5),
    dict(nx=130, ny=65, bc_y=1, nu_l=0.05, nu_g=0.5),
    dict(nx=1, ny=1),
    dict(nx=200, ny=3, nu_l=0.1, nu_g=0.1),
    dict(nx=257, ny=129, nu_l=0.1, nu_g=0.002),
    dict(nx=90, ny=40, bc_y=1, nu_l=0.1, nu_g=0.1, wall_vx_bottom=-2e-3, wall_vx_top=4e-3, wall_gradient=0.04),
]


def _states(seed):
    return [inputs.smooth_state(b["nx"], b["ny"], seed=seed + k) for k, b in enumerate(BOXES)]


def _singles(prec, steps, seed):
    out = []
    for b, st in zip(BOXES, _states(seed)):
        lat = lbcm.Lattice(precision=prec, **b).init(*st).step(steps)
        out.append(lat.get_state())
        lat.close()
    return out


def _batch(prec, seed):
    bt = lbcm.Batch(BOXES, precision=prec)
    for box, st in zip(bt, _states(seed)):
        box.init(*st)
    return bt


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_batch_matches_single_lattices(prec, graph, order):
    """Every tile order (boxes in turn, largest first, one XCD per box with empty slots in the
    grid) gives the single-lattice result bit for bit."""
    say(f"case batch {prec} graph={graph} order={order}")
    ref = _singles(prec, 7, 50)
    bt = _batch(prec, 50)
    bt.set_graph(graph)
    bt.set_order(order)
    with pytest.raises(lbcm.LbcmError):
        bt.set_order(3)
    bt.step(3).step(4)  # odd first call: phase handling around the two-step graph
    for k, box in enumerate(bt):
        assert np.array_equal(box.get_state(), ref[k]), k
        assert box.diag()["step"] == 7
    bt.close()


def test_batch_looped_equals_batched():
    a = _batch("fp32", 60)
    b = _batch("fp32", 60)
    a.step(5)
    b.step_looped(5)
    for x, y in zip(a, b):
        assert np.array_equal(x.get_state(), y.get_state())
    a.close()
    b.close()


@pytest.mark.parametrize("nstreams", [1, 3, 8])
def test_batch_looped_over_streams_equals_batched(nstreams):
    """Single-box launches dealt to several streams (forked from and joined to the batch's
    stream every step) give the batched result bit for bit; bad stream counts are rejected."""
    a = _batch("fp32", 61)
    b = _batch("fp32", 61)
    a.step(5)
    b.step_looped_streams(5, nstreams)
    for x, y in zip(a, b):
        assert np.array_equal(x.get_state(), y.get_state())
    for bad in (0, 65):
        with pytest.raises(lbcm.LbcmError) as e:
            b.step_looped_streams(1, bad)
        assert e.value.code == lbcm.LBCM_EINVAL
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_batch_autotune_keeps_state_and_results(prec):
    """Autotuning changes no state; afterwards the batched launch and the boxes' own tuned
    single-lattice launches (two-row waves with 16-bit storage) both match fresh single runs."""
    bt = _batch(prec, 70)
    before = [box.get_state() for box in bt]
    info = bt.autotune(trials=2)
    say(f"  autotuned: {info}")
    assert info["waves"] in (8, 12, 16) and info["order"] in (0, 1, 2)
    for b, w, r in zip(BOXES, info["wx"], info["rows"]):
        # a full workgroup unless the box is smaller than the tile
        assert w * r == info["waves"] or (w * 64 >= b["nx"] and r >= b["ny"]) or r * w < info["waves"] and r >= b["ny"]
    for box, st in zip(bt, before):
        assert np.array_equal(box.get_state(), st)
    bt.step(6)
    ref = _singles(prec, 6, 70)
    for k, box in enumerate(bt):
        assert np.array_equal(box.get_state(), ref[k]), k
    bt.step_looped(3)
    ref = _singles(prec, 9, 70)
    for k, box in enumerate(bt):
        assert np.array_equal(box.get_state(), ref[k]), k
    bt.close()


def test_box_stepped_alone_then_batch():
    bt = _batch("fp32", 80)
    bt[0].step(1)
    bt.step(4)
    ref = _singles("fp32", 4, 80)
    ref0 = _singles("fp32", 5, 80)[0]
    assert np.array_equal(bt[0].get_state(), ref0)
    for k in range(1, len(BOXES)):
        assert np.array_equal(bt[k].get_state(), ref[k]), k
    bt.close()


def test_graph_replays_match_eager():
    """Several graph replays with eager work (diagnostics, host reads) in between, each checked
    against a batch stepped without graphs."""
    g = _batch("fp32", 90)
    e = _batch("fp32", 90)
    e.set_graph(False)
    for rep in range(4):
        g.step(2)
        e.step(2)
        for x, y in zip(g, e):
            x.diag()
            assert np.array_equal(x.get_state(), y.get_state()), rep
    g.close()
    e.close()


def test_ensemble_generator_runs_finite():
    spec = inputs.ensemble(12, seed=3, sides=(64, 128))
    bt = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    for box, (_, phi0) in zip(bt, spec):
        box.init(phi0)
    bt.autotune(trials=2)
    bt.step(200)
    for box in bt:
        assert box.diag()["nonfinite"] == 0
    bt.close()


def test_full_ensemble_matches_single_lattices_on_sampled_boxes():
    """The 512-box FP16 ensemble of the benchmark (seed 7, sides 64 ... 1024, droplets and
    layered channels), autotuned and advanced with graphs as the benchmark does: sampled boxes
    (the first and last box, the largest and smallest of each kind) equal the same boxes stepped
    as single lattices, bit for bit."""
    spec = inputs.ensemble(512, seed=7)
    bt = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    for box, (_, phi0) in zip(bt, spec):
        box.init(phi0)
    info = bt.autotune(trials=3)
    say(f"  ensemble: waves {info['waves']} order {info['order']} tiles {info['ntiles']}")
    bt.step(11)
    size = [p["nx"] * p["ny"] for p, _ in spec]
    picks = {0, len(spec) - 1}
    for walls in (0, 1):
        kind = [k for k, (p, _) in enumerate(spec) if p["bc_y"] == walls]
        picks |= {max(kind, key=lambda k: size[k]), min(kind, key=lambda k: size[k])}
    for k in sorted(picks):
        p, phi0 = spec[k]
        lat = lbcm.Lattice(precision="fp16s", **p).init(phi0).step(11)
        assert np.array_equal(lat.get_state(), bt[k].get_state()), (k, p["nx"], p["bc_y"])
        lat.close()
    bt.close()


# ---------------------------------------------------------------------------------------------
# ensembles against the oracle directly (not only against single-lattice GPU runs)

def _oracle_run(p, phi, steps, rho=None, ux=None, uy=None, nthreads=0):
    import oracle

    okw = {k: v for k, v in p.items() if k not in ("nx", "ny")}
    if "bc_y" in okw:
        okw["walls"] = okw.pop("bc_y")
    for side in ("bottom", "top"):
        if f"wall_vx_{side}" in okw:
            okw[f"wall_ux_{side}"] = okw.pop(f"wall_vx_{side}")
    q = oracle.Params(p["nx"], p["ny"], nthreads=nthreads, **okw)
    return oracle.run(q, *oracle.init(q, phi, rho, ux, uy), steps)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-5), ("fp16s", 3e-4)])
def test_batch_boxes_match_the_oracle(prec, tol):
    """Every box of a mixed ensemble (periodic, walls, force, moving and wetting walls, ragged and
    tiny sizes) advanced 7 steps by the batched launch with graphs, element by element against
    the oracle, within the single-lattice tiers of each storage (FP64 1e-14 per step; FP32 and
    FP16 storage the 50-step tiers)."""
    say(f"case batch vs oracle {prec}")
    steps = 7
    bt = _batch(prec, 110)
    bt.step(steps)
    worst = 0.0
    for k, (b, st) in enumerate(zip(BOXES, _states(110))):
        fo, go = _oracle_run(b, st[0], steps, *st[1:])
        f, g = bt[k].populations()
        e = max(float(np.abs(f - fo).max()), float(np.abs(g - go).max()))
        say(f"  box {k} {b['nx']}x{b['ny']} bc_y={b.get('bc_y', 0)}: max |GPU - oracle| = {e:.2e}")
        worst = max(worst, e)
        assert e < tol, k
    bt.close()


def test_full_ensemble_sampled_boxes_match_the_oracle():
    """The 512-box FP16-storage ensemble of the benchmark, autotuned and advanced with graphs:
    after 11 steps the first and last box and the smallest and largest box of each kind
    (droplets, layered channels with walls and force) against the oracle, element by element,
    within the FP16 tier (3e-4)."""
    spec = inputs.ensemble(512, seed=7)
    bt = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    for box, (_, phi0) in zip(bt, spec):
        box.init(phi0)
    bt.autotune(trials=3)
    bt.step(11)
    size = [p["nx"] * p["ny"] for p, _ in spec]
    picks = {0, len(spec) - 1}
    for walls in (0, 1):
        kind = [k for k, (p, _) in enumerate(spec) if p["bc_y"] == walls]
        picks |= {max(kind, key=lambda k: size[k]), min(kind, key=lambda k: size[k])}
    for k in sorted(picks):
        p, phi0 = spec[k]
        say(f"case ensemble box {k}: {p['nx']}x{p['ny']} bc_y={p['bc_y']}")
        fo, go = _oracle_run(p, phi0, 11)
        f, g = bt[k].populations()
        e = max(float(np.abs(f - fo).max()), float(np.abs(g - go).max()))
        say(f"  max |GPU - oracle| = {e:.2e}")
        assert e < 3e-4, k
    bt.close()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_reports_divergence_of_one_box(graph):
    """A box whose state holds a NaN: with check_every on any box, lbcm_batch_step returns
    LBCM_EDIVERGED naming that box; re-initialising the box clears its flag and the batch steps
    on without error."""
    boxes = [dict(b, check_every=4 if k == 1 else 0) for k, b in enumerate(BOXES)]
    bt = lbcm.Batch(boxes, precision="fp32")
    states = _states(120)
    for box, st in zip(bt, states):
        box.init(*st)
    bt.set_graph(graph)
    bt.step(9)  # all finite: no error
    bad = states[3][0].copy()
    bad[10, 10] = np.nan
    bt[3].init(bad, *states[3][1:])
    with pytest.raises(lbcm.LbcmError) as e:
        bt.step(6)
    assert e.value.code == lbcm.LBCM_EDIVERGED and "box 3" in str(e.value)
    bt[3].init(*states[3])
    bt.step(6)
    for box in bt:
        assert box.diag()["nonfinite"] == 0
    bt.close()


# ---------------------------------------------------------------------------------------------
# persistent launches (one launch for all the steps of a call)

@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
@pytest.mark.parametrize("order", [1, 2])
def test_persistent_launch_matches_single_lattices(mode, prec, order):
    """Both persistent schedules (grid barrier per step; per-tile dataflow) give the single-lattice
    result bit for bit, for an odd first call (phase handling) and in both tile orders (order 2
    has empty slots in its table)."""
    say(f"case persistent mode={mode} {prec} order={order}")
    ref = _singles(prec, 7, 130)
    bt = _batch(prec, 130)
    bt.set_order(order)
    bt.set_persistent(mode)
    bt.step(3).step(4)
    for k, box in enumerate(bt):
        assert np.array_equal(box.get_state(), ref[k]), k
        assert box.diag()["step"] == 7
    bt.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_persistent_full_ensemble_matches_per_step_launches(mode):
    """The 512-box FP16-storage benchmark ensemble, autotuned: 23 steps in one persistent launch
    equal 23 per-step launches bit for bit on every box, and sampled boxes match the oracle."""
    spec = inputs.ensemble(512, seed=7)
    a = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    b = lbcm.Batch([p for p, _ in spec], precision="fp16s")
    for x, y, (_, phi0) in zip(a, b, spec):
        x.init(phi0)
        y.init(phi0)
    a.autotune(trials=2)
    info = a.info()
    b.autotune(trials=2)
    say(f"case persistent full ensemble mode={mode}: waves {info['waves']} order {info['order']}")
    a.set_persistent(mode)
    a.step(23)
    b.step(23)
    for k in range(len(spec)):
        assert np.array_equal(a[k].get_state(), b[k].get_state()), k
    size = [p["nx"] * p["ny"] for p, _ in spec]
    for k in (min(range(len(spec)), key=lambda k: size[k]), 1):
        p, phi0 = spec[k]
        fo, go = _oracle_run(p, phi0, 23)
        f, g = a[k].populations()
        assert max(float(np.abs(f - fo).max()), float(np.abs(g - go).max())) < 3e-4, k
    a.close()
    b.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_persistent_launch_checks_divergence(mode):
    """check_every splits a call into one persistent launch per period with a check after each:
    a NaN in one box is reported naming it; re-initialised, the batch steps on."""
    boxes = [dict(b, check_every=3 if k == 2 else 0) for k, b in enumerate(BOXES)]
    bt = lbcm.Batch(boxes, precision="fp32")
    states = _states(140)
    for box, st in zip(bt, states):
        box.init(*st)
    bt.set_persistent(mode)
    bt.step(7)
    ref = _singles("fp32", 7, 140)
    for k, box in enumerate(bt):
        assert np.array_equal(box.get_state(), ref[k]), k
    bad = states[5][0].copy()
    bad[1, 50] = np.nan
    bt[5].init(bad, *states[5][1:])
    with pytest.raises(lbcm.LbcmError) as e:
        bt.step(5)
    assert e.value.code == lbcm.LBCM_EDIVERGED and "box 5" in str(e.value)
    bt[5].init(*states[5])
    bt.step(4)
    for box in bt:
        assert box.diag()["nonfinite"] == 0
    with pytest.raises(lbcm.LbcmError):
        bt.set_persistent(3)
    bt.close()
