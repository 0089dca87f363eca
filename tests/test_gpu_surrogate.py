"""GPU parity of the surrogate network kernels (BF16 MFMA forward, backward, Adam, state packing)
against the FP64 network oracle with BF16 operand rounding emulated, and checks of the hybrid
driver's bookkeeping.  All calls go through the C ABI (paper_1803_11345_amd.net)."""
import sys

import numpy as np
import pytest

from oracle import convnet as cn
from paper_1803_11345_amd import inputs, lbcm, net

pytestmark = pytest.mark.gpu

# Tolerances on random data.  Both sides round the same operands to bfloat16; they differ by
# FP32 versus FP64 rounding of the sums (relative ~1e-7 .. 1e-6) and by the activations whose two
# values fall on opposite sides of a bfloat16 rounding boundary: those differ by one bfloat16 ulp
# (2^-8 relative).  A relative perturbation d of a layer's sums flips a fraction ~d / 2^-8 of its
# activations, which perturbs the layer output by ~2^-8 sqrt(d / 2^-8); iterating from d ~ 1e-6
# gives ~6e-5 after one rounded layer, ~5e-4 after two, ~1.4e-3 after three, tending to 2^-8.
# With two layers (one rounded activation) the bar is 1e-4; deeper networks get 1e-2 for the
# output and 4e-2 for the gradients, whose dZ roundings add a second cascade (bound ~2 L 2^-8;
# measured up to 1.2e-2 for the first layer of six).  A wrong tap, channel or layout gives O(1).
# Exactness itself is pinned by the integer-data tests below.
def tolerances(L):
    """(output rel L2, gradient rel L2, loss rel) for a network of L layers on random data."""
    return (1e-4, 1e-4, 1e-6) if L <= 2 else (1e-2, 4e-2, 1e-4)


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _params(C, L, seed, last_scale=1.0, bias=0.05):
    """He-uniform weights for every layer (the last one scaled) and small random biases."""
    parts = []
    for l, (ci, co, nb) in enumerate(cn.layer_shapes(C, L)):
        lim = np.sqrt(6.0 / (9 * ci)) * (last_scale if l == L - 1 else 1.0)
        parts.append(inputs.uniform(seed * 100 + 2 * l, 9 * ci * co, -lim, lim))
        b = np.zeros(nb)
        b[:co] = inputs.uniform(seed * 100 + 2 * l + 1, co, -bias, bias)
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


S = cn.STATE_C  # phi, v_x, v_y, rho


def _state(B, H, W, seed, amp=1.0):
    s = inputs.uniform(seed, B * H * W * S, -amp, amp).reshape(B, H, W, S)
    return s.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


SHAPES = [  # B, H, W, C, L: full and partial 8 x 32 tiles, several tiles and samples, both widths
    (2, 16, 24, 64, 6),
    (1, 12, 8, 32, 3),
    (2, 3, 16, 64, 2),
    (3, 5, 32, 32, 4),
    (1, 33, 32, 64, 6),
    (1, 8, 16, 64, 3),
    (2, 17, 70, 64, 3),
    (1, 1, 32, 32, 2),
    (1, 2, 48, 64, 4),
]


ALPHA = (0.25, 2.0, 0.5, 4.0)


@pytest.mark.parametrize("B,H,W,C,L", SHAPES)
def test_forward_matches_oracle(B, H, W, C, L):
    import torch

    _note(f"forward B={B} H={H} W={W} C={C} L={L}")
    p = _params(C, L, seed=B + H + W + C + L)
    s = _state(B, H, W, seed=7 + H)
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p)
    m.set_output_scale(ALPHA)
    out = torch.empty(B, H, W, S, dtype=torch.float32, device="cuda")
    m.forward(torch.from_numpy(s).cuda(), out)
    got = out.cpu().numpy().astype(np.float64)
    ref, _ = cn.forward(p.astype(np.float64), s.astype(np.float64), C, L, emulate_bf16=True, alpha=ALPHA)
    r = _rel(got - s, ref - s)
    _note(f"  residual rel L2 {r:.3e}")
    assert r < tolerances(L)[0]
    m.close()


def _integer_case(B, H, W, C, L, seed):
    """Integer state in [-2, 2], integer biases in [-1, 1], layer-0 weights in {-1, 0, 1} and later
    weights in {-1, 0, 1} with 1 in 64 nonzero."""
    u = inputs.uniform(seed, B * H * W * S).reshape(B, H, W, S)
    s = np.floor(5 * u) - 2
    parts = []
    for l, (ci, co, nb) in enumerate(cn.layer_shapes(C, L)):
        w = inputs.uniform(seed * 100 + 2 * l, 9 * ci * co)
        if l == 0:
            w = np.floor(3 * w) - 1
        else:
            w = np.where(w < 1 / 128, -1.0, np.where(w > 1 - 1 / 128, 1.0, 0.0))
        b = np.zeros(nb)
        b[:co] = np.floor(3 * inputs.uniform(seed * 100 + 2 * l + 1, co)) - 1
        parts += [w, b]
    return np.concatenate(parts), s


def _exactness_bound(p, s, C, L):
    """Largest sum of |products| + |bias| over all outputs of all layers (integers): below 2^24
    every partial sum is an exactly representable integer, in any order."""
    worst, a = 0.0, s
    for l, (Wl, bl) in enumerate(cn.unpack(p, C, L)):
        worst = max(worst, cn.conv(np.abs(a), np.abs(Wl if l == 0 else cn.bf16(Wl)), np.abs(bl)).max())
        z = cn.conv(a, Wl, bl)
        a = cn.bf16(np.maximum(z, 0.0))
    return worst


@pytest.mark.parametrize("B,H,W,C,L", SHAPES)
def test_forward_bit_exact_on_integer_data(B, H, W, C, L):
    """On integer data both sides compute every sum exactly and round the same exact values to
    bfloat16, so the outputs agree bit for bit."""
    import torch

    _note(f"integer forward B={B} H={H} W={W} C={C} L={L}")
    p, s = _integer_case(B, H, W, C, L, seed=B + 3 * H + W + L)
    assert _exactness_bound(p, s, C, L) < 2 ** 24
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p.astype(np.float32))
    m.set_output_scale(ALPHA)
    out = torch.empty(B, H, W, S, dtype=torch.float32, device="cuda")
    m.forward(torch.from_numpy(s.astype(np.float32)).cuda(), out)
    ref, _ = cn.forward(p, s, C, L, emulate_bf16=True, alpha=ALPHA)
    got = out.cpu().numpy().astype(np.float64)
    assert np.abs(ref - s).max() > 0
    assert np.array_equal(got, ref), np.abs(got - ref).max()
    m.close()


def _ambiguous(p, s, target, C, L):
    """Output-gradient entries within 1e-6 (relative) of a bfloat16 rounding midpoint, where the
    FP32 and FP64 values could round apart."""
    out, _ = cn.forward(p, s, C, L, emulate_bf16=True, alpha=ALPHA)
    v = 2.0 * (out - target) / np.asarray(ALPHA) / out.size
    return cn.bf16(v * (1 - 1e-6)) != cn.bf16(v * (1 + 1e-6))


def _backward_exactness(p, s, target, C, L):
    """On integer data: the number of ambiguous output-gradient values (see _ambiguous), and the
    largest ratio of sum |g| |W| to the grain of g over the input-gradient sums (below 2^24 they
    are exact)."""
    out, cache = cn.forward(p, s, C, L, emulate_bf16=True, alpha=ALPHA)
    v = 2.0 * (out - target) / np.asarray(ALPHA) / out.size
    ambiguous = int(np.sum(_ambiguous(p, s, target, C, L)))
    g, worst = cn.bf16(v), 0.0
    for l in range(L - 1, 0, -1):
        W = cache["layers"][l][0]
        nz = np.abs(g[g != 0])
        if nz.size == 0:
            break
        grain = 2.0 ** (np.floor(np.log2(nz.min())) - 7)
        S = sum(cn.shifted(np.abs(g), -dy, -dx) @ np.abs(W[t]).T for t, (dy, dx) in enumerate(cn.taps()))
        worst = max(worst, S.max() / grain)
        da = sum(cn.shifted(g, -dy, -dx) @ W[t].T for t, (dy, dx) in enumerate(cn.taps()))
        g = cn.bf16(da * (cache["acts"][l] > 0))
    return ambiguous, worst


@pytest.mark.parametrize("B,H,W,C,L", SHAPES)
def test_backward_on_integer_data(B, H, W, C, L):
    """Integer data (see above) and an integer target: both sides hold the same bfloat16 output
    gradient and compute the input gradients exactly, so the weight and bias gradients differ
    only by FP32 accumulation."""
    import torch

    _note(f"integer backward B={B} H={H} W={W} C={C} L={L}")
    p, s = _integer_case(B, H, W, C, L, seed=B + 3 * H + W + L)
    tgt = s + np.floor(3 * inputs.uniform(99 + W, s.size)).reshape(s.shape) - 1
    for _ in range(4):  # move targets off the few rounding midpoints (when 4 P is not a power of two)
        m = _ambiguous(p, s, tgt, C, L)
        if not m.any():
            break
        tgt = tgt + m
    amb, worst = _backward_exactness(p, s, tgt, C, L)
    assert amb == 0 and worst < 2 ** 24, (amb, worst)
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p.astype(np.float32))
    m.set_output_scale(ALPHA)
    m.forward(torch.from_numpy(s.astype(np.float32)).cuda())
    loss = m.backward(torch.from_numpy(tgt.astype(np.float32)).cuda())
    g = m.grads().astype(np.float64)
    _, cache = cn.forward(p, s, C, L, emulate_bf16=True, alpha=ALPHA)
    gref, lref = cn.backward(cache, tgt, C, L)
    assert abs(loss - lref) <= 1e-6 * lref
    o = 0
    for l, (ci, co, nb) in enumerate(cn.layer_shapes(C, L)):
        nw = 9 * ci * co
        rw = _rel(g[o:o + nw], gref[o:o + nw])
        rb = _rel(g[o + nw:o + nw + co], gref[o + nw:o + nw + co])
        _note(f"  layer {l}: dW rel L2 {rw:.3e}, db rel L2 {rb:.3e}")
        assert rw < 1e-5 and rb < 1e-5, l
        o += nw + nb
    m.close()


@pytest.mark.parametrize("B,H,W,C,L", SHAPES)
def test_backward_matches_oracle(B, H, W, C, L):
    import torch

    _note(f"backward B={B} H={H} W={W} C={C} L={L}")
    p = _params(C, L, seed=3 + B + H + W + C + L)
    s = _state(B, H, W, seed=17 + H)
    tgt = (s + _state(B, H, W, seed=27 + W, amp=0.3)).astype(np.float32)
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p)
    m.set_output_scale(ALPHA)
    m.forward(torch.from_numpy(s).cuda())
    loss = m.backward(torch.from_numpy(tgt).cuda())
    g = m.grads().astype(np.float64)
    out, cache = cn.forward(p.astype(np.float64), s.astype(np.float64), C, L, emulate_bf16=True, alpha=ALPHA)
    gref, lref = cn.backward(cache, tgt.astype(np.float64), C, L)
    _, gtol, ltol = tolerances(L)
    assert abs(loss - lref) <= ltol * lref
    o = 0
    for l, (ci, co, nb) in enumerate(cn.layer_shapes(C, L)):
        nw = 9 * ci * co
        rw = _rel(g[o:o + nw], gref[o:o + nw])
        rb = _rel(g[o + nw:o + nw + co], gref[o + nw:o + nw + co])
        _note(f"  layer {l}: dW rel L2 {rw:.3e}, db rel L2 {rb:.3e}")
        assert rw < gtol and rb < gtol, l
        assert np.all(g[o + nw + co:o + nw + nb] == 0)  # bias padding
        o += nw + nb
    m.close()


def test_full_size_forward_matches_oracle():
    """The 256 x 256, 64-channel, 6-layer network of the benchmark, one box."""
    import torch

    _note("forward 256x256 C=64 L=6")
    C, L = 64, 6
    p = _params(C, L, seed=5, last_scale=0.1)
    ph, rho, ux, uy = inputs.smooth_state(256, 256, seed=3)
    s = np.stack([ph, ux * 20, uy * 20, (rho - 1) * 50], axis=-1)[None].astype(np.float32)
    m = net.Surrogate(1, 256, 256, channels=C, layers=L)
    m.set_params(p)
    out = torch.empty(1, 256, 256, S, dtype=torch.float32, device="cuda")
    m.forward(torch.from_numpy(s).cuda(), out)
    got = out.cpu().numpy().astype(np.float64)
    ref, _ = cn.forward(p.astype(np.float64), s.astype(np.float64), C, L, emulate_bf16=True)
    r = _rel(got - s, ref - s)
    _note(f"  residual rel L2 {r:.3e}")
    assert r < tolerances(L)[0]
    m.close()


@pytest.mark.parametrize("B,H,W,C,L", [(2, 40, 70, 64, 6), (1, 12, 40, 32, 3)])
def test_gradients_are_deterministic(B, H, W, C, L):
    """Every reduction of the backward pass runs in a fixed order (per-unit partials summed in
    unit order, fixed trees, no atomics): two passes on the same data, and a second network with
    the same parameters, give bitwise equal gradients and losses."""
    import torch

    _note(f"deterministic gradients B={B} H={H} W={W} C={C} L={L}")
    p = _params(C, L, seed=21)
    s = torch.from_numpy(_state(B, H, W, seed=22)).cuda()
    tgt = torch.from_numpy(_state(B, H, W, seed=23, amp=0.5)).cuda()
    out = torch.empty_like(s)
    runs = []
    for _ in range(2):
        m = net.Surrogate(B, H, W, channels=C, layers=L)
        m.set_params(p)
        m.set_output_scale(ALPHA)
        for _ in range(2):
            m.forward(s, out)
            loss = m.backward(tgt)
            runs.append((m.grads(), loss))
        m.close()
    for g, loss in runs[1:]:
        assert np.array_equal(g, runs[0][0]) and loss == runs[0][1]
    assert np.abs(runs[0][0]).max() > 0


@pytest.mark.parametrize("B,H,W", [(32, 64, 96), (8, 256, 256)])
def test_batched_pass_equals_single_sample_passes(B, H, W):
    """A batch large enough that every kernel's workgroups take several tiles in turn (32 samples
    of 64 x 96: 768 tiles; 8 of 256 x 256, the training batch: 2048 tiles; grids of 256 to 1024),
    against the same samples one at a time: the forward outputs are equal bit for bit, and the
    batch's weight and bias gradients equal the mean of the single-sample ones up to FP32 summation
    order (a batch of 2^k scales each sample's output gradient by exactly 2^-k, so every BF16
    rounding on the way scales with it)."""
    import torch

    _note(f"batched vs single-sample passes B={B} H={H} W={W}")
    C, L = 64, 6
    p = _params(C, L, seed=51)
    s = _state(B, H, W, seed=52)
    tgt = (s + _state(B, H, W, seed=53, amp=0.3)).astype(np.float32)
    mb = net.Surrogate(B, H, W, channels=C, layers=L)
    mb.set_params(p)
    mb.set_output_scale(ALPHA)
    out = torch.empty(B, H, W, S, dtype=torch.float32, device="cuda")
    mb.forward(torch.from_numpy(s).cuda(), out)
    loss_b = mb.backward(torch.from_numpy(tgt).cuda())
    ob, gb = out.cpu().numpy(), mb.grads().astype(np.float64)
    mb.close()
    m1 = net.Surrogate(1, H, W, channels=C, layers=L)
    m1.set_params(p)
    m1.set_output_scale(ALPHA)
    o1 = torch.empty(1, H, W, S, dtype=torch.float32, device="cuda")
    gsum, lsum = np.zeros_like(gb), 0.0
    for b in range(B):
        m1.forward(torch.from_numpy(s[b:b + 1].copy()).cuda(), o1)
        lsum += m1.backward(torch.from_numpy(tgt[b:b + 1].copy()).cuda())
        assert np.array_equal(o1.cpu().numpy()[0], ob[b]), b
        gsum += m1.grads().astype(np.float64)
    m1.close()
    g1 = gsum / B
    rel = np.linalg.norm(gb - g1) / np.linalg.norm(g1)
    _note(f"  grads rel L2 {rel:.2e}, loss {loss_b:.6e} vs {lsum / B:.6e}")
    assert rel < 1e-5
    assert abs(loss_b - lsum / B) <= 1e-5 * abs(loss_b)


def test_training_steps_follow_the_oracle():
    """Five Adam iterations (forward, backward, update) of the kernels against the same
    iterations of the oracle, each started from the device parameters."""
    import torch

    _note("training parity")
    B, H, W, C, L = 2, 8, 32, 32, 2  # one rounded activation layer: the tight tier
    p = _params(C, L, seed=61, last_scale=0.2)
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p)
    m.set_output_scale(ALPHA)
    mm, vv = np.zeros(p.size), np.zeros(p.size)
    losses = []
    for t in range(1, 6):
        s = _state(B, H, W, seed=70 + t)
        tgt = (s + _state(B, H, W, seed=80 + t, amp=0.2) * np.array(ALPHA)).astype(np.float32)
        pr = m.params().astype(np.float64)
        m.forward(torch.from_numpy(s).cuda())
        loss = m.backward(torch.from_numpy(tgt).cuda())
        m.adam(3e-3, 0.9, 0.999, 1e-8)
        _, cache = cn.forward(pr, s.astype(np.float64), C, L, emulate_bf16=True, alpha=ALPHA)
        g, lref = cn.backward(cache, tgt.astype(np.float64), C, L)
        _note(f"  iter {t}: loss {loss:.6e} oracle {lref:.6e}")
        assert abs(loss - lref) <= tolerances(L)[2] * lref
        pref, mm, vv = cn.adam(pr, g, mm, vv, t, 3e-3, 0.9, 0.999, 1e-8)
        got = m.params().astype(np.float64)
        # Adam moves each parameter by about lr; compare the step taken
        step_rel = np.linalg.norm((got - pr) - (pref - pr)) / np.linalg.norm(pref - pr)
        _note(f"  iter {t}: step rel L2 {step_rel:.2e}")
        assert step_rel < 1e-3
        losses.append(loss)


@pytest.mark.parametrize("C,L", [(64, 6), (32, 3)])
def test_adam_updates_the_packs_as_a_fresh_pack(C, L):
    """Adam writes the updated weights into the BF16 packs in the same pass once they exist; the
    next forward must equal a forward from packs made anew from the same parameters, bit for bit."""
    import torch

    _note(f"adam packs C={C} L={L}")
    B, H, W = 2, 16, 40
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(_params(C, L, seed=91))
    m.set_output_scale(ALPHA)
    s = torch.from_numpy(_state(B, H, W, seed=92)).cuda()
    tgt = torch.from_numpy(_state(B, H, W, seed=93)).cuda()
    for _ in range(3):  # the first forward makes the packs; the later updates go through them
        m.forward(s)
        m.backward(tgt, want_loss=False)
        m.adam(1e-2, 0.9, 0.999, 1e-8)
    out = torch.empty(B, H, W, S, dtype=torch.float32, device="cuda")
    m.forward(s, out)
    a = out.cpu().numpy().copy()
    m.set_params(m.params())  # packs made again on the next forward
    m.forward(s, out)
    assert np.array_equal(a, out.cpu().numpy())
    m.close()


def test_adam_matches_oracle():
    import torch

    _note("adam")
    B, H, W, C, L = 1, 8, 8, 32, 3
    p = _params(C, L, seed=41)
    s = _state(B, H, W, seed=42)
    tgt = (s * 0.9).astype(np.float32)
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(p)
    pr = p.astype(np.float64)
    mm, vv = np.zeros_like(pr), np.zeros_like(pr)
    for t in range(1, 4):
        m.forward(torch.from_numpy(s).cuda())
        m.backward(torch.from_numpy(tgt).cuda(), want_loss=False)
        g = m.grads().astype(np.float64)
        m.adam(1e-3, 0.9, 0.999, 1e-8)
        pr, mm, vv = cn.adam(pr, g, mm, vv, t, 1e-3, 0.9, 0.999, 1e-8)
        got = m.params().astype(np.float64)
        # FP32 update of FP32 parameters: a few float32 ulps of the parameters
        assert np.max(np.abs(got - pr)) <= 4e-7 * max(1.0, np.abs(pr).max()), t
        pr = got  # continue from the device parameters (their FP32 rounding)
    m.close()


def test_zero_network_is_identity_and_planes_roundtrip():
    import torch

    _note("planes roundtrip")
    H, W = 12, 16
    us, rs = 0.05, 0.02
    m = net.Surrogate(1, H, W, channels=32, layers=3)
    m.set_params(np.zeros(m.nparams, dtype=np.float32))
    ph, rho, ux, uy = inputs.smooth_state(W, H, seed=9)
    planes = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (ph, ux, uy, rho)]
    outs = [torch.empty_like(planes[0]) for _ in range(4)]
    m.forward_planes(*planes, us, rs, *outs)
    # FP32 round trip of the scaled state
    inv_u, inv_r = np.float32(1 / us), np.float32(1 / rs)
    expect = [ph.astype(np.float32).astype(np.float64),
              (ux.astype(np.float32) * inv_u).astype(np.float64) * us,
              (uy.astype(np.float32) * inv_u).astype(np.float64) * us,
              1.0 + ((rho - 1.0).astype(np.float32) * inv_r).astype(np.float64) * rs]
    for e, b in zip(expect, outs):
        assert np.array_equal(b.cpu().numpy(), e)
    st = torch.empty(1, H, W, S, dtype=torch.float32, device="cuda")
    m.state_from_planes(*planes, us, rs, st)
    st = st.cpu().numpy()[0]
    assert np.allclose(st[..., 0], ph, rtol=1e-7)
    assert np.allclose(st[..., 1], ux / us, rtol=1e-6)
    assert np.allclose(st[..., 2], uy / us, rtol=1e-6)
    assert np.allclose(st[..., 3], (rho - 1) / rs, rtol=1e-6)
    m.close()


@pytest.mark.parametrize("B,H,W,C,L", [(1, 64, 64, 64, 6), (2, 13, 40, 32, 3), (2, 3, 20, 64, 3), (1, 1, 8, 64, 5),
                                       (1, 17, 70, 64, 4), (1, 256, 256, 64, 6)])
def test_forward_planes_equals_state_forward(B, H, W, C, L):
    """The planes path converts inside the first and last layers and, with 64 channels, runs the
    conv layers in fused pairs (the activation between them stays on chip, its halo recomputed);
    it must give bit for bit the state path's output converted back to planes (v = u_scale v',
    rho = 1 + rho_scale rho'), also when the output planes are the input planes.  The shapes
    cover a paired and a single last layer, ragged tiles, and boxes smaller than the halo."""
    import torch

    _note(f"forward_planes vs forward {B}x{H}x{W} C={C} L={L}")
    us, rs = 0.03, 0.01
    m = net.Surrogate(B, H, W, channels=C, layers=L)
    m.set_params(_params(C, L, seed=5, last_scale=0.1))
    m.set_output_scale(ALPHA)
    fields = [inputs.smooth_state(W, H, seed=20 + b) for b in range(B)]
    ph, rho, ux, uy = (np.stack([f[k] for f in fields]) for k in range(4))
    planes = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (ph, ux, uy, rho)]
    st = torch.empty(B, H, W, S, dtype=torch.float32, device="cuda")
    m.state_from_planes(*planes, us, rs, st)
    out = torch.empty_like(st)
    m.forward(st, out)
    out = out.cpu().numpy().astype(np.float64)
    expect = [out[..., 0], out[..., 1] * us, out[..., 2] * us, 1.0 + out[..., 3] * rs]
    outs = [torch.empty_like(planes[0]) for _ in range(4)]
    m.forward_planes(*planes, us, rs, *outs)
    for e, b in zip(expect, outs):
        assert np.array_equal(b.cpu().numpy(), e)
    m.forward_planes(*planes, us, rs, *planes)  # in place
    for e, b in zip(expect, planes):
        assert np.array_equal(b.cpu().numpy(), e)
    m.close()


def _dihedral(ph, vx, vy, rho, k):
    """Reference symmetry k of the square on [n, n] planes: transpose, then flip y, then flip x,
    the velocity swapped and negated with the grid."""
    if k & 4:
        ph, vx, vy, rho = ph.T, vy.T, vx.T, rho.T
    if k & 2:
        ph, vx, vy, rho = ph[::-1], vx[::-1], -vy[::-1], rho[::-1]
    if k & 1:
        ph, vx, vy, rho = ph[:, ::-1], -vx[:, ::-1], vy[:, ::-1], rho[:, ::-1]
    return ph, vx, vy, rho


@pytest.mark.parametrize("h,w,k", [(12, 12, k) for k in range(8)] + [(40, 40, k) for k in range(8)] +
                         [(40, 72, k) for k in range(4)])
def test_gather_states_applies_the_symmetry(h, w, k):
    """The training batch kernel equals, bit for bit, the symmetry applied to the FP64 planes
    followed by the state conversion, for every element of the group (flips only on a
    rectangle): one partial 32 x 32 tile, and several tiles with ragged edges."""
    import torch

    _note(f"gather states {h}x{w} k={k}")
    nf, us, rs = 5, 0.03, 0.01
    frames = np.stack([np.stack(inputs.smooth_state(w, h, seed=40 + f)) for f in range(nf)], axis=1)
    frames = frames[[0, 2, 3, 1]]  # smooth_state gives (phi, rho, ux, uy): reorder to (phi, vx, vy, rho)
    m = net.Surrogate(2, h, w, channels=32, layers=2)
    st = torch.empty(2, h, w, S, dtype=torch.float32, device="cuda")
    idx = [3, 1]
    m.gather_states(torch.from_numpy(np.ascontiguousarray(frames)).cuda(), idx, k, us, rs, st)
    got = st.cpu().numpy()
    inv_u, inv_r = np.float32(1 / us), np.float32(1 / rs)
    for b, f in enumerate(idx):
        ph, vx, vy, rho = _dihedral(*frames[:, f], k)
        expect = np.stack([ph.astype(np.float32), vx.astype(np.float32) * inv_u, vy.astype(np.float32) * inv_u,
                           (rho - 1.0).astype(np.float32) * inv_r], axis=-1)
        assert np.array_equal(got[b], expect)
    m.close()


def test_gather_states_rejects_bad_arguments():
    import torch

    m = net.Surrogate(2, 8, 12, channels=32, layers=2)
    frames = torch.zeros(4, 3, 8, 12, dtype=torch.float64, device="cuda")
    st = torch.empty(2, 8, 12, S, dtype=torch.float32, device="cuda")
    m.gather_states(frames, [0, 2], 3, 1.0, 1.0, st)  # flips only: fine on a rectangle
    for idx, k in (([0, 3], 0), ([0, -1], 0), ([0, 1], 4), ([0, 1], 8)):
        with pytest.raises(lbcm.LbcmError):
            m.gather_states(frames, idx, k, 1.0, 1.0, st)
    m.close()


def _hybrid_setup(threshold, n=64, J=4, K=8):
    import torch

    lat = lbcm.Lattice(n, n, precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    lat.init(inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08)))
    m = net.Surrogate(1, n, n, channels=32, layers=3, stream=lat.stream)
    m.set_params(np.zeros(m.nparams, dtype=np.float32))  # identity jumps
    hy = net.Hybrid(lat, m, steps_per_jump=K, jumps_per_check=J, u_scale=1e-3, rho_scale=1e-3, threshold=threshold)
    return lat, m, hy, torch


@pytest.mark.parametrize("threshold", [np.inf, 0.0])
def test_hybrid_bookkeeping_with_identity_network(threshold):
    _note(f"hybrid threshold={threshold}")
    J, K = 4, 8
    lat, m, hy, torch = _hybrid_setup(threshold, J=J, K=K)
    hy.advance(3)
    st = hy.stats()
    assert st["steps"] == 3 * J * K and st["checks"] >= 1
    if np.isinf(threshold):
        assert st["failed_checks"] == 0 and st["checks"] == 3
        assert st["jumps"] == 3 * (J - 1) and st["lb_steps_run"] == 3 * K
    else:
        # window 1 fails and is redone by the lattice, window 2 is a plain window, window 3 fails
        assert st["checks"] == 2 and st["failed_checks"] == 2 and st["jumps"] == 0
        assert st["lb_steps_run"] == 2 * (K + J * K) + J * K
    assert np.isfinite(lat.fields()["phi"]).all()
    hy.close()
    m.close()
    lat.close()


def test_hybrid_reports_divergence_of_the_lattice():
    """A caller's lattice created with check_every > 0 turns a non-finite state into
    LBCM_EDIVERGED from lbcm_hybrid_advance (here a NaN in the starting phi: the check rejects the
    window, and the lattice's own steps over it report the divergence)."""
    _note("hybrid divergence")
    n = 64
    lat = lbcm.Lattice(n, n, precision="fp32", check_every=4, a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    phi = inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08))
    phi[10, 10] = np.nan
    lat.init(phi)
    m = net.Surrogate(1, n, n, channels=32, layers=3, stream=lat.stream)
    m.set_params(np.zeros(m.nparams, dtype=np.float32))  # identity jumps
    hy = net.Hybrid(lat, m, steps_per_jump=8, jumps_per_check=4, u_scale=1e-3, rho_scale=1e-3, threshold=0.0)
    with pytest.raises(lbcm.LbcmError) as e:
        hy.advance(2)
    assert e.value.code == lbcm.LBCM_EDIVERGED
    hy.close()
    m.close()
    lat.close()


def test_hybrid_check_error_is_the_relative_phi_l2():
    """With identity jumps the check compares the window's starting phi (after the FP32 round
    trip of a jump) with K lattice steps from equilibrium populations of that state; recompute it
    with a second lattice (u_scale = rho_scale = 1e-3 here)."""
    _note("hybrid check error")
    J, K, n, us = 2, 8, 64, 1e-3
    lat, m, hy, torch = _hybrid_setup(np.inf, n=n, J=J, K=K)
    f0 = lat.fields()
    hy.advance(1)
    e = hy.stats()["last_error"]
    # one identity jump: phi -> float32, v -> float32(float32(v) * float32(1 / u_scale)) * u_scale,
    # rho -> 1 + float32(float32(rho - 1) * float32(1 / rho_scale)) * rho_scale
    inv = np.float32(1.0 / us)
    phi = f0["phi"].astype(np.float32).astype(np.float64)
    ux = (f0["ux"].astype(np.float32) * inv).astype(np.float64) * us
    uy = (f0["uy"].astype(np.float32) * inv).astype(np.float64) * us
    rho = 1.0 + ((f0["rho"] - 1.0).astype(np.float32) * inv).astype(np.float64) * us
    ref = lbcm.Lattice(n, n, precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    ref.init(phi, rho, ux, uy)
    ref.step(K)
    phi_lb = ref.fields()["phi"]
    expect = np.linalg.norm(phi - phi_lb) / np.linalg.norm(phi_lb)
    _note(f"  check error {e:.6e} expected {expect:.6e}")
    assert expect > 0 and abs(e - expect) <= 1e-12 * expect
    # the window ends in the lattice Boltzmann result of the checked jump
    assert np.array_equal(lat.fields()["phi"], phi_lb)
    for o in (hy, m, lat, ref):
        o.close()


@pytest.mark.parametrize("mode", ["accept", "reject", "mixed"])
def test_hybrid_one_call_equals_window_by_window(mode):
    """Inside one advance call an accepted window hands its check's lattice fields to the next
    window and the next window's first jumps are launched before the decision; the result must
    equal, bit for bit and in every statistic, the same windows advanced one call at a time
    (where neither shortcut applies).  A random network makes the jumps non-trivial; "mixed"
    puts the threshold at the median error of a first run."""
    _note(f"hybrid one call vs window by window: {mode}")
    J, K, n, W = 4, 8, 64, 6

    def run(threshold, calls):
        lat, m, hy, torch = _hybrid_setup(threshold, n=n, J=J, K=K)
        m.set_params(_params(32, 3, seed=11, last_scale=0.02))
        errs = []
        for c in calls:
            hy.advance(c)
            errs.append(hy.stats()["last_error"])
        out = (lat.get_state(), hy.stats(), errs)
        for o in (hy, m, lat):
            o.close()
        return out

    threshold = {"accept": np.inf, "reject": 0.0}.get(mode)
    if threshold is None:
        threshold = float(np.median(run(np.inf, [1] * W)[2]))
    s1, st1, _ = run(threshold, [W])
    s2, st2, _ = run(threshold, [1] * W)
    _note(f"  threshold {threshold:.3e}: {st1['checks']} checks, {st1['failed_checks']} failed")
    assert st1 == st2
    assert np.array_equal(s1, s2)
    if mode == "accept":
        assert st1["failed_checks"] == 0 and st1["checks"] == W
    if mode == "reject":
        assert st1["jumps"] == 0


def test_rejected_window_continues_the_exact_lattice_state():
    """A rejected window leaves the caller's lattice exactly where a plain run of the same number
    of steps from the same populations would be: the checks run on a scratch lattice."""
    _note("hybrid exact fallback")
    J, K, n = 2, 8, 64
    lat, m, hy, torch = _hybrid_setup(0.0, n=n, J=J, K=K)
    lat.step(5)  # non-equilibrium populations at the window start
    ref = lbcm.Lattice(n, n, precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    ref.init(inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08)))
    ref.step(5)
    hy.advance(2)  # a rejected window, then a plain one
    ref.step(2 * J * K)
    st = hy.stats()
    assert st["failed_checks"] == 1 and st["checks"] == 1 and st["jumps"] == 0
    assert np.array_equal(lat.get_state(), ref.get_state())
    assert lbcm.lbcm_step_count(lat.h) == 5 + 2 * J * K
    for o in (hy, m, lat, ref):
        o.close()


@pytest.mark.parametrize("threshold", [np.inf, 0.0])
def test_audited_windows_measure_the_accumulated_error(threshold):
    """With every window audited (identity jumps) the lattice runs each window with the plain step
    from its own populations, so after W windows it equals a plain run of W J K steps bit for bit,
    whatever the outcome; the audited error is ||phi_start' - phi_end|| / ||phi_end|| of the
    window (phi_start' the starting phi after the FP32 round trip of the identity jumps), the
    largest over the windows, recomputed here on the host; with a zero threshold every audit fails
    and the back-off then runs plain windows, which are not audited."""
    _note(f"hybrid audits threshold={threshold}")
    J, K, n, W = 2, 8, 64, 3
    lat, m, hy, torch = _hybrid_setup(threshold, n=n, J=J, K=K)
    net.lbcm_hybrid_set_audit(hy.h, 1)
    ref = lbcm.Lattice(n, n, precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    ref.init(inputs.droplet(n, n, 16, inputs.interface_width(0.04, 0.08)))
    want = 0.0
    audited = 0
    st = hy.stats()
    for w in range(W):
        p0 = ref.fields()["phi"].astype(np.float32).astype(np.float64)
        ref.step(J * K)
        before = hy.stats()
        hy.advance(1)
        st = hy.stats()
        if st["audits"] > before["audits"]:
            audited += 1
            p1 = ref.fields()["phi"]
            want = max(want, np.linalg.norm(p0 - p1) / np.linalg.norm(p1))
        assert np.array_equal(lat.get_state(), ref.get_state()), w
    _note(f"  {st}")
    assert st["audits"] == audited and st["checks"] == 0 and st["jumps"] == 0
    assert st["lb_steps_run"] == st["steps"] == W * J * K
    assert abs(st["max_audited_error"] - want) <= 1e-12 * want
    if np.isinf(threshold):
        assert audited == W and st["failed_audits"] == 0
    else:
        assert audited == 2 and st["failed_audits"] == 2  # window 2 is a back-off plain window
    with pytest.raises(lbcm.LbcmError):
        net.lbcm_hybrid_set_audit(hy.h, -1)
    for o in (hy, m, lat, ref):
        o.close()


def test_copy_state_is_exact():
    _note("copy state")
    n = 48
    kw = dict(precision="fp32", a=0.04, gamma=0.08, mobility=0.1, nu_l=0.05, nu_g=0.05)
    a = lbcm.Lattice(n, n, **kw)
    b = lbcm.Lattice(n, n, **kw)
    a.init(inputs.droplet(n, n, 12, 2.0))
    b.init(inputs.droplet(n, n, 8, 2.0))
    a.step(7)
    lbcm.lbcm_copy_state(b.h, a.h, 7)
    assert np.array_equal(a.get_state(), b.get_state())
    a.step(9)
    b.step(9)
    assert np.array_equal(a.get_state(), b.get_state()) and lbcm.lbcm_step_count(b.h) == 16
    c = lbcm.Lattice(n + 1, n, **kw)
    c.init(np.zeros((n, n + 1)))
    with pytest.raises(lbcm.LbcmError):
        lbcm.lbcm_copy_state(c.h, a.h, 0)
    for o in (a, b, c):
        o.close()


def test_trained_network_gains_over_the_method_without_it():
    """Train the 6-layer, 64-channel network briefly on lattice Boltzmann runs of two-droplet
    coalescence (a 128 x 128 version of the workload) and check what it gains: on a held-out
    run its one-jump phi error is well below that of keeping the state (the method without the
    network must run all 16 steps to do better), and in the hybrid the lattice runs fewer steps
    than the simulated time while every accepted window meets the phi threshold."""
    from paper_1803_11345_amd import train as T

    _note("trained network gain")
    n, K = 128, 16
    cases = inputs.coalescence_cases(6, seed=23, rmin=10.0, rmax=20.0)
    model, info = T.fit(n, K, T.dataset_runs(n, (), cases[:4]), 150, iters=600, batch=8)
    m1 = T.single_box(model)
    model.close()
    frames, pairs = T.build_dataset(n, K, T.dataset_runs(n, (), cases[4:5]), 150)
    e = T.jump_errors(m1, frames, pairs[5:], info["u_scale"], info["rho_scale"])
    _note(f"  one jump phi error: net {e['phi_net'].mean():.3e}, keep {e['phi_keep'].mean():.3e}")
    assert e["phi_net"].mean() < 0.5 * e["phi_keep"].mean()
    h = T.hybrid_vs_lb(m1, T.coalescence_phi(n, cases[5]), info["u_scale"], info["rho_scale"], 12)
    _note(f"  hybrid: {h}")
    assert h["accepted_jumps"] > 0 and h["lb_steps_run"] < h["steps"]
    assert h["max_accepted_phi_error"] <= 1e-2
    # the trajectory at equal simulated time stays close to plain lattice Boltzmann
    assert h["final_phi_rel_l2_vs_lb"] < 0.1
    m1.close()
