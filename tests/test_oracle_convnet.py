"""Pins of the FP64 network oracle (oracle/convnet.py) against what fixes it independently:
a library correlation, brute-force sums, finite differences of the loss, torch's bfloat16
conversion and torch's Adam, and the symmetries of a circular convolution."""
import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import convnet as cn
from paper_1803_11345_amd import inputs


def _rand(seed, shape, lo=-1.0, hi=1.0):
    return inputs.uniform(seed, int(np.prod(shape)), lo, hi).reshape(shape)


def _params(seed, C, L, scale=0.4):
    return cn.pack([(_rand(seed + 10 * l, (9, ci, co), -scale, scale), _rand(seed + 10 * l + 1, (co,), -0.1, 0.1))
                    for l, (ci, co, _) in enumerate(cn.layer_shapes(C, L))], C, L)


def test_param_count_of_the_six_layer_64_channel_net():
    # 4->64, four 64->64, 64->4; the last bias is padded to 32 entries
    assert cn.param_count(64, 6) == (9 * 4 * 64 + 64) + 4 * (9 * 64 * 64 + 64) + (9 * 64 * 4 + 32)


def test_pack_unpack_roundtrip():
    p = _params(3, 5, 4)
    assert np.array_equal(cn.pack(cn.unpack(p, 5, 4), 5, 4), p)


def test_bf16_matches_torch_round_to_nearest_even():
    x = _rand(11, (4000,), -3.0, 3.0) * np.exp(_rand(12, (4000,), -20, 20))
    # exact ties of the bfloat16 grid (odd and even lower halves) and values just beside them
    base = np.array([1.0, 1.0 + 2 ** -7, -1.5, 3.0 + 2 ** -6], dtype=np.float64)
    ties = np.concatenate([base + 2 ** -8 * np.abs(base), base + 2 ** -8 * np.abs(base) * (1 + 2 ** -20)])
    for v in (x, ties):
        ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(cn.bf16(v), ref)


def test_conv_matches_scipy_wrap_correlation():
    B, H, W, ci, co = 2, 7, 5, 3, 4
    a = _rand(21, (B, H, W, ci))
    Wt = _rand(22, (9, ci, co))
    b = _rand(23, (co,))
    z = cn.conv(a, Wt, b)
    ref = np.zeros_like(z)
    for n in range(B):
        for o in range(co):
            ref[n, :, :, o] = b[o] + sum(scipy.ndimage.correlate(a[n, :, :, i], Wt[:, i, o].reshape(3, 3), mode="wrap")
                                         for i in range(ci))
    assert np.allclose(z, ref, rtol=0, atol=1e-13)


def test_conv_brute_force():
    B, H, W, ci, co = 1, 4, 3, 2, 2
    a = _rand(31, (B, H, W, ci))
    Wt = _rand(32, (9, ci, co))
    b = _rand(33, (co,))
    z = cn.conv(a, Wt, b)
    for y in range(H):
        for x in range(W):
            for o in range(co):
                s = b[o]
                for ky in range(3):
                    for kx in range(3):
                        for i in range(ci):
                            s += a[0, (y + ky - 1) % H, (x + kx - 1) % W, i] * Wt[3 * ky + kx, i, o]
                assert abs(z[0, y, x, o] - s) < 1e-13


def test_zero_network_is_the_identity():
    s = _rand(41, (2, 6, 5, 4))
    out, _ = cn.forward(np.zeros(cn.param_count(8, 4)), s, 8, 4)
    assert np.array_equal(out, s)


def test_forward_commutes_with_circular_shifts():
    C, L = 6, 4
    p = _params(51, C, L)
    s = _rand(52, (1, 9, 8, 4))
    out, _ = cn.forward(p, s, C, L)
    out2, _ = cn.forward(p, np.roll(s, (2, -3), axis=(1, 2)), C, L)
    assert np.allclose(out2, np.roll(out, (2, -3), axis=(1, 2)), rtol=0, atol=1e-13)


@pytest.mark.parametrize("alpha", [(1.0, 1.0, 1.0, 1.0), (0.01, 0.3, 2.0, 0.05)])
def test_gradient_matches_central_differences(alpha):
    C, L = 4, 3
    p = _params(61, C, L)
    s = _rand(62, (2, 5, 6, 4))
    target = s + _rand(63, s.shape, -0.2, 0.2) * np.asarray(alpha)
    out, cache = cn.forward(p, s, C, L, alpha=alpha)
    g, l0 = cn.backward(cache, target, C, L)
    assert abs(l0 - cn.loss(out, target, alpha)) < 1e-15
    # 40 random entries, plus every real bias entry and the first weight of every layer
    idx = list((inputs.splitmix64(64, 40) % np.uint64(p.size)).astype(np.int64))
    o = 0
    for ci, co, nb in cn.layer_shapes(C, L):
        idx += [o] + list(range(o + 9 * ci * co, o + 9 * ci * co + co))
        o += 9 * ci * co + nb
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cn.loss(cn.forward(pp, s, C, L, alpha=alpha)[0], target, alpha)
              - cn.loss(cn.forward(pm, s, C, L, alpha=alpha)[0], target, alpha)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-10, (i, fd, g[i])
    # bias padding entries of the last layer have zero gradient
    assert np.all(g[-(cn.LAST_BIAS_PAD - cn.STATE_C):] == 0)


def test_gradient_of_every_layer_is_exercised():
    # every layer's weight block gets a nonzero gradient (no silently dropped layer)
    C, L = 4, 4
    p = _params(71, C, L)
    s = _rand(72, (1, 6, 6, 4))
    out, cache = cn.forward(p, s, C, L)
    g, _ = cn.backward(cache, s + 0.1, C, L)
    o = 0
    for ci, co, nb in cn.layer_shapes(C, L):
        assert np.abs(g[o:o + 9 * ci * co]).max() > 0
        o += 9 * ci * co + nb


def test_output_scale_multiplies_the_residual():
    C, L = 5, 3
    p = _params(75, C, L)
    s = _rand(76, (1, 6, 7, 4))
    a, _ = cn.forward(p, s, C, L)
    b, _ = cn.forward(p, s, C, L, alpha=(2.0, -1.0, 0.5, 4.0))
    assert np.allclose(b - s, (a - s) * np.array([2.0, -1.0, 0.5, 4.0]), rtol=0, atol=1e-14)


def test_emulated_bf16_forward_stays_close_to_fp64():
    C, L = 8, 4
    p = _params(81, C, L, scale=0.3)
    s = _rand(82, (1, 8, 8, 4))
    a, _ = cn.forward(p, s, C, L)
    b, _ = cn.forward(p, s, C, L, emulate_bf16=True)
    r = np.linalg.norm(b - a) / np.linalg.norm(a - s)
    assert 1e-5 < r < 5e-2  # BF16 operands: visible but small


def test_adam_matches_torch():
    n = 50
    p0 = _rand(91, (n,))
    grads = [_rand(92 + k, (n,)) for k in range(4)]
    w = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.99), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        w.grad = torch.tensor(g)
        opt.step()
        p, m, v = cn.adam(p, g, m, v, t, 1e-2, 0.9, 0.99, 1e-8)
    assert np.allclose(p, w.detach().numpy(), rtol=0, atol=1e-14)
