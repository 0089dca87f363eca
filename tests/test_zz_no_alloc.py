"""The allocation-free diagnostics entry point (lbcm_diag_state) through the C-ABI: its partial
sums live in the library's fixed device array instead of a handle's workspace.  Its results
must equal those of lbcm_diag on the same state bit for bit (the same kernels, launch shape and
reduction order), on two calls in a row with the second on a smaller lattice, so that nothing of
the first call's contents in the shared array leaks into the second."""
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


def _device_sets(lat, prec):
    """The lattice's raw state split into its f and g sets, each copied into its own device
    tensor (torch allocations are 256-byte aligned)."""
    import torch

    raw = lat.get_state()
    nf = 9 * lat.nx * lat.ny * {"fp64": 8, "fp32": 4, "fp16s": 2, "bf16s": 2}[prec]
    f = torch.from_numpy(raw[:nf].copy()).cuda()
    g = torch.from_numpy(raw[nf:].copy()).cuda()
    return f, g


CASES = [
    ("fp64", 130, 70, dict(bc_y=1, force_x=1e-5, wall_vx_top=2e-3, wall_gradient=0.03)),
    ("fp32", 67, 33, dict(force_y=-2e-5)),
    ("fp16s", 41, 29, dict(bc_y=1, force_x=1e-5)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_diag_state_equals_diag_on_two_calls(prec):
    import torch

    sizes = [(nx, ny, kw) for p, nx, ny, kw in CASES if p == prec]
    nx0, ny0, kw0 = sizes[0]
    calls = [(nx0, ny0, kw0), (max(1, nx0 // 2 - 3), max(1, ny0 // 2 - 1), kw0)]  # the second is smaller
    for nx, ny, kw in calls:
        print(f"case diag_state {prec} {nx}x{ny} {kw}", flush=True)
        phi, rho, ux, uy = inputs.smooth_state(nx, ny, seed=71 + nx)
        lat = lbcm.Lattice(nx, ny, precision=prec, nu_l=0.1, nu_g=0.02, **kw).init(phi, rho, ux, uy)
        lat.step(6)
        f_prev, _ = _device_sets(lat, prec)
        lat.step(1)
        want = lat.diag()  # max_du from the handle's spare pair (the state before the last step)
        f, g = _device_sets(lat, prec)
        got = lbcm.lbcm_diag_state(lat.params, f, g, f_prev, step=7)
        torch.cuda.synchronize()
        for k in want:
            assert got[k] == want[k], (k, got[k], want[k])
        assert want["max_du"] > 0 and np.isfinite(want["max_du"])
        plain = lbcm.lbcm_diag_state(lat.params, f, g)
        assert np.isnan(plain["max_du"])
        for k in ("sum_phi", "sum_abs_phi", "sum_rho", "sum_jx", "sum_jy", "max_u", "nonfinite"):
            assert plain[k] == want[k], k
        lat.close()


def test_diag_state_rejects_bad_arguments():
    import torch

    p = lbcm.make_params(16, 8, precision="fp32")
    buf = torch.zeros(9 * 16 * 8 * 4 + 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbcm.LbcmError) as e:
        lbcm.lbcm_diag_state(p, None, buf)
    assert e.value.code == lbcm.LBCM_EINVAL
    with pytest.raises(lbcm.LbcmError) as e:
        lbcm.lbcm_diag_state(p, buf.data_ptr() + 2, buf.data_ptr())  # misaligned: rejected before any launch
    assert e.value.code == lbcm.LBCM_EINVAL
    bad = lbcm.make_params(0, 8, precision="fp32")
    with pytest.raises(lbcm.LbcmError) as e:
        lbcm.lbcm_diag_state(bad, buf, buf)
    assert e.value.code == lbcm.LBCM_EINVAL
