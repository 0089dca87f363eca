"""Measures of a simulated phi field used to compare runs (not part of the lattice Boltzmann path)."""
from __future__ import annotations


def structure_factor(phi):
    """Radially averaged structure factor of phi - mean(phi): the mean of |FFT|^2 / N over the
    wavevectors whose length (in units of 2 pi / n) rounds to k, for k = 1 .. n / 2.  phi: a
    numpy array or a torch tensor (computed on the GPU)."""
    import torch

    t = phi if isinstance(phi, torch.Tensor) else torch.from_numpy(phi)
    t = t.to(device="cuda", dtype=torch.float64)
    t = t - t.mean()
    F = torch.fft.fft2(t)
    pw = (F.real ** 2 + F.imag ** 2) / t.numel()
    ny, nx = t.shape
    ky = torch.fft.fftfreq(ny, d=1.0 / ny, device="cuda", dtype=torch.float64)
    kx = torch.fft.fftfreq(nx, d=1.0 / nx, device="cuda", dtype=torch.float64)
    shell = torch.round(torch.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)).long()
    kmax = min(nx, ny) // 2
    m = (shell >= 1) & (shell <= kmax)
    s = torch.zeros(kmax + 1, dtype=torch.float64, device="cuda").index_add_(0, shell[m], pw[m])
    c = torch.zeros(kmax + 1, dtype=torch.float64, device="cuda").index_add_(0, shell[m], torch.ones_like(pw[m]))
    return (s[1:] / c[1:]).cpu().numpy()


def rel_l2(a, b) -> float:
    """||a - b|| / ||b|| of two numpy arrays."""
    import numpy as np

    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sk_rel_l2(phi, ref) -> float:
    """Relative L2 difference of the structure factors of phi and ref."""
    return rel_l2(structure_factor(phi), structure_factor(ref))
