"""Seeded synthetic particle stacks for alignment workloads.

This module only synthesises inputs; it contains none of the alignment
arithmetic.  It is shared by the tests, the benchmark and the oracle checks,
and imports nothing from the rest of the package.

Recipe (stands in for the down-sampled Ribosome-80S stacks of the paper's
experiments, which are not available here):

* A reference is a sum of n_b ~ U{8..20} isotropic Gaussian blobs with
  sigma ~ U[2, 6] px and amplitude ~ U[0.5, 1.5]; each blob centre is uniform
  in a disk of radius rho_max - 2*sigma around the box centre, so every
  blob's 2-sigma contour stays inside rho_max.
* A particle is a uniformly drawn reference transformed analytically as
  Shift_t o Mirror^m o Rot_alpha: blob centres mu -> c + t + Mir^m Rot(alpha)(mu - c),
  with alpha ~ U[0, 2*pi) (or an on-grid angle), t uniform in {-T..T}^2,
  m ~ Bernoulli(0.5), Mir = diag(1, -1) about the box centre; then iid
  Gaussian noise with variance var_box(clean particle) / SNR is added.
* Pixel (x = column, y = row) centres sit at integer coordinates; the box
  centre is (floor(L/2), floor(L/2)).

Parameters are drawn with ``numpy.random.default_rng((seed, stream))``;
rendering and noise run in torch (CPU or GPU) so that 100k-particle stacks
are generated on the device in milliseconds.  Results are float32.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

MAX_BLOBS = 20


@dataclasses.dataclass
class BlobSet:
    """Blob parameters of K references: centres [K, B, 2] (x, y), sigma and
    amplitude [K, B]; unused slots have amplitude 0."""

    centres: np.ndarray
    sigma: np.ndarray
    amp: np.ndarray
    L: int


@dataclasses.dataclass
class Truth:
    """Planted parameters of every particle."""

    ref: np.ndarray
    alpha: np.ndarray          # radians, counter-clockwise
    shift_x: np.ndarray
    shift_y: np.ndarray
    mirror: np.ndarray
    psi_index: np.ndarray | None   # set when angles were drawn on the grid
    noise_sigma: np.ndarray


def make_blobs(K: int, L: int, seed, rho_max: float | None = None,
               n_blobs=(8, 20), sigma=(2.0, 6.0), amp=(0.5, 1.5)) -> BlobSet:
    rng = np.random.default_rng(seed)
    if rho_max is None:
        rho_max = L / 2 - 4
    c = L // 2
    centres = np.zeros((K, MAX_BLOBS, 2))
    sig = np.ones((K, MAX_BLOBS))
    am = np.zeros((K, MAX_BLOBS))
    for k in range(K):
        nb = int(rng.integers(n_blobs[0], n_blobs[1] + 1))
        s = rng.uniform(sigma[0], sigma[1], nb)
        rad = np.maximum(rho_max - 2.0 * s, 0.0) * np.sqrt(rng.uniform(0.0, 1.0, nb))
        phi = rng.uniform(0.0, 2.0 * math.pi, nb)
        centres[k, :nb, 0] = c + rad * np.cos(phi)
        centres[k, :nb, 1] = c + rad * np.sin(phi)
        sig[k, :nb] = s
        am[k, :nb] = rng.uniform(amp[0], amp[1], nb)
    return BlobSet(centres, sig, am, L)


def _render(centres: torch.Tensor, sigma: torch.Tensor, amp: torch.Tensor, L: int) -> torch.Tensor:
    """Sum of isotropic Gaussians, [N, B] parameters -> [N, L, L] (row = y).

    Each Gaussian is separable, so the sum over blobs is a batched product of
    [N, L(y), B] and [N, B, L(x)] factors."""
    grid = torch.arange(L, dtype=centres.dtype, device=centres.device)
    inv = 1.0 / (2.0 * sigma * sigma)                                  # [N, B]
    gx = torch.exp(-(grid[None, None, :] - centres[..., 0:1]) ** 2 * inv[..., None])  # [N,B,L]
    gy = torch.exp(-(grid[None, None, :] - centres[..., 1:2]) ** 2 * inv[..., None])
    gy = gy * amp[..., None]
    return torch.bmm(gy.transpose(1, 2).contiguous(), gx)               # [N, L, L]


def render_refs(blobs: BlobSet, device="cpu") -> torch.Tensor:
    dt = torch.float64
    out = _render(torch.as_tensor(blobs.centres, dtype=dt, device=device),
                  torch.as_tensor(blobs.sigma, dtype=dt, device=device),
                  torch.as_tensor(blobs.amp, dtype=dt, device=device), blobs.L)
    return out.to(torch.float32)


def make_particles(blobs: BlobSet, N: int, shift_max: int, snr: float | None, seed,
                   mirror: bool = True, n_phi_grid: int | None = None,
                   device="cpu", chunk: int = 8192):
    """Render N particles from ``blobs``; returns (float32 [N, L, L] tensor, Truth).

    ``snr=None`` gives noise-free particles.  With ``n_phi_grid`` the rotation
    is drawn on the grid alpha = psi * 2*pi/n_phi_grid.
    """
    rng = np.random.default_rng(seed)
    K = blobs.centres.shape[0]
    L = blobs.L
    c = L // 2
    ref = rng.integers(0, K, N)
    if n_phi_grid:
        psi = rng.integers(0, n_phi_grid, N)
        alpha = psi * (2.0 * math.pi / n_phi_grid)
    else:
        psi = None
        alpha = rng.uniform(0.0, 2.0 * math.pi, N)
    tx = rng.integers(-shift_max, shift_max + 1, N)
    ty = rng.integers(-shift_max, shift_max + 1, N)
    mir = rng.integers(0, 2, N) if mirror else np.zeros(N, dtype=np.int64)
    noise_seed = int(rng.integers(0, 2**62))

    dt = torch.float64
    cen = torch.as_tensor(blobs.centres, dtype=dt, device=device)
    sig = torch.as_tensor(blobs.sigma, dtype=dt, device=device)
    am = torch.as_tensor(blobs.amp, dtype=dt, device=device)
    out = torch.empty((N, L, L), dtype=torch.float32, device=device)
    noise_sigma = np.zeros(N)
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    for lo in range(0, N, chunk):
        hi = min(N, lo + chunk)
        k = torch.as_tensor(ref[lo:hi], device=device)
        a = torch.as_tensor(alpha[lo:hi], dtype=dt, device=device)
        v = cen[k] - c                                                  # [n, B, 2]
        ca = torch.cos(a)[:, None]
        sa = torch.sin(a)[:, None]
        rx = ca * v[..., 0] - sa * v[..., 1]
        ry = sa * v[..., 0] + ca * v[..., 1]
        sign = torch.as_tensor(1 - 2 * mir[lo:hi], dtype=dt, device=device)[:, None]
        ry = ry * sign
        moved = torch.stack(
            [c + torch.as_tensor(tx[lo:hi], dtype=dt, device=device)[:, None] + rx,
             c + torch.as_tensor(ty[lo:hi], dtype=dt, device=device)[:, None] + ry], dim=-1)
        clean = _render(moved, sig[k], am[k], L)
        if snr is not None:
            var = clean.reshape(hi - lo, -1).var(dim=1, unbiased=False)
            s = torch.sqrt(var / snr)
            noise = torch.randn((hi - lo, L, L), dtype=dt, device=device, generator=gen)
            clean = clean + s[:, None, None] * noise
            noise_sigma[lo:hi] = s.cpu().numpy()
        out[lo:hi] = clean.to(torch.float32)
    truth = Truth(ref=ref, alpha=alpha, shift_x=tx, shift_y=ty, mirror=mir,
                  psi_index=psi, noise_sigma=noise_sigma)
    return out, truth


# Workload recipes of the benchmark configurations (sizes of each case).
WORKLOADS = {
    # small case that the oracle checks in full
    "mra_small": dict(N=1000, L=64, K=10, shift_max=2, r_min=1, r_max=30, n_phi=256,
                      snr=0.1, rho_max=28.0, seed=0),
    # the throughput workload: 100k particles, 76 px, 100 references, +-3 px
    "mra_c1": dict(N=100000, L=76, K=100, shift_max=3, r_min=1, r_max=35, n_phi=256,
                   snr=0.05, rho_max=28.0, seed=1),
}


def uneven_stack_specs(n_stacks: int = 64, seed: int = 3):
    """Size distribution of the uneven-stack batch: L in {64,76,96,128},
    N ~ U{2000..50000}, K ~ U{20..400}, T ~ U{2..5}, rings 1..L/2-2."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_stacks):
        L = int(rng.choice([64, 76, 96, 128]))
        specs.append(dict(L=L, N=int(rng.integers(2000, 50001)), K=int(rng.integers(20, 401)),
                          shift_max=int(rng.integers(2, 6)), r_min=1, r_max=L // 2 - 2,
                          n_phi=256, snr=0.05, rho_max=L / 2 - 4, seed=(seed, i)))
    return specs
