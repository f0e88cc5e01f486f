"""Seeded synthetic halo catalogues for the anisotropic 3PCF estimator.

This module only draws inputs. It holds none of the estimator's arithmetic,
so both the GPU path and the CPU reference can be fed from it.

The catalogues stand in for the N-body halo boxes the paper measures
(Sec. 3: periodic boxes of side 1500 Mpc/h, halo density 2.13e-4 (h/Mpc)^3,
redshift-space positions along a fixed line of sight z, Sec. 4). Two kinds:

* ``poisson``   : uniform (unclustered) points, also used as randoms.
* ``zeldovich`` : a clustered catalogue. A Gaussian random field with
  P(k) ~ k^-1.5 exp(-(k/0.3)^2) on a periodic grid gives a Zel'dovich
  displacement field Psi(k) = i k delta(k) / k^2, rescaled so that the rms of
  each Cartesian component is ``sigma_psi``. Uniform Lagrangian points q take
  x = q + Psi(q) (cloud-in-cell interpolation), then the plane-parallel
  redshift-space shift x_z += f Psi_z(q), and finally wrap into [0, box).

Two back ends draw the same recipe: numpy (PCG64, the canonical stream used
by the tests) and torch on any device (used to make large benchmark batches
quickly; its random stream differs from numpy's).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2408030360
RANDOMS_SEED_OFFSET = 1_000_000


def catalogue_seed(i: int) -> int:
    return BASE_SEED + int(i)


def randoms_seed(i: int) -> int:
    return BASE_SEED + RANDOMS_SEED_OFFSET + int(i)


def _wrap(x: np.ndarray, box: float) -> np.ndarray:
    x = np.mod(x, box)
    x[x >= box] -= box  # np.mod can round up to box itself
    return x


def poisson(n: int, box: float, seed: int) -> np.ndarray:
    """n points uniform in [0, box)^3, float64 (n, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _wrap(rng.random((int(n), 3)) * box, box)


def randoms(n: int, box: float, seed: int) -> np.ndarray:
    return poisson(n, box, seed)


def log_uniform_sizes(ncat: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Catalogue sizes drawn log-uniform in [lo, hi] (int64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(int(ncat))
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def _kgrid(grid: int, box: float):
    k1 = 2.0 * np.pi * np.fft.fftfreq(grid, d=box / grid)
    kz = 2.0 * np.pi * np.fft.rfftfreq(grid, d=box / grid)
    return k1, kz


def power_shape(k):
    """P(k) ~ k^-1.5 exp(-(k/0.3)^2), k in h/Mpc (the amplitude is irrelevant:
    the displacement field is rescaled to a target rms)."""
    with np.errstate(divide="ignore"):
        return np.where(k > 0, k ** -1.5 * np.exp(-(k / 0.3) ** 2), 0.0)


def _cic(field: np.ndarray, q: np.ndarray, box: float) -> np.ndarray:
    """Cloud-in-cell interpolation of a periodic grid field at positions q."""
    g = field.shape[0]
    u = q * (g / box)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    i0 %= g
    i1 = (i0 + 1) % g
    out = np.zeros(q.shape[0])
    for cx in (0, 1):
        ix = i1[:, 0] if cx else i0[:, 0]
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        for cy in (0, 1):
            iy = i1[:, 1] if cy else i0[:, 1]
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            for cz in (0, 1):
                iz = i1[:, 2] if cz else i0[:, 2]
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                out += wx * wy * wz * field[ix, iy, iz]
    return out


def zeldovich(n: int, box: float, sigma_psi: float, f_growth: float, seed: int,
              grid: int = 256) -> np.ndarray:
    """Clustered catalogue (float64 (n, 3) in [0, box)) from the Zel'dovich
    recipe above, with redshift-space distortion along z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((grid, grid, grid))
    dk = np.fft.rfftn(white)
    del white
    k1, kz = _kgrid(grid, box)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kzz = kz[None, None, :]
    k2 = kx * kx + ky * ky + kzz * kzz
    kk = np.sqrt(k2)
    dk *= np.sqrt(power_shape(kk))
    k2[0, 0, 0] = 1.0
    dk[0, 0, 0] = 0.0
    psi = []
    for kc in (kx, ky, kzz):
        comp = np.fft.irfftn(1j * kc * dk / k2, s=(grid, grid, grid), axes=(0, 1, 2))
        psi.append(comp)
    del dk
    rms = math.sqrt(sum(float(np.mean(c * c)) for c in psi) / 3.0)
    scale = sigma_psi / rms if rms > 0 else 0.0
    q = rng.random((int(n), 3)) * box
    disp = np.stack([_cic(c, q, box) for c in psi], axis=1) * scale
    x = q + disp
    x[:, 2] += f_growth * disp[:, 2]
    return _wrap(x, box)


def zeldovich_torch(n: int, box: float, sigma_psi: float, f_growth: float, seed: int,
                    grid: int = 256, device="cpu"):
    """The same recipe as ``zeldovich`` drawn with torch on ``device``
    (returns a float64 (n, 3) tensor on that device). Used to build large
    benchmark batches fast; the random stream differs from numpy's."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.float64
    white = torch.randn((grid, grid, grid), generator=gen, device=device, dtype=dt)
    dk = torch.fft.rfftn(white)
    del white
    k1 = 2.0 * math.pi * torch.fft.fftfreq(grid, d=box / grid, device=device, dtype=dt)
    kz = 2.0 * math.pi * torch.fft.rfftfreq(grid, d=box / grid, device=device, dtype=dt)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kzz = kz[None, None, :]
    k2 = kx * kx + ky * ky + kzz * kzz
    kk = torch.sqrt(k2)
    pk = torch.where(kk > 0, kk.clamp_min(1e-30) ** -1.5 * torch.exp(-(kk / 0.3) ** 2),
                     torch.zeros_like(kk))
    dk = dk * torch.sqrt(pk)
    k2[0, 0, 0] = 1.0
    dk[0, 0, 0] = 0.0
    psi = [torch.fft.irfftn(1j * kc * dk / k2, s=(grid, grid, grid)) for kc in (kx, ky, kzz)]
    del dk
    rms = math.sqrt(sum(float(torch.mean(c * c)) for c in psi) / 3.0)
    scale = sigma_psi / rms if rms > 0 else 0.0
    q = torch.rand((int(n), 3), generator=gen, device=device, dtype=dt) * box
    u = q * (grid / box)
    i0 = torch.floor(u).long()
    fr = u - i0
    i0 = i0 % grid
    i1 = (i0 + 1) % grid
    disp = torch.zeros((int(n), 3), device=device, dtype=dt)
    for cx in (0, 1):
        ix = i1[:, 0] if cx else i0[:, 0]
        wx = fr[:, 0] if cx else 1.0 - fr[:, 0]
        for cy in (0, 1):
            iy = i1[:, 1] if cy else i0[:, 1]
            wy = fr[:, 1] if cy else 1.0 - fr[:, 1]
            for cz in (0, 1):
                iz = i1[:, 2] if cz else i0[:, 2]
                wz = fr[:, 2] if cz else 1.0 - fr[:, 2]
                wgt = wx * wy * wz
                for c in range(3):
                    disp[:, c] += wgt * psi[c][ix, iy, iz]
    disp *= scale
    x = q + disp
    x[:, 2] += f_growth * disp[:, 2]
    x = torch.remainder(x, box)
    x = torch.where(x >= box, x - box, x)
    return x


def dr_weights(n_data: int, n_rand: int) -> np.ndarray:
    """Per-point weights for the data-minus-randoms field: 1 for data,
    -n_data/n_rand for randoms (data first, then randoms)."""
    w = np.ones(n_data + n_rand)
    if n_rand:
        w[n_data:] = -float(n_data) / float(n_rand)
    return w


def dyadic_lattice(n: int, box: float, bits: int, seed: int) -> np.ndarray:
    """Uniform points snapped to a dyadic lattice of spacing box/2^bits, so that
    90-degree rotations, reflections and lattice translations are exact in
    floating point (box itself must be a power of two times a small integer)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = 1 << bits
    idx = rng.integers(0, m, size=(int(n), 3))
    return idx.astype(np.float64) * (box / m)
