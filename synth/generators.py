"""Seeded specimens, masks, noise and workload presets.

The paper's data (TiO2 beads in agarose, cucumber tissue; 1024 x 1024 A-scans
over 4 mm^2 at 830 nm, Sec. 3.1) are not available.  These generators stand in
for them with the same structure: sparse point scatterers (beads), layered
interfaces with depth falloff and speckle (tissue), a smooth random background,
and the three sub-sampling schemes of Sec. 3.1 (random, equispaced, partial).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "OPTICS", "PRESETS", "preset", "complex_normal", "standard_normal",
    "scatterers", "layers", "random_field", "smooth_field_coarse", "mask_ones", "mask_random_exact",
    "mask_bernoulli", "mask_equispaced", "mask_partial", "noisy", "is_smooth7",
    "serving_mix",
]

# Optics shared by every workload: k in [2 pi/0.9, 2 pi/0.75] rad/um (830 nm
# class source), lateral pitch 2 um, Gaussian waist 5 um, focus at mid-depth,
# quadratic dispersion 1e-3 rad/px^2, KB width 6, oversampling 2.
OPTICS = dict(k_min=2.0 * math.pi / 0.9, k_max=2.0 * math.pi / 0.75, dx=2.0, dy=2.0,
              dz=0.0, z_focus=-1.0, beam_waist=5.0, disp_a=1e-3, disp_b=0.0,
              kb_width=6, oversamp=2.0, kb_beta=0.0)

PRESETS = {
    # small B-scan: 512 depth x 64 lateral, 20 scatterers, l1, 50 iterations
    "bscan_512x64_l1": dict(geom=dict(n_depth=512, n_x=64, n_k=512), pen="l1", lam=0.01,
                            iters=50, scatterers=20, mask="ones", noise=0.01),
    # full B-scan: 2048 x 1000, 500 scatterers + 3 layers, 50% random mask, TV, 100 it.
    "bscan_2048x1000_tv": dict(geom=dict(n_depth=2048, n_x=1000, n_k=2048), pen="tv", lam=0.005,
                               iters=100, scatterers=500, layers=3, mask="random_half",
                               noise=0.01),
    # volume: 2048 x 256 x 256, 5000 scatterers + smooth field, 3-level Haar, 50 it.
    "volume_2048x256x256_haar": dict(geom=dict(n_depth=2048, n_x=256, n_y=256, lateral_dims=2,
                                               n_k=2048), pen="haar", lam=0.01, iters=50,
                                     scatterers=5000, field=0.05, mask="ones", noise=0.01),
    # differentiation batch: 32 B-scans of 1024 x 512
    "batch32_1024x512_grad": dict(geom=dict(n_depth=1024, n_x=512, n_k=1024, batch=32),
                                  pen=None, mask="ones", noise=0.01),
}


def preset(name: str) -> dict:
    p = dict(PRESETS[name])
    g = dict(OPTICS)
    g.update(dict(lateral_dims=1, n_y=1, batch=1))
    g.update(p["geom"])
    p["geom"] = g
    return p


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """CN(0, 1): independent N(0, 1/2) real and imaginary parts."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def standard_normal(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape)


def scatterers(rng: np.random.Generator, shape, count: int, amp=(0.5, 1.0)) -> np.ndarray:
    """On-grid point scatterers: positions uniform without replacement over the
    voxels of each batch item, amplitudes U(amp), phases U(0, 2 pi)."""
    shape = tuple(shape)
    out = np.zeros(shape, dtype=np.complex128)
    per = int(np.prod(shape[1:]))
    for b in range(shape[0]):
        pos = rng.choice(per, size=min(count, per), replace=False)
        a = rng.uniform(amp[0], amp[1], size=pos.size)
        ph = rng.uniform(0.0, 2.0 * math.pi, size=pos.size)
        out[b].reshape(-1)[pos] = a * np.exp(1j * ph)
    return out


def layers(rng: np.random.Generator, n_depth: int, n_lat: int, count: int = 3) -> np.ndarray:
    """Smooth layered interfaces z_i(l) = z_i0 + A_i sin(2 pi l / P_i + phi_i),
    z_i0 ~ U(0.2, 0.8) N_z, A_i ~ U(10, 50) px, P_i ~ U(300, 1000) A-scans; below
    each interface a Gaussian intensity falloff exp(-d^2 / (2 s_i^2)),
    s_i ~ U(20, 60) px, times CN(0, 1) speckle.  Shape (n_lat, n_depth)."""
    out = np.zeros((n_lat, n_depth), dtype=np.complex128)
    n = np.arange(n_depth)[None, :]
    lat = np.arange(n_lat)[:, None]
    for _ in range(count):
        z0 = rng.uniform(0.2, 0.8) * n_depth
        A = rng.uniform(10.0, 50.0)
        P = rng.uniform(300.0, 1000.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        s = rng.uniform(20.0, 60.0)
        zi = z0 + A * np.sin(2.0 * math.pi * lat / P + ph)
        d = n - zi
        env = np.where(d >= 0.0, np.exp(-d * d / (2.0 * s * s)), 0.0)
        out += env * complex_normal(rng, (n_lat, n_depth))
    return out


def random_field(rng: np.random.Generator, shape, sigma_px: float, rms: float) -> np.ndarray:
    """Smooth complex random field: CN(0,1) filtered by a Gaussian of sigma_px
    pixels along every axis, rescaled to the given RMS amplitude."""
    from scipy.ndimage import gaussian_filter
    w = complex_normal(rng, shape)
    f = gaussian_filter(w.real, sigma_px, mode="wrap") + 1j * gaussian_filter(w.imag, sigma_px, mode="wrap")
    return f * (rms / np.sqrt(np.mean(np.abs(f) ** 2)))


def smooth_field_coarse(rng: np.random.Generator, shape, factor: int, rms: float) -> np.ndarray:
    """Smooth complex random field for large volumes: CN(0,1) on a grid
    `factor` times coarser along every axis, linearly upsampled, rescaled
    to the given RMS amplitude."""
    from scipy.ndimage import zoom
    shape = tuple(shape)
    coarse = tuple(max(2, s // factor) for s in shape)
    w = complex_normal(rng, coarse)
    zf = [s / c for s, c in zip(shape, coarse)]
    f = zoom(w.real, zf, order=1) + 1j * zoom(w.imag, zf, order=1)
    f = f[tuple(slice(0, s) for s in shape)]
    return f * (rms / np.sqrt(np.mean(np.abs(f) ** 2)))


def mask_ones(lat_shape, n_k: int) -> np.ndarray:
    return np.ones(tuple(lat_shape) + (n_k,), dtype=np.uint8)


def mask_random_exact(rng: np.random.Generator, lat_shape, n_k: int, keep: int) -> np.ndarray:
    """Exactly ``keep`` of the n_k spectral pixels per A-scan, seeded permutation."""
    lat_shape = tuple(lat_shape)
    m = np.zeros(lat_shape + (n_k,), dtype=np.uint8)
    flat = m.reshape(-1, n_k)
    for i in range(flat.shape[0]):
        flat[i, rng.permutation(n_k)[:keep]] = 1
    return m


def mask_bernoulli(rng: np.random.Generator, lat_shape, n_k: int, p: float = 0.5) -> np.ndarray:
    """Random sub-sampling of Sec. 3.1: binomial with expectation p."""
    return (rng.random(tuple(lat_shape) + (n_k,)) < p).astype(np.uint8)


def mask_equispaced(lat_shape, n_k: int) -> np.ndarray:
    """Equispaced sub-sampling of Sec. 3.1: every other spectral pixel."""
    m = np.zeros(tuple(lat_shape) + (n_k,), dtype=np.uint8)
    m[..., ::2] = 1
    return m


def mask_partial(lat_shape, n_k: int) -> np.ndarray:
    """Partial sub-sampling of Sec. 3.1: the central half of the band."""
    m = np.zeros(tuple(lat_shape) + (n_k,), dtype=np.uint8)
    m[..., n_k // 4: n_k // 4 + n_k // 2] = 1
    return m


def noisy(y_clean: np.ndarray, noise: np.ndarray, mask, rel: float) -> np.ndarray:
    """Additive Gaussian noise of standard deviation rel * max|y_clean|, masked."""
    sigma = rel * float(np.max(np.abs(y_clean)))
    y = y_clean + sigma * noise
    if mask is not None:
        y = y * mask
    return y


def is_smooth7(n: int) -> bool:
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def serving_mix(rng: np.random.Generator, count: int):
    """Request mix for the serving loop: 60% B-scans with 1024-2048 spectral
    pixels x 256-2000 A-scans, 30% small volumes 1024 x {64..128}^2, 10% small
    512 x 64 B-scans; every size a multiple of 8 and 7-smooth; a random penalty
    among l1 / TV / Haar and 50-100 iterations."""
    bs_k = [n for n in range(1024, 2049, 8) if is_smooth7(n)]
    bs_x = [n for n in range(256, 2001, 8) if is_smooth7(n)]
    vol = [n for n in range(64, 129, 8) if is_smooth7(n)]
    out = []
    for rid in range(count):
        u = rng.random()
        if u < 0.6:
            nk = int(rng.choice(bs_k))
            geom = dict(n_depth=nk, n_k=nk, n_x=int(rng.choice(bs_x)), n_y=1, lateral_dims=1)
        elif u < 0.9:
            n = int(rng.choice(vol))
            geom = dict(n_depth=1024, n_k=1024, n_x=n, n_y=n, lateral_dims=2)
        else:
            geom = dict(n_depth=512, n_k=512, n_x=64, n_y=1, lateral_dims=1)
        pen = ["l1", "tv", "haar"][int(rng.integers(0, 3))]
        lam = {"l1": 0.01, "tv": 0.005, "haar": 0.01}[pen]
        out.append(dict(id=rid, geom=geom, pen=pen, lam=lam, iters=int(rng.integers(50, 101)),
                        seed=4_000_000 + rid))
    return out
