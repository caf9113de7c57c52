"""Seeded synthetic inputs shared by the CPU oracle, the GPU tests and the bench.

This module holds input generation only: angle sets, disk and Gaussian-blob
phantoms, pixel noise and random sinograms. It contains none of the Radon /
gridding arithmetic, so both the oracle and the HIP path may use it.

Conventions (shared by every consumer):
  * image ``x`` is ``n x n`` row-major; pixel (i, j) sits at
    (x, y) = (j - n/2, i - n/2) in pixel units;
  * angles are radians, float64, uniform in [0, pi) unless stated.

Phantom recipe (the paper images glass spheres, whose slices are disks):
disks are additive, each pixel's value is the disk's area coverage measured
by 8x8 supersampling in float64, and every disk lies inside the inscribed
circle with a 2-pixel margin so no projection wraps at n_det = n.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_angles",
    "disk_params",
    "disk_phantom",
    "gaussian_blob",
    "config1_phantom",
    "config2_phantom",
    "disk_sinogram",
    "config4_problem",
    "random_sinogram",
    "random_image",
]


def uniform_angles(n_views: int) -> np.ndarray:
    """theta_a = a * pi / n_views, a = 0 .. n_views-1 (float64)."""
    return np.arange(n_views, dtype=np.float64) * (np.pi / n_views)


def disk_params(rng: np.random.Generator, n: int, k: int, r_lo: float, r_hi: float,
                d_lo: float = 0.5, d_hi: float = 1.0):
    """Draw k disks: radius U(r_lo, r_hi), density U(d_lo, d_hi), centre
    uniform in the disk |c| <= n/2 - 2 - r (rejection sampling)."""
    out = []
    for _ in range(k):
        r = float(rng.uniform(r_lo, r_hi))
        rmax = n / 2 - 2 - r
        if rmax <= 0:
            r = max(1.0, n / 2 - 3)
            rmax = n / 2 - 2 - r
        while True:
            cx, cy = rng.uniform(-rmax, rmax, size=2)
            if cx * cx + cy * cy <= rmax * rmax:
                break
        rho = float(rng.uniform(d_lo, d_hi))
        out.append((float(cx), float(cy), r, rho))
    return out


def disk_phantom(n: int, disks, ss: int = 8) -> np.ndarray:
    """Sum of uniform disks as float64 area coverage (ss x ss supersampling).

    Pixels whose centre is farther than r + 0.75 from a disk centre are 0,
    nearer than r - 0.75 are fully covered, and only the boundary ring is
    supersampled; this gives the same values as supersampling every pixel.
    """
    img = np.zeros((n, n), dtype=np.float64)
    off = (np.arange(ss) + 0.5) / ss - 0.5
    for cx, cy, r, rho in disks:
        j0 = max(0, int(np.floor(cx + n / 2 - r - 2)))
        j1 = min(n, int(np.ceil(cx + n / 2 + r + 3)))
        i0 = max(0, int(np.floor(cy + n / 2 - r - 2)))
        i1 = min(n, int(np.ceil(cy + n / 2 + r + 3)))
        if j0 >= j1 or i0 >= i1:
            continue
        xs = np.arange(j0, j1, dtype=np.float64) - n / 2 - cx
        ys = np.arange(i0, i1, dtype=np.float64) - n / 2 - cy
        d = np.sqrt(ys[:, None] ** 2 + xs[None, :] ** 2)
        cov = np.where(d < r - 0.75, 1.0, 0.0)
        ring = np.nonzero((d >= r - 0.75) & (d <= r + 0.75))
        if ring[0].size:
            px = xs[ring[1]][:, None, None] + off[None, None, :]
            py = ys[ring[0]][:, None, None] + off[None, :, None]
            inside = (px * px + py * py) < r * r
            cov[ring] = inside.reshape(inside.shape[0], -1).mean(axis=1)
        img[i0:i1, j0:j1] += rho * cov
    return img


def gaussian_blob(n: int, cx: float, cy: float, sigma_g: float, amp: float = 1.0) -> np.ndarray:
    """amp * exp(-|p - c|^2 / (2 sigma_g^2)) point-sampled at pixel centres."""
    xs = np.arange(n, dtype=np.float64) - n / 2
    d2 = (xs[None, :] - cx) ** 2 + (xs[:, None] - cy) ** 2
    return amp * np.exp(-d2 / (2.0 * sigma_g * sigma_g))


def config1_phantom(seed: int, n: int = 128):
    """Parity workload: n x n image of 3-8 disks, radii U(5,30), densities
    U(0.5,1). Returns (float32 image, disk list)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(3, 9))
    r_hi = min(30.0, n / 2 - 4)
    disks = disk_params(rng, n, k, min(5.0, r_hi / 2), r_hi)
    return disk_phantom(n, disks).astype(np.float32), disks


def config2_phantom(seed: int = 0, n: int = 2560, k: int = 200, noise: float = 1e-2):
    """Throughput workload: n x n image of k disks, radii U(10,300), plus
    i.i.d. N(0, noise^2) pixel noise. Returns float32 image."""
    rng = np.random.default_rng(seed)
    disks = disk_params(rng, n, k, 10.0, min(300.0, n / 2 - 4))
    img = disk_phantom(n, disks)
    img += rng.normal(0.0, noise, size=img.shape)
    return img.astype(np.float32)


def random_image(seed: int, n: int) -> np.ndarray:
    """i.i.d. U(-1, 1) float32 image (adjoint identity, parity)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n)).astype(np.float32)


def random_sinogram(seed: int, n_views: int, n_det: int) -> np.ndarray:
    """i.i.d. U(-1, 1) float32 sinogram (adjoint identity, parity)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n_views, n_det)).astype(np.float32)


def disk_sinogram(disks, angles, n_det: int) -> np.ndarray:
    """Exact line integrals of the disks (float64, n_views x n_det): a disk of
    radius r, density rho and centre c contributes rho * 2 sqrt(r^2 - t^2) at
    detector s_d = d - n_det/2, t = s_d - (c_x cos th + c_y sin th)."""
    angles = np.asarray(angles, dtype=np.float64)
    s = np.arange(n_det, dtype=np.float64) - n_det / 2
    c, sn = np.cos(angles)[:, None], np.sin(angles)[:, None]
    out = np.zeros((angles.size, n_det))
    for cx, cy, r, rho in disks:
        t = s[None, :] - (cx * c + cy * sn)
        out += rho * 2.0 * np.sqrt(np.maximum(r * r - t * t, 0.0))
    return out


def config4_problem(seed: int = 0, n: int = 1024, n_views: int = 128, n_det: int = 1024, k: int = 60,
                    snr_db: float = 30.0, gain_sd: float = 0.02):
    """Reduced-view reconstruction workload: an n x n piecewise-constant disk
    phantom (k disks, radii U(8, n/8), densities U(0.5, 1)), measured at
    n_views angles uniform in [0, pi) on n_det bins by exact line integrals,
    each detector scaled by a gain N(1, gain_sd^2) (ring stripes), then i.i.d.
    Gaussian noise at the given SNR (20 log10 ||signal|| / ||noise||).
    Returns (float32 image, float32 sinogram, angles)."""
    rng = np.random.default_rng(seed)
    disks = disk_params(rng, n, k, 8.0, n / 8)
    img = disk_phantom(n, disks)
    ang = uniform_angles(n_views)
    clean = disk_sinogram(disks, ang, n_det)
    gains = rng.normal(1.0, gain_sd, size=n_det)
    noise_sd = np.linalg.norm(clean) / np.sqrt(clean.size) * 10.0 ** (-snr_db / 20.0)
    b = clean * gains[None, :] + rng.normal(0.0, noise_sd, size=clean.shape)
    return img.astype(np.float32), b.astype(np.float32), ang
