"""Pins for O-grid (the FP64 gridding oracle).

O-grid is pinned to O-exact on tiny inputs (G1; O-exact is pinned on its own
in test_oracle_exact.py), to closed forms (axis sums G2, mass G3, Gaussian
blobs G5, disk chords G6), to the adjoint identity (G7) and to a dense-matrix
brute force (G8). The last block plants plausible mistakes in copies of the
oracle's steps and checks that at least one pin catches each of them.
"""
import numpy as np
import pytest

import oracle.grid as og
from oracle.exact import radon_exact, radon_exact_adjoint
from oracle.grid import grid_adjoint, grid_forward
from radon_inputs import (config1_phantom, gaussian_blob, random_image,
                          random_sinogram, uniform_angles)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def special_angles(nv, seed):
    ang = np.random.default_rng(seed).uniform(0, np.pi, nv)
    ang[0], ang[1] = 0.0, np.pi / 2
    return ang


# --- pin checks (return the measured error so planted mistakes can reuse them)

def g1_forward_err(n=16, N=16, nv=9, seed=0):
    ang = special_angles(nv, seed)
    x = random_image(seed + 10, n).astype(np.float64)
    return rel(grid_forward(x, ang, N), radon_exact(x, ang, N))


def g1_adjoint_err(n=16, N=16, nv=9, seed=0):
    ang = special_angles(nv, seed)
    y = random_sinogram(seed + 20, nv, N).astype(np.float64)
    return rel(grid_adjoint(y, ang, n), radon_exact_adjoint(y, ang, n))


def g2_err(n=32):
    x = random_image(3, n).astype(np.float64)
    y = grid_forward(x, np.array([0.0, np.pi / 2]), n)
    return max(rel(y[0], x.sum(axis=0)), rel(y[1], x.sum(axis=1)))


def g3_err(n=32, N=40):
    x = random_image(4, n).astype(np.float64) + 0.5
    y = grid_forward(x, uniform_angles(7), N)
    return float(np.abs(y.sum(axis=1) - x.sum()).max() / abs(x.sum()))


def g5_err(n=128, nv=24):
    cx, cy, sg, A = 17.3, -9.6, 2.5, 1.0
    x = gaussian_blob(n, cx, cy, sg, A)
    ang = uniform_angles(nv)
    y = grid_forward(x, ang, n)
    s = np.arange(n) - n / 2
    ref = np.stack([A * np.sqrt(2 * np.pi) * sg *
                    np.exp(-(s - (cx * np.cos(t) + cy * np.sin(t))) ** 2 / (2 * sg * sg))
                    for t in ang])
    return rel(y, ref)


def g7_err(n=24, N=28, nv=10):
    ang = special_angles(nv, 8)
    x = random_image(11, n).astype(np.float64)
    y = random_sinogram(12, nv, N).astype(np.float64)
    Ax, Aty = grid_forward(x, ang, N), grid_adjoint(y, ang, n)
    return abs(np.sum(Ax * y) - np.sum(x * Aty)) / (np.linalg.norm(Ax) * np.linalg.norm(y))


# --- the pins

@pytest.mark.parametrize("n,N,nv", [(8, 8, 6), (16, 16, 9), (16, 24, 7), (32, 32, 12)])
def test_g1_forward_vs_exact(n, N, nv):
    assert g1_forward_err(n, N, nv) <= 1e-4


@pytest.mark.parametrize("n,N,nv", [(8, 8, 6), (16, 16, 9), (16, 24, 7), (32, 32, 12)])
def test_g1_adjoint_vs_exact(n, N, nv):
    assert g1_adjoint_err(n, N, nv) <= 1e-4


def test_g1_wider_kernel_is_more_accurate():
    """The gridding error falls fast with W (W=8 is far below W=6)."""
    n, N, nv = 16, 16, 9
    ang = special_angles(nv, 0)
    x = random_image(10, n).astype(np.float64)
    ye = radon_exact(x, ang, N)
    e6 = rel(grid_forward(x, ang, N, W=6), ye)
    e8 = rel(grid_forward(x, ang, N, W=8), ye)
    assert e8 < 0.05 * e6


def test_g2_axis_sums():
    assert g2_err() <= 1e-4


def test_g3_mass_per_view():
    assert g3_err() <= 1e-4


def test_g5_gaussian_blob():
    assert g5_err() <= 1e-4


def test_g6_disk_chords_config1():
    """Disks project to sum_k 2 rho_k sqrt(r_k^2 - (s - c_k . e)^2)_+ up to
    the pixelisation of the phantom (loose bound)."""
    x, disks = config1_phantom(0)
    n = x.shape[0]
    ang = uniform_angles(180)
    y = grid_forward(x, ang, n)
    s = np.arange(n) - n / 2
    ref = np.zeros_like(y)
    for (cx, cy, r, rho) in disks:
        t = s[None, :] - (cx * np.cos(ang)[:, None] + cy * np.sin(ang)[:, None])
        ref += 2 * rho * np.sqrt(np.clip(r * r - t * t, 0, None))
    assert rel(y, ref) <= 2e-2


def test_g7_adjoint_identity():
    assert g7_err() <= 1e-12


def test_g8_dense_transpose_n8():
    n, N = 8, 8
    ang = np.array([0.0, 0.4, np.pi / 2, 2.5])
    nv = len(ang)
    A = np.stack([grid_forward(e.reshape(n, n), ang, N).ravel() for e in np.eye(n * n)], axis=1)
    At = np.stack([grid_adjoint(e.reshape(nv, N), ang, n).ravel() for e in np.eye(nv * N)], axis=1)
    assert np.abs(At - A.T).max() <= 1e-12 * np.abs(A).max()


def test_full_size_gaussian_runs_without_quadratic_work():
    """G5 at a larger grid: the FFT path stays accurate at n=512."""
    assert g5_err(n=512, nv=16) <= 1e-4


# --- planted mistakes: each must be caught by at least one pin

def _bad_fft2_transposed(x, gp):
    xp = np.asarray(x, dtype=np.float64) / (gp.psi[:, None] * gp.psi[None, :])
    P = np.zeros((gp.G, gp.G), dtype=np.complex128)
    r = (np.arange(gp.n) - gp.n // 2) % gp.G
    P[np.ix_(r, r)] = xp.T
    return og.sfft.fft2(P)


def _bad_fft2_sign(x, gp):
    xp = np.asarray(x, dtype=np.float64) / (gp.psi[:, None] * gp.psi[None, :])
    P = np.zeros((gp.G, gp.G), dtype=np.complex128)
    r = (np.arange(gp.n) - gp.n // 2) % gp.G
    P[np.ix_(r, r)] = xp
    return og.sfft.ifft2(P) * (gp.G * gp.G)


def _bad_fft2_uncentred(x, gp):
    xp = np.asarray(x, dtype=np.float64) / (gp.psi[:, None] * gp.psi[None, :])
    P = np.zeros((gp.G, gp.G), dtype=np.complex128)
    P[:gp.n, :gp.n] = xp
    return og.sfft.fft2(P)


def _bad_ray_synthesis_no_norm(Xt, n_det):
    return (np.asarray(Xt) @ og.ray_synthesis_matrix(n_det)).real


def _bad_ray_spectrum_sign(y, n_det):
    return (np.asarray(y) @ og.ray_synthesis_matrix(n_det).T) / n_det


class _ShiftedFootprint(og.GridParams):
    def offsets(self):
        return range(-self.W // 2, self.W // 2)


def _all_pins_pass():
    return (g1_forward_err() <= 1e-4 and g1_adjoint_err() <= 1e-4 and g2_err() <= 1e-4
            and g3_err() <= 1e-4 and g5_err(n=64, nv=8) <= 1e-4 and g7_err() <= 1e-12)


@pytest.mark.parametrize("mistake", [
    "no_deapod", "shifted_footprint", "transposed_pad", "fft_sign",
    "uncentred_pad", "dropped_1_over_N", "adjoint_spectrum_sign", "wrong_beta",
])
def test_planted_mistake_is_caught(monkeypatch, mistake):
    assert _all_pins_pass()
    if mistake == "no_deapod":
        monkeypatch.setattr(og, "deapod_factors", lambda n, G, W, beta: np.ones(n))
    elif mistake == "shifted_footprint":
        monkeypatch.setattr(og, "GridParams", _ShiftedFootprint)
    elif mistake == "transposed_pad":
        monkeypatch.setattr(og, "grid_fft2", _bad_fft2_transposed)
    elif mistake == "fft_sign":
        monkeypatch.setattr(og, "grid_fft2", _bad_fft2_sign)
    elif mistake == "uncentred_pad":
        monkeypatch.setattr(og, "grid_fft2", _bad_fft2_uncentred)
    elif mistake == "dropped_1_over_N":
        monkeypatch.setattr(og, "ray_synthesis", _bad_ray_synthesis_no_norm)
    elif mistake == "adjoint_spectrum_sign":
        monkeypatch.setattr(og, "ray_spectrum", _bad_ray_spectrum_sign)
    elif mistake == "wrong_beta":
        monkeypatch.setattr(og, "kb_beta", lambda W, sigma: 0.5 * np.pi * W)
    assert not _all_pins_pass()
