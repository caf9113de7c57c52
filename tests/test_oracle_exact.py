"""Pins for O-exact (the discrete Fourier-slice Radon transform with exact
interpolation) against closed forms, special cases and brute force.

The Dirichlet closed form used below is derived independently of the oracle:
sum_{q=-N/2}^{N/2-1} exp(2 pi i q t / N) = exp(-i pi t/N) sin(pi t)/sin(pi t/N),
so Re D_N(t) = (1/N) sin(pi t) cos(pi t/N) / sin(pi t/N), with D_N(0) = 1.
"""
import numpy as np
import pytest

from oracle.exact import radon_exact, radon_exact_adjoint
from radon_inputs import gaussian_blob, random_image, random_sinogram, uniform_angles


def dirichlet_re(t, N):
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    nz = np.abs(np.sin(np.pi * t / N)) > 1e-300
    tt = t[nz]
    out[nz] = np.sin(np.pi * tt) * np.cos(np.pi * tt / N) / np.sin(np.pi * tt / N) / N
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_axis_sums(n):
    """G2: theta=0 gives column sums, theta=pi/2 gives row sums (N = n)."""
    x = random_image(3, n).astype(np.float64)
    ang = np.array([0.0, np.pi / 2])
    y = radon_exact(x, ang, n)
    assert np.allclose(y[0], x.sum(axis=0), rtol=0, atol=1e-12)
    assert np.allclose(y[1], x.sum(axis=1), rtol=0, atol=1e-12)


def test_mass_per_view():
    """G3: every view carries the total mass (the q = 0 sample)."""
    n = 16
    x = random_image(4, n).astype(np.float64)
    y = radon_exact(x, uniform_angles(13), 20)
    assert np.allclose(y.sum(axis=1), x.sum(), rtol=0, atol=1e-11)


@pytest.mark.parametrize("n,N", [(16, 16), (16, 24)])
def test_impulse_is_dirichlet(n, N):
    """G4: a unit pixel at p projects to Re D_N(s_d - e_a . p)."""
    ang = np.array([0.0, 0.3, 1.1, np.pi / 2, 2.9])
    s = np.arange(N) - N / 2
    for (i, j) in [(n // 2, n // 2), (3, 11), (12, 2)]:
        x = np.zeros((n, n))
        x[i, j] = 1.0
        px, py = j - n / 2, i - n / 2
        y = radon_exact(x, ang, N)
        ref = np.stack([dirichlet_re(s - (np.cos(t) * px + np.sin(t) * py), N) for t in ang])
        assert np.allclose(y, ref, rtol=0, atol=1e-12)
        if (i, j) == (n // 2, n // 2):
            onehot = np.zeros(N)
            onehot[N // 2] = 1.0
            assert np.allclose(y, onehot[None, :], atol=1e-12)


def test_adjoint_of_onehot_is_dirichlet():
    """G4: the adjoint of a one-hot sinogram at (a, d) is Re D_N(s_d - e_a . p)."""
    n, N = 12, 16
    ang = np.array([0.2, 0.7, 2.0])
    xs = np.arange(n) - n / 2
    for a, d in [(0, 3), (1, 8), (2, 15)]:
        y = np.zeros((len(ang), N))
        y[a, d] = 1.0
        img = radon_exact_adjoint(y, ang, n)
        proj = np.cos(ang[a]) * xs[None, :] + np.sin(ang[a]) * xs[:, None]
        assert np.allclose(img, dirichlet_re((d - N / 2) - proj, N), rtol=0, atol=1e-12)


def test_gaussian_blob_closed_form():
    """G5: a band-limited Gaussian projects to A sqrt(2 pi) sg exp(-(s - c.e)^2 / 2 sg^2)."""
    n = 64
    cx, cy, sg, A = 5.3, -7.1, 3.0, 1.7
    x = gaussian_blob(n, cx, cy, sg, A)
    ang = uniform_angles(16)
    y = radon_exact(x, ang, n)
    s = np.arange(n) - n / 2
    ref = np.stack([A * np.sqrt(2 * np.pi) * sg *
                    np.exp(-(s - (cx * np.cos(t) + cy * np.sin(t))) ** 2 / (2 * sg * sg))
                    for t in ang])
    assert np.abs(y - ref).max() < 1e-9 * np.abs(ref).max()


def test_adjoint_identity():
    """G7: <A x, y> = <x, A^T y>."""
    n, N = 16, 20
    ang = np.random.default_rng(5).uniform(0, np.pi, 11)
    x = random_image(6, n).astype(np.float64)
    y = random_sinogram(7, 11, N).astype(np.float64)
    Ax = radon_exact(x, ang, N)
    Aty = radon_exact_adjoint(y, ang, n)
    lhs, rhs = np.sum(Ax * y), np.sum(x * Aty)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_dense_matrix_transpose_n8():
    """G8: at n=8 the adjoint's matrix is the transpose of the forward's, and
    every forward entry equals the Dirichlet closed form."""
    n, N = 8, 8
    ang = np.array([0.0, 0.4, np.pi / 2, 2.5, 3.0])
    nv = len(ang)
    A = np.zeros((nv * N, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        A[:, k] = radon_exact(e.reshape(n, n), ang, N).ravel()
    At = np.zeros((n * n, nv * N))
    for k in range(nv * N):
        e = np.zeros(nv * N)
        e[k] = 1.0
        At[:, k] = radon_exact_adjoint(e.reshape(nv, N), ang, n).ravel()
    assert np.abs(At - A.T).max() < 1e-12
    xs = np.arange(n) - n / 2
    s = np.arange(N) - N / 2
    for a, t in enumerate(ang):
        proj = (np.cos(t) * xs[None, :] + np.sin(t) * xs[:, None]).ravel()
        ref = dirichlet_re(s[:, None] - proj[None, :], N)
        assert np.abs(A[a * N:(a + 1) * N] - ref).max() < 1e-12
