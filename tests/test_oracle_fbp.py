"""Pins for the oracle's filtered adjoint (filtered back-projection).

The ramp weights are checked against the closed-form cosine series of the
spatial Ramachandran-Lakshminarayanan kernel (no FFT), and the whole
filtered adjoint against the inversion it is meant to perform: FBP of the
projections of a band-limited Gaussian returns the Gaussian inside the
inscribed circle, with an error that falls with n.
"""
import numpy as np
import pytest

from oracle.grid import fbp_weights, grid_fbp, grid_forward
from radon_inputs import gaussian_blob, uniform_angles


@pytest.mark.parametrize("N", [8, 24, 128, 2560])
def test_ramp_weights_closed_form(N):
    nv = 90
    w = fbp_weights(nv, N)
    q = np.arange(N) - N // 2
    kk = np.arange(1, N // 2, 2)                   # odd k in (0, N/2)
    H = 0.25 - 2.0 * np.sum(np.cos(2 * np.pi * np.outer(q, kk) / N) / (np.pi * kk) ** 2, axis=1)
    assert np.allclose(w, (np.pi / nv) * H, rtol=0, atol=1e-14)
    # close to |q|/N away from DC, small positive DC weight, even in q
    nz = (q != 0) & (q != -N // 2)
    assert np.all(np.abs(w[nz] * nv / np.pi - np.abs(q[nz]) / N) <= 0.03 * np.abs(q[nz]) / N + 1e-12)
    assert 0 < w[N // 2] < (np.pi / nv) * 0.25 / N * 1.0
    assert np.allclose(w[1:], w[1:][::-1], atol=1e-15)


@pytest.mark.parametrize("n,tol", [(64, 1e-2), (128, 2e-3), (256, 3e-4)])
def test_fbp_inverts_projection_of_gaussian(n, tol):
    x = gaussian_blob(n, 7.3, -5.1, 4.0) + 0.5 * gaussian_blob(n, -12.0, 9.0, 3.0)
    ang = uniform_angles(2 * n)
    r = grid_fbp(grid_forward(x, ang, n), ang, n)
    xs = np.arange(n) - n / 2
    inside = np.sqrt(xs[None, :] ** 2 + xs[:, None] ** 2) < n / 2 - 2
    err = np.linalg.norm(r[inside] - x[inside]) / np.linalg.norm(x[inside])
    assert err < tol
