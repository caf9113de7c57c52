"""O-exact: the discrete Fourier-slice Radon transform with exact interpolation
(oracle, test infrastructure).

Section "fast radon transform", paragraph 1: Radon{x} is a 2D Fourier
transform of x, taken on the polar grid, followed by 1D inverse Fourier
transforms along each radial line. Taking the polar values exactly (a type-2
non-uniform DFT instead of interpolation from a Cartesian grid) gives the
transform that gridding approximates (paragraph 2: gridding "allows us to
perform a non-uniform FFT"):

    X_a[q]  = sum_p x[p] exp(-2 pi i k_{a,q} . p),     k_{a,q} = (q/N) e_a
    y[a,d]  = Re( (1/N) sum_q X_a[q] exp(+2 pi i q s_d / N) )

The "inverse Radon" the solver needs is read as the exact transpose of this
real-to-real map (the solver of the problem statement needs A and A^T):

    Yhat_a[q] = (1/N) sum_d y[a,d] exp(-2 pi i q s_d / N)
    (A^T y)[p] = Re sum_{a,q} Yhat_a[q] exp(+2 pi i k_{a,q} . p)

Cost is O(n^2 * n_views * N): for tiny inputs only.
"""
from __future__ import annotations

import numpy as np

from .geometry import angle_cos_sin, ray_q

__all__ = ["radon_exact", "radon_exact_adjoint", "ray_synthesis_matrix"]


def _pixel_coords(n: int):
    idx = np.arange(n, dtype=np.float64) - n / 2
    px = np.broadcast_to(idx[None, :], (n, n)).ravel()   # column offset j - n/2
    py = np.broadcast_to(idx[:, None], (n, n)).ravel()   # row offset    i - n/2
    return px, py


def ray_synthesis_matrix(n_det: int) -> np.ndarray:
    """E[q, d] = exp(+2 pi i q s_d / N): the 1D inverse DFT along one ray."""
    q = ray_q(n_det).astype(np.float64)
    s = np.arange(n_det, dtype=np.float64) - n_det / 2
    return np.exp(2j * np.pi * np.outer(q, s) / n_det)


def radon_exact(x, angles, n_det: int) -> np.ndarray:
    """Forward transform, float64 (n_views, n_det)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    assert x.shape == (n, n)
    c, s = angle_cos_sin(angles)
    px, py = _pixel_coords(n)
    q = ray_q(n_det).astype(np.float64)
    E = ray_synthesis_matrix(n_det)
    xv = x.ravel()
    y = np.empty((len(c), n_det), dtype=np.float64)
    for a in range(len(c)):
        proj = c[a] * px + s[a] * py                       # e_a . p
        X = np.exp(-2j * np.pi * np.outer(q, proj) / n_det) @ xv
        y[a] = (X @ E).real / n_det
    return y


def radon_exact_adjoint(y, angles, n: int) -> np.ndarray:
    """Exact transpose of ``radon_exact``, float64 (n, n)."""
    y = np.asarray(y, dtype=np.float64)
    n_views, n_det = y.shape
    c, s = angle_cos_sin(angles)
    assert len(c) == n_views
    px, py = _pixel_coords(n)
    q = ray_q(n_det).astype(np.float64)
    E = ray_synthesis_matrix(n_det)
    Yhat = (y @ np.conj(E).T) / n_det                     # (n_views, N)
    acc = np.zeros(n * n, dtype=np.complex128)
    for a in range(n_views):
        proj = c[a] * px + s[a] * py
        acc += Yhat[a] @ np.exp(2j * np.pi * np.outer(q, proj) / n_det)
    return acc.real.reshape(n, n)
