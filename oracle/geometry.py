"""Polar sample geometry (oracle, test infrastructure).

Discretisation readings (the paper is silent on them; section "fast radon
transform" only says the 2D transform is interpolated "onto a polar grid" and
1D inverse transforms are taken "along the same radial lines"):

  * image pixel (i, j) is the point (px, py) = (j - n/2, i - n/2);
  * detector bin d is the signed offset s_d = d - N/2 (unit spacing, N = n_det);
  * view a has direction e_a = (cos theta_a, sin theta_a); theta = 0 projects
    along y, so its sinogram row is the column sums of the image;
  * ray a carries N frequency samples q = -N/2 .. N/2-1 at radius q/N
    cycles/pixel, i.e. at k_{a,q} = (q/N) e_a; sample j = a*N + q + N/2;
  * on an oversampled grid of G = sigma*n points the sample sits at grid
    coordinates (u, v) = (G q / N) (cos theta_a, sin theta_a).

Per-angle cos/sin come from ``math.cos``/``math.sin`` (the C library), and
(u, v) is one IEEE float64 division G*q/N followed by one multiplication, so
any other code that makes the same two operations on the same cos/sin gets
bit-identical floor(u), floor(v).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["angle_cos_sin", "ray_q", "polar_uv"]


def angle_cos_sin(angles):
    """Per-view (cos theta, sin theta) in float64 from the C library."""
    a = np.asarray(angles, dtype=np.float64)
    c = np.array([math.cos(float(t)) for t in a], dtype=np.float64)
    s = np.array([math.sin(float(t)) for t in a], dtype=np.float64)
    return c, s


def ray_q(n_det: int) -> np.ndarray:
    """Signed radial index q = -N/2 .. N/2-1 of the samples on one ray."""
    return np.arange(n_det, dtype=np.int64) - n_det // 2


def polar_uv(angles, n_det: int, G: int, q=None):
    """Grid coordinates (u, v) of samples, shape (n_views, len(q)).

    u = (G*q/N) * cos theta_a, v = (G*q/N) * sin theta_a, in float64.
    """
    c, s = angle_cos_sin(angles)
    if q is None:
        q = ray_q(n_det)
    q = np.asarray(q, dtype=np.int64)
    fq = (G * q).astype(np.float64) / float(n_det)
    u = fq[None, :] * c[:, None]
    v = fq[None, :] * s[:, None]
    return u, v
