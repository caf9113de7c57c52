"""O-grid: FP64 gridding forward and adjoint Radon transform (oracle, test
infrastructure).

Section "fast radon transform": paragraph 1 gives the three steps (2D FFT on a
regular grid, interpolation onto the polar grid, 1D inverse FFTs along each
radial line); paragraphs 2-3 say the interpolation is done by gridding, a
convolution of the irregular samples with a kernel evaluated at regular grid
positions, and the reverse ("and vice versa") for the adjoint. The abstract
calls the pair "gridding and inverse gridding".

Readings for what the paper leaves open (kernel: ``kb``; sample positions:
``geometry``):

  forward
    1. x'[i,j] = x[i,j] / (psi1[i] psi1[j])                 (deapodize)
    2. P[py mod G, px mod G] = x'[p], zero elsewhere, G = sigma n  (zero-pad)
    3. Ghat = unnormalised 2D FFT of P (exp(-) sign)
    4. Xt[a,q] = sum_{alpha,gamma} phi(v - mv) phi(u - mu) Ghat[mv mod G, mu mod G]
       over mu = floor(u) + alpha, mv = floor(v) + gamma,
       alpha, gamma in {-W/2+1, ..., W/2} (the footprint wraps periodically)
    5. y[a,d] = Re((1/N) sum_q Xt[a,q] exp(+2 pi i q s_d / N))
  adjoint (exact transpose of the above, real inner product)
    1. Yhat[a,q] = (1/N) sum_d y[a,d] exp(-2 pi i q s_d / N)
    2. H[m] = sum_samples Yhat phi(v - mv) phi(u - mu) over the same footprints
    3. h = unnormalised inverse 2D FFT of H (exp(+) sign)
    4. (A^T y)[i,j] = Re(h[py mod G, px mod G]) / (psi1[i] psi1[j])

The FFTs are library calls (scipy.fft); everything else is written out.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from .exact import ray_synthesis_matrix
from .geometry import polar_uv
from .kb import deapod_factors, kb_beta, kb_phi

__all__ = ["GridParams", "grid_forward", "grid_adjoint", "grid_fbp", "fbp_weights", "grid_fft2",
           "grid_interp", "grid_spread", "ray_spectrum", "ray_synthesis"]

# FFT worker threads: the CPUs this process may use, at most 16 (the host
# share of one GPU on the machines this runs on).
_WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


class GridParams:
    """n, n_det, sigma, W and the derived G, beta, psi1."""

    def __init__(self, n: int, n_det: int, sigma: float = 2.0, W: int = 6):
        G = int(round(sigma * n))
        if abs(G - sigma * n) > 1e-9:
            raise ValueError("sigma * n must be an integer")
        self.n, self.n_det, self.sigma, self.W, self.G = n, n_det, float(sigma), int(W), G
        self.beta = kb_beta(W, sigma)
        self.psi = deapod_factors(n, G, W, self.beta)

    def offsets(self):
        """Footprint offsets alpha = -W/2+1 .. W/2 relative to floor(u)."""
        return range(-self.W // 2 + 1, self.W // 2 + 1)


def _pad_index(n: int, G: int):
    """Grid row/column that holds pixel row/column i: (i - n/2) mod G."""
    return (np.arange(n) - n // 2) % G


def grid_fft2(x, gp: GridParams) -> np.ndarray:
    """Steps 1-3 of the forward: deapodize, zero-pad, unnormalised FFT2."""
    xp = np.asarray(x, dtype=np.float64) / (gp.psi[:, None] * gp.psi[None, :])
    P = np.zeros((gp.G, gp.G), dtype=np.complex128)
    r = _pad_index(gp.n, gp.G)
    P[np.ix_(r, r)] = xp
    return sfft.fft2(P, workers=_WORKERS)


def grid_interp(Ghat, u, v, gp: GridParams) -> np.ndarray:
    """Step 4 of the forward: sum over each sample's W x W footprint."""
    G = gp.G
    bu = np.floor(u).astype(np.int64)
    bv = np.floor(v).astype(np.int64)
    wx = {a: kb_phi(u - (bu + a), gp.W, gp.beta) for a in gp.offsets()}
    wy = {g: kb_phi(v - (bv + g), gp.W, gp.beta) for g in gp.offsets()}
    out = np.zeros(u.shape, dtype=np.complex128)
    for g in gp.offsets():
        rows = (bv + g) % G
        for a in gp.offsets():
            cols = (bu + a) % G
            out += wy[g] * wx[a] * Ghat[rows, cols]
    return out


def grid_spread(Yhat, u, v, gp: GridParams) -> np.ndarray:
    """Step 2 of the adjoint: H[m] = sum of Yhat * phi * phi over footprints."""
    G = gp.G
    bu = np.floor(u).astype(np.int64).ravel()
    bv = np.floor(v).astype(np.int64).ravel()
    uu, vv, Y = u.ravel(), v.ravel(), np.asarray(Yhat).ravel()
    wx = {a: kb_phi(uu - (bu + a), gp.W, gp.beta) for a in gp.offsets()}
    wy = {g: kb_phi(vv - (bv + g), gp.W, gp.beta) for g in gp.offsets()}
    Hr = np.zeros(G * G, dtype=np.float64)
    Hi = np.zeros(G * G, dtype=np.float64)
    for g in gp.offsets():
        rows = (bv + g) % G
        for a in gp.offsets():
            flat = rows * G + (bu + a) % G
            w = wy[g] * wx[a]
            Hr += np.bincount(flat, weights=w * Y.real, minlength=G * G)
            Hi += np.bincount(flat, weights=w * Y.imag, minlength=G * G)
    return (Hr + 1j * Hi).reshape(G, G)


def ray_synthesis(Xt, n_det: int) -> np.ndarray:
    """Step 5 of the forward: y = Re((1/N) Xt E)."""
    return (np.asarray(Xt) @ ray_synthesis_matrix(n_det)).real / n_det


def ray_spectrum(y, n_det: int) -> np.ndarray:
    """Step 1 of the adjoint: Yhat = (1/N) y conj(E)^T."""
    return (np.asarray(y, dtype=np.float64) @ np.conj(ray_synthesis_matrix(n_det)).T) / n_det


def grid_forward(x, angles, n_det: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """O-grid forward Radon transform, float64 (n_views, n_det)."""
    x = np.asarray(x, dtype=np.float64)
    gp = GridParams(x.shape[0], n_det, sigma, W)
    Ghat = grid_fft2(x, gp)
    u, v = polar_uv(angles, n_det, gp.G)
    return ray_synthesis(grid_interp(Ghat, u, v, gp), n_det)


def grid_adjoint(y, angles, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """O-grid adjoint (transpose) Radon transform, float64 (n, n)."""
    y = np.asarray(y, dtype=np.float64)
    n_det = y.shape[1]
    gp = GridParams(n, n_det, sigma, W)
    u, v = polar_uv(angles, n_det, gp.G)
    H = grid_spread(ray_spectrum(y, n_det), u, v, gp)
    h = sfft.ifft2(H, workers=_WORKERS) * (gp.G * gp.G)
    r = _pad_index(n, gp.G)
    return h[np.ix_(r, r)].real / (gp.psi[:, None] * gp.psi[None, :])



def fbp_weights(n_views: int, n_det: int) -> np.ndarray:
    """Ramp weights w_q of the filtered adjoint, q = -N/2..N/2-1.

    The 2D inverse Fourier integral over the polar samples uses the area
    element |rho| drho dtheta, dtheta = pi/n_views over [0, pi). The ramp
    |rho| is taken as the DFT of the band-limited spatial ramp kernel
    (Ramachandran-Lakshminarayanan): h[0] = 1/4, h[k] = -1/(pi k)^2 for odd k,
    0 for even k != 0, on the N-periodic window |k| < N/2. It equals |q|/N up
    to a few per cent and gives the DC term its correct small weight.
    """
    k = np.arange(n_det) - n_det // 2
    h = np.zeros(n_det)
    h[n_det // 2] = 0.25
    odd = (k % 2) != 0
    h[odd] = -1.0 / (np.pi * k[odd]) ** 2
    H = np.fft.fft(np.fft.ifftshift(h)).real          # index q mod N
    return (np.pi / n_views) * np.fft.fftshift(H)       # q = -N/2 .. N/2-1


def grid_fbp(y, angles, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """Filtered adjoint (filtered back-projection through the Fourier slice
    theorem): the O-grid adjoint with the ray spectra weighted by fbp_weights.
    The paper's 'standard tomographic processing' of the projections
    (introduction) is read as this reconstruction."""
    y = np.asarray(y, dtype=np.float64)
    n_views, n_det = y.shape
    gp = GridParams(n, n_det, sigma, W)
    u, v = polar_uv(angles, n_det, gp.G)
    Yhat = ray_spectrum(y, n_det) * fbp_weights(n_views, n_det)[None, :]
    H = grid_spread(Yhat, u, v, gp)
    h = sfft.ifft2(H, workers=_WORKERS) * (gp.G * gp.G)
    r = _pad_index(n, gp.G)
    return h[np.ix_(r, r)].real / (gp.psi[:, None] * gp.psi[None, :])
