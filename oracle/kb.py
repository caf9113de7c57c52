"""Kaiser-Bessel gridding kernel and deapodization (oracle, test infrastructure).

The paper says gridding convolves the irregular samples with "a kernel
calculated at regular sample position" and refers to Jackson et al. for it
(section "fast radon transform", paragraph 3). The kernel family, width and
shape are not given; the reading taken is the Kaiser-Bessel kernel of Jackson
et al. (1991) with Beatty et al.'s (2005) shape parameter:

    beta      = pi * sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8)
    phi(t)    = I0(beta sqrt(1 - (2t/W)^2)) / I0(beta)   for |t| < W/2, else 0
    phihat(f) = (W / I0(beta)) sinh(z) / z,  z = sqrt(beta^2 - (pi W f)^2)

phihat is the continuous Fourier transform of phi (integral of
phi(t) exp(-2 pi i f t) dt); for (pi W f) > beta, sinh(z)/z becomes sin(z')/z'.
Support is strict: phi(+-W/2) = 0 although the limit from inside is 1/I0(beta).
"""
from __future__ import annotations

import numpy as np
from scipy.special import i0

__all__ = ["kb_beta", "kb_phi", "kb_phihat", "deapod_factors"]


def kb_beta(W: int, sigma: float) -> float:
    """Beatty-Brodsky-Nishimura-Pauly shape parameter for width W, oversampling sigma."""
    return float(np.pi * np.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8))


def kb_phi(t, W: int, beta: float) -> np.ndarray:
    """phi(t), strict support |t| < W/2, phi(0) = 1."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    inside = np.abs(t) < W / 2.0
    r = 2.0 * t[inside] / W
    out[inside] = i0(beta * np.sqrt(1.0 - r * r)) / i0(beta)
    return out


def kb_phihat(f, W: int, beta: float) -> np.ndarray:
    """Continuous Fourier transform of kb_phi at frequency f (cycles per unit)."""
    f = np.asarray(f, dtype=np.float64)
    z2 = beta * beta - (np.pi * W * f) ** 2
    out = np.empty_like(f)
    pos = z2 > 0
    neg = z2 < 0
    zero = ~(pos | neg)
    zp = np.sqrt(z2[pos])
    out[pos] = np.sinh(zp) / zp
    zn = np.sqrt(-z2[neg])
    out[neg] = np.sin(zn) / zn
    out[zero] = 1.0
    return out * (W / i0(beta))


def deapod_factors(n: int, G: int, W: int, beta: float) -> np.ndarray:
    """psi1[i] = phihat((i - n/2) / G), i = 0..n-1 (pixel coordinate / grid size)."""
    return kb_phihat((np.arange(n, dtype=np.float64) - n / 2) / G, W, beta)
