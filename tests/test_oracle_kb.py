"""Pins for the Kaiser-Bessel kernel and deapodization of the oracle.

phi and phihat are pinned against each other through the Fourier integral
(numerical quadrature), and phi against its defining properties; a mistake in
either function (wrong beta use, wrong width, a dropped factor W or 1/I0)
breaks the quadrature identity.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle.kb import deapod_factors, kb_beta, kb_phi, kb_phihat


@pytest.mark.parametrize("W,sigma", [(6, 2.0), (4, 2.0), (8, 2.0), (6, 1.5)])
def test_phi_shape(W, sigma):
    beta = kb_beta(W, sigma)
    assert kb_phi(0.0, W, beta) == pytest.approx(1.0, abs=1e-15)
    # strict support: zero at and beyond W/2
    assert kb_phi(W / 2, W, beta) == 0.0
    assert kb_phi(-W / 2, W, beta) == 0.0
    assert kb_phi(W / 2 + 0.3, W, beta) == 0.0
    # even and strictly decreasing on [0, W/2)
    t = np.linspace(0.0, W / 2 - 1e-9, 2001)
    p = kb_phi(t, W, beta)
    assert np.array_equal(p, kb_phi(-t, W, beta))
    assert np.all(np.diff(p) < 0)
    # the limit from inside the support is 1/I0(beta)
    from scipy.special import i0
    assert kb_phi(W / 2 - 1e-12, W, beta) == pytest.approx(1.0 / i0(beta), rel=1e-6)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("W,sigma", [(6, 2.0), (4, 2.0), (8, 2.0)])
@pytest.mark.parametrize("f", [0.0, 0.05, 0.137, 0.25, 0.5, 0.9, 1.3])
def test_phihat_is_fourier_transform_of_phi(W, sigma, f):
    """G12: phihat(f) = integral of phi(t) cos(2 pi f t) dt (phi even)."""
    beta = kb_beta(W, sigma)
    val, err = quad(lambda t: kb_phi(t, W, beta) * np.cos(2 * np.pi * f * t),
                    -W / 2, W / 2, limit=400, epsabs=1e-13, epsrel=1e-12)
    assert kb_phihat(f, W, beta) == pytest.approx(val, rel=1e-9, abs=1e-13)


def test_deapod_factors_symmetric_and_centred():
    n, G, W = 64, 128, 6
    beta = kb_beta(W, 2.0)
    psi = deapod_factors(n, G, W, beta)
    # psi[n/2] = phihat(0) = integral of phi
    total, _ = quad(lambda t: kb_phi(t, W, beta), -W / 2, W / 2, epsabs=1e-14)
    assert psi[n // 2] == pytest.approx(total, rel=1e-12)
    # symmetric about the centre pixel
    k = np.arange(1, n // 2)
    assert np.allclose(psi[n // 2 + k], psi[n // 2 - k], rtol=0, atol=1e-15)
    # positive, peaked at the centre
    assert np.all(psi > 0) and np.argmax(psi) == n // 2


def test_beta_matches_published_rule_value():
    """Beatty et al. 2005 rule at W=6, sigma=2: pi*sqrt(9*2.25-0.8) = 13.8551."""
    assert kb_beta(6, 2.0) == pytest.approx(13.855096, abs=1e-5)
