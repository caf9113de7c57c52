"""Pins of the reference warm-start network (oracle/cnn.py).

The network is this project's design, not the paper's, so the pins check
that the reference computes what its definition says: the last layer starts
the network as the identity, a hand-built parameter set reduces the whole
network to one explicitly looped 3x3 cross-correlation, and autograd's
gradient agrees with central differences.
"""
import numpy as np

from oracle.cnn import CHANNELS, forward, loss_and_grads


def _zeros():
    return np.zeros(sum(co * ci * 9 + co for ci, co in CHANNELS))


def _layer_slices():
    out, off = [], 0
    for ci, co in CHANNELS:
        nw = co * ci * 9
        out.append((slice(off, off + nw), slice(off + nw, off + nw + co)))
        off += nw + co
    return out


def test_zero_last_layer_is_identity():
    rng = np.random.default_rng(0)
    p = 0.1 * rng.standard_normal(_zeros().size)
    ws, bs = _layer_slices()[-1]
    p[ws] = 0.0
    p[bs] = 0.0
    x = rng.standard_normal((2, 16, 24))
    assert np.allclose(forward(p, x), x, atol=1e-14)


def test_network_reduces_to_one_correlation():
    """conv_a passes relu(x) into channel 0 (centre tap 1), every other layer
    is zero except conv_h, whose channel-0 kernel K and bias c act on d0 = e0:
    y = x + c + sum_{dy,dx} K[dy+1, dx+1] relu(x)[i+dy, j+dx] (zero outside)."""
    rng = np.random.default_rng(1)
    p = _zeros()
    sl = _layer_slices()
    wa = np.zeros((32, 1, 3, 3))
    wa[0, 0, 1, 1] = 1.0
    p[sl[0][0]] = wa.ravel()
    K = rng.standard_normal((3, 3))
    wh = np.zeros((1, 32, 3, 3))
    wh[0, 0] = K
    p[sl[7][0]] = wh.ravel()
    p[sl[7][1]] = 0.25
    x = rng.standard_normal((1, 8, 16))
    y = forward(p, x)
    r = np.maximum(x[0], 0.0)
    ref = x[0] + 0.25
    H, W = r.shape
    for i in range(H):
        for j in range(W):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if 0 <= i + dy < H and 0 <= j + dx < W:
                        ref[i, j] += K[dy + 1, dx + 1] * r[i + dy, j + dx]
    assert np.allclose(y[0], ref, atol=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = 0.2 * rng.standard_normal(_zeros().size)
    x = rng.standard_normal((1, 8, 8))
    t = rng.standard_normal((1, 8, 8))
    f0, g = loss_and_grads(p, x, t)
    h = 1e-6
    for k in rng.choice(p.size, 12, replace=False):
        e = np.zeros_like(p)
        e[k] = h
        fp, _ = loss_and_grads(p + e, x, t)
        fm, _ = loss_and_grads(p - e, x, t)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
