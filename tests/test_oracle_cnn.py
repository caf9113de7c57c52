"""Pins of the reference warm-start network (oracle/cnn.py).

The network is this project's design, not the paper's, so the pins check
that the reference computes what its definition says: the last layer starts
the network as the identity, a hand-built parameter set reduces the whole
network to one explicitly looped 3x3 cross-correlation, the whole network
with random weights equals a forward written out in loops (average pooling,
nearest upsampling and the skip of every level included), and autograd's
gradient agrees with central differences. Planted one-change copies of the
network (max pooling, bilinear upsampling, a decoder conv one level coarse,
a skip taken before the ReLU, a skip added inside the ReLU, a dropped skip)
must each fail the looped forward.
"""
import numpy as np
import pytest

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


# --- an independent forward of the whole network, written out in loops

def _conv3(a, w, b):
    """3x3 cross-correlation, stride 1, zero padding 1: out[o, i, j] = b[o] +
    sum_{c, dy, dx} w[o, c, dy+1, dx+1] a[c, i+dy, j+dx] (zero outside)."""
    C, H, W = a.shape
    ap = np.zeros((C, H + 2, W + 2))
    ap[:, 1:-1, 1:-1] = a
    out = np.empty((w.shape[0], H, W))
    for i in range(H):
        for j in range(W):
            patch = ap[:, i:i + 3, j:j + 3]                       # (C, 3, 3) around (i, j)
            out[:, i, j] = b + np.tensordot(w, patch, axes=([1, 2, 3], [0, 1, 2]))
    return out


def _avgpool2(a):
    C, H, W = a.shape
    out = np.empty((C, H // 2, W // 2))
    for i in range(H // 2):
        for j in range(W // 2):
            out[:, i, j] = 0.25 * (a[:, 2 * i, 2 * j] + a[:, 2 * i + 1, 2 * j] +
                                   a[:, 2 * i, 2 * j + 1] + a[:, 2 * i + 1, 2 * j + 1])
    return out


def _nearest2(a):
    C, H, W = a.shape
    out = np.empty((C, 2 * H, 2 * W))
    for i in range(2 * H):
        for j in range(2 * W):
            out[:, i, j] = a[:, i // 2, j // 2]
    return out


def _looped_forward(p, x):
    sl = _layer_slices()
    L = [(p[ws].reshape(co, ci, 3, 3), p[bs]) for (ws, bs), (ci, co) in zip(sl, CHANNELS)]
    relu = lambda t: np.maximum(t, 0.0)   # noqa: E731
    e0 = relu(_conv3(x[None], *L[0]))
    e1 = relu(_conv3(_avgpool2(e0), *L[1]))
    e2 = relu(_conv3(_avgpool2(e1), *L[2]))
    e3 = relu(_conv3(_avgpool2(e2), *L[3]))
    d2 = relu(_conv3(_nearest2(e3), *L[4])) + e2
    d1 = relu(_conv3(_nearest2(d2), *L[5])) + e1
    d0 = relu(_conv3(_nearest2(d1), *L[6])) + e0
    return _conv3(d0, *L[7])[0] + x


def _random_params(seed):
    """He-scaled weights and biases of both signs, so every ReLU is active on
    part of its input and every level contributes to the output."""
    rng = np.random.default_rng(seed)
    p = _zeros()
    for (ws, bs), (ci, co) in zip(_layer_slices(), CHANNELS):
        p[ws] = rng.standard_normal(ws.stop - ws.start) * np.sqrt(2.0 / (9 * ci))
        p[bs] = 0.1 * rng.standard_normal(co)
    return p


def _looped_error(seed=5, H=16, W=16):
    p = _random_params(seed)
    x = np.random.default_rng(seed + 1).standard_normal((1, H, W))
    y = forward(p, x)[0]
    ref = _looped_forward(p, x[0])
    return float(np.abs(y - ref).max() / np.abs(ref - x[0]).max())


def test_whole_network_matches_looped_forward():
    """Pooling (2x2 average), upsampling (nearest), the skip of every level and
    every layer, all at once, against the loops above (16 x 16: levels 16, 8,
    4, 2)."""
    assert _looped_error() <= 1e-12


# planted mistakes: one-change copies of the oracle's network, each caught by
# the looped forward

def _net_variant(pool="avg", up="nearest", skip="ok"):
    import torch
    import torch.nn.functional as Fn

    def net(layers, x):
        conv = lambda i, t: Fn.conv2d(t, layers[i][0], layers[i][1], padding=1)   # noqa: E731
        pl = (lambda t: Fn.max_pool2d(t, 2)) if pool == "max" else (lambda t: Fn.avg_pool2d(t, 2))
        if up == "bilinear":
            u = lambda t: Fn.interpolate(t, scale_factor=2, mode="bilinear", align_corners=False)  # noqa: E731
        else:
            u = lambda t: Fn.interpolate(t, scale_factor=2, mode="nearest")  # noqa: E731
        e0 = torch.relu(conv(0, x))
        e1 = torch.relu(conv(1, pl(e0)))
        e2 = torch.relu(conv(2, pl(e1)))
        e3 = torch.relu(conv(3, pl(e2)))
        # a skip tensor from another level has another channel count, so the
        # plausible level mistakes are the decoder conv run one level coarser
        # (before the upsampling) and the skip taken before the encoder's ReLU
        s2 = conv(2, pl(e1)) if skip == "pre_relu" else e2
        if skip == "inside_relu":
            d2 = torch.relu(conv(4, u(e3)) + s2)
        elif skip == "conv_coarse":
            d2 = u(torch.relu(conv(4, e3))) + s2
        else:
            d2 = torch.relu(conv(4, u(e3))) + s2
        d1 = torch.relu(conv(5, u(d2))) + (0 if skip == "dropped" else e1)
        d0 = torch.relu(conv(6, u(d1))) + e0
        return conv(7, d0) + x
    return net



@pytest.mark.parametrize("variant", [dict(), dict(pool="max"), dict(up="bilinear"), dict(skip="conv_coarse"), dict(skip="pre_relu"),
                                     dict(skip="inside_relu"), dict(skip="dropped")])
def test_planted_network_mistake_is_caught(monkeypatch, variant):
    import oracle.cnn as oc
    monkeypatch.setattr(oc, "_net", _net_variant(**variant))
    err = _looped_error()
    if variant:
        assert err > 1e-3, (variant, err)
    else:
        assert err <= 1e-12        # the unchanged copy passes
