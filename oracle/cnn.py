"""Reference of the learned warm start's network (oracle, test infrastructure).

The paper has no learned component; the network is this project's extension
(a start image for the basis-pursuit solve). Its plain definition, in float64
with PyTorch CPU operations and autograd:

    e0 = relu(conv_a(x))            32 channels, full size
    e1 = relu(conv_b(pool(e0)))     64, 1/2
    e2 = relu(conv_c(pool(e1)))    128, 1/4
    e3 = relu(conv_d(pool(e2)))    256, 1/8
    d2 = relu(conv_e(up(e3))) + e2
    d1 = relu(conv_f(up(d2))) + e1
    d0 = relu(conv_g(up(d1))) + e0
    y  = conv_h(d0) + x

conv: 3x3, stride 1, zero padding 1, with bias; pool: 2x2 average; up:
nearest 2x. Parameters are one flat array in layer order, each layer's
weights (Cout, Cin, 3, 3) followed by its biases. Loss: mean squared error.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

__all__ = ["CHANNELS", "unpack", "forward", "loss_and_grads"]

CHANNELS = [(1, 32), (32, 64), (64, 128), (128, 256), (256, 128), (128, 64), (64, 32), (32, 1)]


def unpack(params):
    """Flat parameter array -> list of (w, b) float64 tensors."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, off = [], 0
    for cin, cout in CHANNELS:
        nw = cout * cin * 9
        w = p[off:off + nw].reshape(cout, cin, 3, 3)
        b = p[off + nw:off + nw + cout]
        out.append((w, b))
        off += nw + cout
    if off != p.numel():
        raise ValueError(f"expected {off} parameters, got {p.numel()}")
    return out


def _net(layers, x):
    conv = lambda i, t: Fn.conv2d(t, layers[i][0], layers[i][1], padding=1)   # noqa: E731
    pool = lambda t: Fn.avg_pool2d(t, 2)                                       # noqa: E731
    up = lambda t: Fn.interpolate(t, scale_factor=2, mode="nearest")           # noqa: E731
    e0 = torch.relu(conv(0, x))
    e1 = torch.relu(conv(1, pool(e0)))
    e2 = torch.relu(conv(2, pool(e1)))
    e3 = torch.relu(conv(3, pool(e2)))
    d2 = torch.relu(conv(4, up(e3))) + e2
    d1 = torch.relu(conv(5, up(d2))) + e1
    d0 = torch.relu(conv(6, up(d1))) + e0
    return conv(7, d0) + x


def forward(params, x) -> np.ndarray:
    """y for a batch x (B, H, W), float64."""
    layers = unpack(params)
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64))[:, None]
    with torch.no_grad():
        return _net(layers, xt)[:, 0].numpy()


def loss_and_grads(params, x, target):
    """Mean squared error of the network's output against target, and its
    gradient with respect to the flat parameter array (float64)."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64)).clone().requires_grad_(True)
    layers, off = [], 0
    for cin, cout in CHANNELS:
        nw = cout * cin * 9
        layers.append((p[off:off + nw].reshape(cout, cin, 3, 3), p[off + nw:off + nw + cout]))
        off += nw + cout
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64))[:, None]
    tt = torch.as_tensor(np.asarray(target, dtype=np.float64))[:, None]
    loss = ((_net(layers, xt) - tt) ** 2).mean()
    loss.backward()
    return float(loss), p.grad.numpy().copy()
