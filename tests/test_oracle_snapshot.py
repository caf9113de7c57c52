"""The oracle still reproduces its stored regression snapshot (tests/golden)."""
import json
import os

import numpy as np

from oracle.binning import sample_keys, stable_sort
from oracle.exact import radon_exact, radon_exact_adjoint
from oracle.geometry import polar_uv
from oracle.grid import grid_adjoint, grid_forward
from radon_inputs import random_image, random_sinogram

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_snapshot_n8():
    with open(os.path.join(HERE, "golden", "oracle_snapshot_n8.json")) as f:
        g = json.load(f)
    n, N, W, sigma, T, ang = g["n"], g["n_det"], g["W"], g["sigma"], g["T"], g["angles"]
    x = random_image(g["x_seed"], n).astype(np.float64)
    y = random_sinogram(g["y_seed"], len(ang), N).astype(np.float64)
    for name, val in [("exact_forward", radon_exact(x, ang, N)),
                      ("exact_adjoint", radon_exact_adjoint(y, ang, n)),
                      ("grid_forward", grid_forward(x, ang, N, sigma, W)),
                      ("grid_adjoint", grid_adjoint(y, ang, n, sigma, W))]:
        ref = np.array(g[name])
        assert np.abs(val - ref).max() <= 1e-12 * np.abs(ref).max(), name
    u, v = polar_uv(np.array(ang), N, int(sigma * n))
    keys = sample_keys(u, v, int(sigma * n), W, T).ravel()
    assert keys.tolist() == g["keys"]
    assert stable_sort(keys).tolist() == g["perm"]
