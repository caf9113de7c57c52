"""Write the oracle regression snapshot (calls only oracle/ and radon_inputs).

The paper prints no worked example of the transform (its only numbers are
timings, section "fast radon transform", last paragraph), so the stored values
here are the oracle's own outputs on a fixed tiny input. They guard the
oracle against silent changes; the oracle itself is pinned by the closed-form,
invariant and brute-force tests. Regenerate only together with an oracle
change whose commit message names the passage that justifies it.

    python tests/golden/make_oracle_snapshot.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle.binning import sample_keys, stable_sort  # noqa: E402
from oracle.exact import radon_exact, radon_exact_adjoint  # noqa: E402
from oracle.geometry import polar_uv  # noqa: E402
from oracle.grid import grid_adjoint, grid_forward  # noqa: E402
from radon_inputs import random_image, random_sinogram  # noqa: E402


def main():
    n, N, W, sigma, T = 8, 8, 6, 2.0, 8
    angles = [0.0, 0.4, np.pi / 2, 2.5]
    x = random_image(101, n).astype(np.float64)
    y = random_sinogram(102, len(angles), N).astype(np.float64)
    u, v = polar_uv(np.array(angles), N, int(sigma * n))
    keys = sample_keys(u, v, int(sigma * n), W, T).ravel()
    out = {
        "about": "oracle outputs on a fixed tiny input (regression guard); see make_oracle_snapshot.py",
        "n": n, "n_det": N, "W": W, "sigma": sigma, "T": T, "angles": angles,
        "x_seed": 101, "y_seed": 102,
        "exact_forward": radon_exact(x, angles, N).tolist(),
        "exact_adjoint": radon_exact_adjoint(y, angles, n).tolist(),
        "grid_forward": grid_forward(x, angles, N, sigma, W).tolist(),
        "grid_adjoint": grid_adjoint(y, angles, n, sigma, W).tolist(),
        "keys": keys.tolist(),
        "perm": stable_sort(keys).tolist(),
    }
    with open(os.path.join(HERE, "oracle_snapshot_n8.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
