"""Pins for the sample-to-tile keys and their stable sort.

The keys are checked against what they are for: the tile with a given key
contains each sample's footprint origin, and every grid point of the footprint
lies in that tile or its right/lower/lower-right neighbours (so an output tile
needs only its own and three neighbouring bins). The sort is checked against
Python's own ``sorted`` on (key, index) pairs, and the offsets against a
direct count.
"""
import math

import numpy as np
import pytest

from oracle.binning import bin_offsets, edge_class, refined_keys, sample_keys, stable_sort
from oracle.geometry import angle_cos_sin, polar_uv, ray_q
from radon_inputs import uniform_angles


@pytest.mark.parametrize("n,N,nv,T", [(16, 16, 12, 8), (32, 24, 20, 16), (64, 64, 30, 32)])
def test_keys_cover_footprints(n, N, nv, T):
    G, W = 2 * n, 6
    ang = uniform_angles(nv)
    u, v = polar_uv(ang, N, G)
    keys = sample_keys(u, v, G, W, T)
    nt = G // T
    for uu, vv, k in zip(u.ravel(), v.ravel(), keys.ravel()):
        tx, ty = int(k) % nt, int(k) // nt
        # centred grid coordinates of every footprint point
        fx = [(math.floor(uu) + a + G // 2) % G for a in range(-W // 2 + 1, W // 2 + 1)]
        fy = [(math.floor(vv) + g + G // 2) % G for g in range(-W // 2 + 1, W // 2 + 1)]
        assert fx[0] // T == tx and fy[0] // T == ty          # origin in own tile
        assert all(c // T in (tx, (tx + 1) % nt) for c in fx)   # rest in the next tile
        assert all(c // T in (ty, (ty + 1) % nt) for c in fy)


def test_stable_sort_matches_python_sorted():
    n, N, nv, T = 32, 32, 16, 8
    G, W = 2 * n, 6
    u, v = polar_uv(uniform_angles(nv), N, G)
    keys = sample_keys(u, v, G, W, T).ravel()
    perm = stable_sort(keys)
    ref = sorted(range(keys.size), key=lambda j: (int(keys[j]), j))
    assert perm.tolist() == ref
    offs = bin_offsets(keys, (G // T) ** 2)
    for b in range((G // T) ** 2):
        assert offs[b + 1] - offs[b] == int(np.sum(keys == b))
    assert offs[-1] == keys.size


def test_geometry_uses_one_multiply_per_coordinate():
    """u = (G q / N) * cos theta exactly (one division, one multiplication)."""
    ang = np.array([0.0, np.pi / 3, np.pi / 2, 2.0])
    N, G = 24, 40
    u, v = polar_uv(ang, N, G)
    c, s = angle_cos_sin(ang)
    for a in range(len(ang)):
        for t, q in enumerate(ray_q(N)):
            fq = (G * int(q)) / N                 # correctly rounded division
            assert u[a, t] == fq * math.cos(ang[a])
            assert v[a, t] == fq * math.sin(ang[a])
    # theta = pi/2: cos is +6.1e-17, so floor(u) is 0 for q > 0 and -1 for q < 0
    assert c[2] > 0 and c[2] < 1e-16
    q = ray_q(N)
    assert np.all(np.floor(u[2][q > 0]) == 0) and np.all(np.floor(u[2][q < 0]) == -1)


@pytest.mark.parametrize("n,N,nv,T", [(16, 16, 12, 8), (32, 24, 20, 16), (64, 64, 30, 32)])
def test_edge_class_matches_tiles_touched(n, N, nv, T):
    """Brute force: the class says exactly which neighbouring tiles the
    footprint reaches (class 0: own only; 1: +u; 3: +v; 2: +u, +v and diagonal)."""
    G, W = 2 * n, 6
    u, v = polar_uv(uniform_angles(nv), N, G)
    cls = edge_class(u, v, G, W, T)
    keys = sample_keys(u, v, G, W, T)
    rk = refined_keys(u, v, G, W, T)
    assert np.array_equal(rk, 4 * keys + cls)
    nt = G // T
    for uu, vv, c, k in zip(u.ravel(), v.ravel(), cls.ravel(), keys.ravel()):
        tx, ty = int(k) % nt, int(k) // nt
        touched = set()
        for a in range(-W // 2 + 1, W // 2 + 1):
            for g in range(-W // 2 + 1, W // 2 + 1):
                cx = ((math.floor(uu) + a + G // 2) % G) // T
                cy = ((math.floor(vv) + g + G // 2) % G) // T
                touched.add(((cx - tx) % nt, (cy - ty) % nt))
        expect = {0: {(0, 0)}, 1: {(0, 0), (1, 0)}, 3: {(0, 0), (0, 1)},
                  2: {(0, 0), (1, 0), (0, 1), (1, 1)}}[int(c)]
        assert touched == expect
