"""Sample-to-tile keys and their stable sort (oracle, test infrastructure).

The paper load-balances gridding by splitting the sample set into bins (start
with one bin, repeatedly split the costliest bin into four, cost = samples x
grid points; one thread block per bin; section "fast radon transform",
paragraph 4). It prints no bins and no stop rule. The reading taken here is
uniform T x T tiles of the oversampled grid, keyed by the tile that holds the
first (top-left) point of each sample's W x W footprint, in centred grid
coordinates:

    o_u = (floor(u) - W/2 + 1 + G/2) mod G         (likewise o_v from v)
    key = (o_v div T) * (G/T) + (o_u div T)

and a stable sort of the samples by key (ties keep increasing sample index).
With W <= T a footprint whose origin is in tile (tx, ty) lies inside tiles
tx..tx+1 by ty..ty+1, so the samples touching an output tile are those of its
own bin and of its left, upper and upper-left neighbours.

Within a bin the samples are further grouped by which tile edges their
footprint crosses (edge class: 0 inside the tile, 1 crosses only the edge of
increasing o_u, 2 crosses both, 3 crosses only the edge of increasing o_v), so
that each neighbouring tile reads one contiguous run of the samples that
actually reach it: the u-neighbour classes 1-2, the v-neighbour classes 2-3,
the diagonal neighbour class 2. The refined key is 4 * key + class.
"""
from __future__ import annotations

import numpy as np

__all__ = ["sample_keys", "edge_class", "refined_keys", "stable_sort", "bin_offsets"]


def sample_keys(u, v, G: int, W: int, T: int) -> np.ndarray:
    """Tile key of each sample's footprint origin, int64, same shape as u."""
    if G % T or (G // 2) % T:
        raise ValueError("T must divide G/2")
    ou = (np.floor(u).astype(np.int64) - W // 2 + 1 + G // 2) % G
    ov = (np.floor(v).astype(np.int64) - W // 2 + 1 + G // 2) % G
    return (ov // T) * (G // T) + (ou // T)


def edge_class(u, v, G: int, W: int, T: int) -> np.ndarray:
    """0: footprint inside its tile; 1: crosses the o_u edge only; 2: both;
    3: the o_v edge only."""
    ou = (np.floor(u).astype(np.int64) - W // 2 + 1 + G // 2) % G
    ov = (np.floor(v).astype(np.int64) - W // 2 + 1 + G // 2) % G
    cu = (ou % T) + W - 1 >= T
    cv = (ov % T) + W - 1 >= T
    return np.where(cu & cv, 2, np.where(cu, 1, np.where(cv, 3, 0))).astype(np.int64)


def refined_keys(u, v, G: int, W: int, T: int) -> np.ndarray:
    """4 * tile key + edge class."""
    return 4 * sample_keys(u, v, G, W, T) + edge_class(u, v, G, W, T)


def stable_sort(keys) -> np.ndarray:
    """Permutation that sorts keys, ties in increasing index (int64)."""
    return np.argsort(np.asarray(keys).ravel(), kind="stable")


def bin_offsets(keys, n_bins: int) -> np.ndarray:
    """offsets[b] = number of keys < b, b = 0..n_bins (int64, length n_bins+1)."""
    counts = np.bincount(np.asarray(keys).ravel(), minlength=n_bins)
    return np.concatenate([[0], np.cumsum(counts)])
