"""Work-decomposition tuning, the autotuner and uneven-slice batches (MI355X).

Every decomposition must give the same transform (checked against the FP64
gridding oracle); a batch recorded into a HIP graph must give, bit for bit,
what the per-slice calls give, on every replay, also with other work on the
stream between replays.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.grid import grid_adjoint, grid_forward  # noqa: E402
from radon_inputs import random_image, random_sinogram, uniform_angles  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1009_1380_amd import Batch, Plan, autotune  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,nv", [(48, 20), (64, 31)])
def test_tuned_plans_match_oracle(n, nv):
    note(f"tuned plans n={n} nv={nv}")
    ang = uniform_angles(nv)
    x = random_image(7, n)
    y = random_sinogram(8, nv, n)
    ref_f = grid_forward(x.astype(np.float64), ang, n)
    ref_a = grid_adjoint(y.astype(np.float64), ang, n)
    tiles = [t for t in (8, 16, 32) if (n % t) == 0]
    for tile in tiles:
        for a2 in (64, 512):
            for f3 in (256, 2048):
                plan = Plan(n, ang, n, tuning={"tile": tile, "a2_chunk": a2, "f3_chunk": f3})
                assert plan.tuning() == {"tile": tile, "a2_chunk": a2, "f3_chunk": f3}
                f = plan.forward(to_dev(x)).cpu().numpy()
                a = plan.adjoint(to_dev(y)).cpu().numpy()
                assert rel(f, ref_f) <= 1e-5, (tile, a2, f3)
                assert rel(a, ref_a) <= 1e-5, (tile, a2, f3)


def test_tuning_rejected():
    ang = uniform_angles(10)
    with pytest.raises(ValueError):
        Plan(48, ang, 48, tuning={"tile": 12})            # not a tile size
    with pytest.raises(ValueError):
        Plan(48, ang, 48, tuning={"tile": 32})            # 32 does not divide G/2 = 48
    with pytest.raises(ValueError):
        Plan(48, ang, 48, tuning={"a2_chunk": 1000})      # above the kernel's item capacity
    with pytest.raises(ValueError):
        Plan(48, ang, 48, tuning={"f3_chunk": 100})
    assert Plan(48, ang, 48).tuning() == {"tile": 16, "a2_chunk": 512, "f3_chunk": 2048}


SHAPES = [(16, 12), (24, 20), (32, 36), (48, 24), (64, 40), (40, 8), (32, 5)]


def _slices(shapes, seed=0):
    plans, imgs, sinos = [], [], []
    for k, (n, nv) in enumerate(shapes):
        ang = uniform_angles(nv) + 0.01 * k
        plans.append(Plan(n, ang, n))
        imgs.append(to_dev(random_image(seed + k, n)))
        sinos.append(to_dev(random_sinogram(seed + 100 + k, nv, n)))
    return plans, imgs, sinos


def test_batch_matches_per_slice_and_oracle():
    note("batch vs per-slice")
    plans, imgs, sinos = _slices(SHAPES)
    batch = Batch(plans, n_branches=3)
    outs_f = [torch.empty((p.n_views, p.n_det), device=DEV) for p in plans]
    outs_a = [torch.empty((p.n, p.n), device=DEV) for p in plans]
    batch.forward(imgs, outs_f)
    batch.adjoint(sinos, outs_a)
    torch.cuda.synchronize()
    for p, x, y, f, a in zip(plans, imgs, sinos, outs_f, outs_a):
        assert torch.equal(f, p.forward(x)) and torch.equal(a, p.adjoint(y))
        fo = grid_forward(x.cpu().numpy().astype(np.float64), p.angles, p.n)
        ao = grid_adjoint(y.cpu().numpy().astype(np.float64), p.angles, p.n)
        assert rel(f.cpu().numpy(), fo) <= 1e-5 and rel(a.cpu().numpy(), ao) <= 1e-5


def test_batch_graph_replays():
    note("batch graph replays")
    plans, imgs, sinos = _slices(SHAPES, seed=20)
    batch = Batch(plans, n_branches=4)
    outs = [torch.empty((p.n_views, p.n_det), device=DEV) for p in plans]
    refs = [p.forward(x).clone() for p, x in zip(plans, imgs)]
    junk = torch.randn(1 << 20, device=DEV)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        batch.forward(imgs, outs)
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r), rep
        # other work on the stream and the plans between replays
        junk = torch.sort(junk * 1.0001)[0]
        _ = plans[rep % len(plans)].adjoint(sinos[rep % len(plans)])
        torch.cuda.synchronize()
    assert batch.graphs_recorded() == 1
    # new output buffers record a new graph with the new pointers
    outs2 = [torch.empty_like(o) for o in outs]
    batch.forward(imgs, outs2)
    torch.cuda.synchronize()
    assert batch.graphs_recorded() == 2
    for o, r in zip(outs2, refs):
        assert torch.equal(o, r)


def test_batch_rejected():
    plans, imgs, sinos = _slices(SHAPES[:3])
    with pytest.raises(ValueError):
        Batch([plans[0], plans[1], plans[0]])            # a workspace used twice
    with pytest.raises(ValueError):
        Batch(plans, n_branches=0)
    batch = Batch(plans)
    outs = [torch.empty((p.n_views, p.n_det), device=DEV) for p in plans]
    with pytest.raises(ValueError):
        batch.forward(imgs[:2], outs[:2])                # wrong count (binding)
    with pytest.raises(ValueError):
        batch.forward([imgs[1], imgs[0], imgs[2]], outs)  # wrong shapes (binding)
    plans[1].set_profiling(True)
    with pytest.raises(ValueError):
        batch.forward(imgs, outs)                        # profiling events cannot be recorded
    plans[1].set_profiling(False)
    batch.forward(imgs, outs)
    torch.cuda.synchronize()


def test_batch_uneven_full_sizes_bitwise():
    """The uneven-slice workload's sizes: batch equals per-slice calls bit for bit."""
    note("batch at full sizes")
    shapes = [(512, 90), (1024, 180), (1536, 360), (2048, 720), (2560, 1024)]
    plans, imgs, sinos = _slices(shapes, seed=40)
    batch = Batch(plans, n_branches=4)
    outs_f = [torch.empty((p.n_views, p.n_det), device=DEV) for p in plans]
    outs_a = [torch.empty((p.n, p.n), device=DEV) for p in plans]
    batch.forward(imgs, outs_f)
    batch.adjoint(sinos, outs_a)
    torch.cuda.synchronize()
    for p, x, y, f, a in zip(plans, imgs, sinos, outs_f, outs_a):
        assert torch.equal(f, p.forward(x)) and torch.equal(a, p.adjoint(y))


def test_autotune_returns_a_working_decomposition():
    note("autotune")
    n, nv = 64, 40
    ang = uniform_angles(nv)
    best, best_ms, def_ms = autotune(n, ang, n, repeats=2)
    assert best["tile"] in (8, 16, 32) and best["a2_chunk"] in (256, 512) and best["f3_chunk"] in (1024, 2048, 4096)
    assert 0 < best_ms <= def_ms
    plan = Plan(n, ang, n, tuning=best)
    x = random_image(3, n)
    f = plan.forward(to_dev(x)).cpu().numpy()
    assert rel(f, grid_forward(x.astype(np.float64), ang, n)) <= 1e-5
    with pytest.raises(ValueError):
        autotune(50, ang, n)                             # not a supported size


def test_batch_mixed_widths_and_tiles_bitwise():
    """Slices with different kernel widths and tile sizes go to separate
    gridding launches of one batch; every slice still equals its per-slice
    call bit for bit, forward and adjoint."""
    note("batch with mixed W and T")
    specs = [(64, 40, 6, None), (64, 33, 4, None), (96, 21, 8, None), (64, 45, 6, {"tile": 8}),
             (128, 60, 6, {"tile": 16, "a2_chunk": 256}), (48, 17, 4, {"f3_chunk": 1024})]
    plans, imgs, sinos = [], [], []
    for k, (n, nv, W, tn) in enumerate(specs):
        plans.append(Plan(n, uniform_angles(nv) + 0.02 * k, n, W=W, tuning=tn))
        imgs.append(to_dev(random_image(60 + k, n)))
        sinos.append(to_dev(random_sinogram(160 + k, nv, n)))
    batch = Batch(plans, n_branches=2)
    outs_f = [torch.empty((p.n_views, p.n_det), device=DEV) for p in plans]
    outs_a = [torch.empty((p.n, p.n), device=DEV) for p in plans]
    for _ in range(2):
        batch.forward(imgs, outs_f)
        batch.adjoint(sinos, outs_a)
        torch.cuda.synchronize()
        for p, x, y, f, a in zip(plans, imgs, sinos, outs_f, outs_a):
            assert torch.equal(f, p.forward(x)) and torch.equal(a, p.adjoint(y))
