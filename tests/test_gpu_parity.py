"""GPU parity of the HIP path against the CPU oracle (run on an MI355X).

Bars (float32 path vs float64 oracle):
  * relative L2 <= 1e-5 against O-grid (the FP64 gridding oracle),
  * relative L2 <= 1e-4 against O-exact (the exact discrete transform),
  * bit-exact sample sort (perm, bin offsets) against the oracle's keys,
  * bitwise identical results on repeated runs (no atomics).
Every call goes through the C ABI via the ctypes binding.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.binning import bin_offsets, refined_keys, sample_keys, stable_sort  # noqa: E402
from oracle.exact import radon_exact, radon_exact_adjoint  # noqa: E402
from oracle.geometry import polar_uv, ray_q  # noqa: E402
from oracle.grid import (GridParams, grid_adjoint, grid_fft2, grid_forward,  # noqa: E402
                         grid_spread, ray_spectrum)
from radon_inputs import (config1_phantom, gaussian_blob, random_image,  # noqa: E402
                          random_sinogram, uniform_angles)

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1009_1380_amd import Plan, fft_test  # noqa: E402

DEV = "cuda:0"
TOL_GRID = 1e-5
TOL_EXACT = 1e-4


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def special_angles(nv, seed):
    ang = np.random.default_rng(seed).uniform(0, np.pi, nv)
    ang[0] = 0.0
    if nv > 1:
        ang[1] = np.pi / 2
    return ang


# ------------------------------------------------------------------ FFT engine

@pytest.mark.parametrize("length", [8, 12, 16, 20, 24, 40, 48, 64, 96, 128, 160, 256, 320,
                                    384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072, 4096])
def test_fft_engine_vs_numpy(length):
    """G11: each supported length, forward and inverse, vs numpy FP64."""
    note(f"fft length {length}")
    rng = np.random.default_rng(length)
    x = (rng.standard_normal((5, length)) + 1j * rng.standard_normal((5, length))).astype(np.complex64)
    xd = torch.from_numpy(x).to(DEV)
    f = fft_test(xd).cpu().numpy()
    b = fft_test(xd, inverse=True).cpu().numpy()
    ref_f = np.fft.fft(x.astype(np.complex128), axis=1)
    ref_b = np.fft.ifft(x.astype(np.complex128), axis=1) * length
    tol = 2e-6 * max(1.0, np.log2(length) / 4)
    assert rel(f, ref_f) < tol
    assert rel(b, ref_b) < tol


# ------------------------------------------------------------------ sort

def extended_keys(angles, n, n_det, W, T, refined=True):
    """Oracle keys of the plan's samples: the n_views*n_det polar samples, then
    one mirrored Nyquist sample (q = +N/2) per view."""
    G = 2 * n
    fn = refined_keys if refined else sample_keys
    u, v = polar_uv(angles, n_det, G)
    um, vm = polar_uv(angles, n_det, G, q=np.array([n_det // 2]))
    return np.concatenate([fn(u, v, G, W, T).ravel(), fn(um, vm, G, W, T).ravel()])


@pytest.mark.parametrize("n,n_det,nv", [(16, 16, 12), (32, 40, 33), (128, 128, 180), (64, 96, 7),
                                        (2560, 2560, 1024)])
def test_sort_bit_exact(n, n_det, nv):
    """G10: perm and class offsets equal the oracle's stable argsort / counts
    of the refined keys; the tile bins hold exactly the oracle's tile keys."""
    note(f"sort n={n} n_det={n_det} nv={nv}")
    ang = special_angles(nv, 3) if nv not in (180, 1024) else uniform_angles(nv)
    plan = Plan(n, ang, n_det)
    info = plan.info()
    perm, offs = plan.sort_indices()
    T = info["T"]
    keys = extended_keys(ang, n, n_det, plan.W, T)
    assert perm.size == keys.size == info["n_samples"]
    assert np.array_equal(perm, stable_sort(keys).astype(np.int32))
    assert np.array_equal(offs, bin_offsets(keys, 4 * info["n_bins"]).astype(np.int32))
    # tile bins (every 4th offset) hold exactly the samples of each tile key
    tkeys = extended_keys(ang, n, n_det, plan.W, T, refined=False)
    assert np.array_equal(offs[::4], bin_offsets(tkeys, info["n_bins"]).astype(np.int32))
    # within a class run the real samples keep increasing id
    M = nv * n_det
    assert np.all(np.diff(keys[perm]) >= 0)
    same = np.diff(keys[perm]) == 0
    assert np.all(np.diff(perm)[same] > 0)
    assert perm[perm >= M].size == nv


# ------------------------------------------------------------------ kernel-level grids

@pytest.mark.parametrize("n", [8, 32, 128])
def test_forward_grid_vs_oracle(n):
    """F1+F2: the half-plane oversampled FFT equals the oracle's FFT2."""
    note(f"forward grid n={n}")
    x = random_image(21, n)
    plan = Plan(n, uniform_angles(4), n)
    g = plan.debug_forward_grid(to_dev(x)).cpu().numpy()
    gp = GridParams(n, n)
    ref = grid_fft2(x.astype(np.float64), gp)[:, : gp.G // 2 + 1].T
    assert rel(g, ref) < TOL_GRID


@pytest.mark.parametrize("n,n_det,nv", [(8, 8, 6), (32, 40, 13), (128, 128, 180)])
def test_adjoint_grid_vs_oracle(n, n_det, nv):
    """A1+A2: the spread grid equals the Hermitian part of the oracle's spread."""
    note(f"adjoint grid n={n} n_det={n_det} nv={nv}")
    ang = special_angles(nv, 4) if nv != 180 else uniform_angles(nv)
    y = random_sinogram(22, nv, n_det)
    plan = Plan(n, ang, n_det)
    g = plan.debug_adjoint_grid(to_dev(y)).cpu().numpy()
    gp = GridParams(n, n_det)
    G = gp.G
    u, v = polar_uv(ang, n_det, G)
    H = grid_spread(ray_spectrum(y.astype(np.float64), n_det), u, v, gp)
    idx = (-np.arange(G)) % G
    Hh = 0.5 * (H + np.conj(H[np.ix_(idx, idx)]))
    ref = Hh[:, : G // 2 + 1].T
    assert rel(g, ref) < TOL_GRID


# ------------------------------------------------------------------ end to end

SMALL = [(8, 8, 6), (8, 16, 5), (16, 16, 9), (16, 24, 1), (16, 40, 11), (32, 32, 12),
         (32, 48, 17), (64, 64, 30), (64, 80, 31), (128, 96, 20)]


@pytest.mark.parametrize("n,n_det,nv", SMALL)
def test_forward_adjoint_small_vs_oracles(n, n_det, nv):
    note(f"small n={n} n_det={n_det} nv={nv}")
    ang = special_angles(nv, n + nv)
    x = random_image(n + 1, n)
    y = random_sinogram(n + 2, nv, n_det)
    plan = Plan(n, ang, n_det)
    yg = plan.forward(to_dev(x)).cpu().numpy()
    ag = plan.adjoint(to_dev(y)).cpu().numpy()
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    assert rel(yg, grid_forward(x64, ang, n_det)) < TOL_GRID
    assert rel(ag, grid_adjoint(y64, ang, n)) < TOL_GRID
    if n <= 32:
        assert rel(yg, radon_exact(x64, ang, n_det)) < TOL_EXACT
        assert rel(ag, radon_exact_adjoint(y64, ang, n)) < TOL_EXACT


@pytest.mark.parametrize("seed", range(10))
def test_config1_forward_adjoint(seed):
    """Parity workload: 128^2 disk phantom, 180 views x 128 bins."""
    note(f"config1 seed={seed}")
    x, _ = config1_phantom(seed)
    ang = uniform_angles(180)
    plan = Plan(128, ang, 128)
    yd = plan.forward(to_dev(x))
    ad = plan.adjoint(yd)
    y_ref = grid_forward(x.astype(np.float64), ang, 128)
    assert rel(yd.cpu().numpy(), y_ref) < TOL_GRID
    a_ref = grid_adjoint(yd.cpu().numpy().astype(np.float64), ang, 128)
    assert rel(ad.cpu().numpy(), a_ref) < TOL_GRID


def test_config1_vs_exact():
    """Config 1 against O-exact, forward and adjoint (seed 0)."""
    note("config1 vs exact")
    x, _ = config1_phantom(0)
    ang = uniform_angles(180)
    plan = Plan(128, ang, 128)
    yd = plan.forward(to_dev(x)).cpu().numpy()
    assert rel(yd, radon_exact(x.astype(np.float64), ang, 128)) < TOL_EXACT
    y = random_sinogram(5, 180, 128)
    ad = plan.adjoint(to_dev(y)).cpu().numpy()
    assert rel(ad, radon_exact_adjoint(y.astype(np.float64), ang, 128)) < TOL_EXACT


def test_gaussian_blob_closed_form():
    """G5 on the GPU: a band-limited blob projects to a Gaussian profile."""
    note("gaussian blob")
    n, nv = 256, 64
    cx, cy, sg = 23.3, -41.6, 3.0
    x = gaussian_blob(n, cx, cy, sg).astype(np.float32)
    ang = uniform_angles(nv)
    y = Plan(n, ang, n).forward(to_dev(x)).cpu().numpy()
    s = np.arange(n) - n / 2
    ref = np.stack([np.sqrt(2 * np.pi) * sg * np.exp(-(s - (cx * np.cos(t) + cy * np.sin(t))) ** 2 / (2 * sg * sg))
                    for t in ang])
    assert rel(y, ref) < TOL_EXACT


def test_adjoint_identity_fp32():
    """G7: <A x, y> = <x, A^T y> for the GPU operators."""
    note("adjoint identity")
    n, n_det, nv = 128, 128, 90
    ang = uniform_angles(nv)
    plan = Plan(n, ang, n_det)
    x = random_image(31, n)
    y = random_sinogram(32, nv, n_det)
    Ax = plan.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    Aty = plan.adjoint(to_dev(y)).cpu().numpy().astype(np.float64)
    lhs, rhs = np.sum(Ax * y), np.sum(x.astype(np.float64) * Aty)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_determinism_bitwise():
    """G13: repeated runs give bitwise identical outputs."""
    note("determinism")
    n, nv = 128, 180
    plan = Plan(n, uniform_angles(nv), n)
    x = to_dev(config1_phantom(3)[0])
    y1 = plan.forward(x).clone()
    a1 = plan.adjoint(y1).clone()
    for _ in range(3):
        assert torch.equal(plan.forward(x), y1)
        assert torch.equal(plan.adjoint(y1), a1)


def test_batched_equals_loop():
    note("batched")
    n, nv, B = 64, 30, 3
    plan = Plan(n, uniform_angles(nv), n)
    xs = torch.stack([to_dev(random_image(40 + b, n)) for b in range(B)])
    ys = plan.forward_batched(xs)
    for b in range(B):
        assert torch.equal(ys[b], plan.forward(xs[b].contiguous()))
    a = plan.adjoint_batched(ys)
    for b in range(B):
        assert torch.equal(a[b], plan.adjoint(ys[b].contiguous()))
    # an empty batch is a no-op that launches nothing
    assert plan.forward_batched(xs[:0]).shape == (0, nv, n)
    assert plan.adjoint_batched(ys[:0]).shape == (0, n, n)


def test_binding_rejects_bad_tensors():
    plan = Plan(16, uniform_angles(4), 16)
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(16, 16, device=DEV, dtype=torch.float64))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(16, 17, device=DEV))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(16, 16))
    with pytest.raises(ValueError):
        plan.adjoint(torch.zeros(16, 4, device=DEV).t())


def test_stream_and_profiling():
    """Work is enqueued on the given stream; stage times are reported."""
    n, nv = 64, 32
    plan = Plan(n, uniform_angles(nv), n)
    x = to_dev(random_image(50, n))
    ref = plan.forward(x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    plan.set_profiling(True)
    with torch.cuda.stream(s):
        y = plan.forward(x)
        a = plan.adjoint(y)
    s.synchronize()
    assert torch.equal(y, ref)
    times = plan.stage_times()
    assert times["F1_row_fft"][1] == 1 and times["F3_interp"][1] == 1 and times["A2_spread"][1] == 1
    assert all(ms >= 0 for ms, _ in times.values())
    plan.set_profiling(False)
    assert torch.isfinite(a).all()


# ------------------------------------------------------------------ full size

def test_full_size_slice_vs_oracle():
    """Full-size slice (the benchmark's launch configuration): 2560^2 disk
    phantom with noise, 1024 views x 2560 bins; forward and adjoint of the
    whole arrays against O-grid (FP64)."""
    from radon_inputs import config2_phantom
    note("full size: phantom + plan")
    n, nv = 2560, 1024
    x = config2_phantom(0, n)
    ang = uniform_angles(nv)
    plan = Plan(n, ang, n)
    yd = plan.forward(to_dev(x))
    ad = plan.adjoint(yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    a = ad.cpu().numpy()
    note("full size: oracle forward")
    y_ref = grid_forward(x.astype(np.float64), ang, n)
    ey = rel(y, y_ref)
    note(f"full size forward rel L2 {ey:.3e}")
    assert ey < TOL_GRID
    note("full size: oracle adjoint")
    a_ref = grid_adjoint(y.astype(np.float64), ang, n)
    ea = rel(a, a_ref)
    note(f"full size adjoint rel L2 {ea:.3e}")
    assert ea < TOL_GRID


@pytest.mark.parametrize("n", [1536, 2048])
def test_large_sizes_vs_oracle(n):
    """The row passes' workgroup shapes at the other large sizes (2048: eight
    rows per workgroup, one round; 1536: four rows): forward and adjoint of an
    n^2 disk phantom at 90 views x n bins against O-grid (FP64)."""
    from radon_inputs import config2_phantom
    note(f"large size n={n}: phantom + plan")
    nv = 90
    x = config2_phantom(3, n)
    ang = uniform_angles(nv)
    plan = Plan(n, ang, n)
    y = plan.forward(to_dev(x)).cpu().numpy()
    a = plan.adjoint(to_dev(y)).cpu().numpy()
    note(f"large size n={n}: oracle")
    ey = rel(y, grid_forward(x.astype(np.float64), ang, n))
    ea = rel(a, grid_adjoint(y.astype(np.float64), ang, n))
    note(f"large size n={n}: forward {ey:.3e}, adjoint {ea:.3e}")
    assert ey < TOL_GRID and ea < TOL_GRID


def test_full_size_gaussian_closed_form():
    """G5 at full size: no O(n^2 M) work, closed-form projections."""
    note("full size gaussian")
    n, nv = 2560, 64
    cx, cy, sg = 311.7, -402.2, 4.0
    x = gaussian_blob(n, cx, cy, sg).astype(np.float32)
    ang = uniform_angles(nv)
    y = Plan(n, ang, n).forward(to_dev(x)).cpu().numpy()
    s = np.arange(n) - n / 2
    ref = np.stack([np.sqrt(2 * np.pi) * sg * np.exp(-(s - (cx * np.cos(t) + cy * np.sin(t))) ** 2 / (2 * sg * sg))
                    for t in ang])
    assert rel(y, ref) < TOL_EXACT


def test_full_size_adjoint_identity_and_determinism():
    note("full size adjoint identity")
    n, nv = 2560, 1024
    plan = Plan(n, uniform_angles(nv), n)
    x = to_dev(random_image(61, n))
    y = to_dev(random_sinogram(62, nv, n))
    Ax = plan.forward(x)
    Aty = plan.adjoint(y)
    Ax2 = plan.forward(x)
    Aty2 = plan.adjoint(y)
    assert torch.equal(Ax, Ax2) and torch.equal(Aty, Aty2)
    lhs = float(torch.sum(Ax.double() * y.double()))
    rhs = float(torch.sum(x.double() * Aty.double()))
    assert abs(lhs - rhs) <= 1e-5 * float(torch.linalg.norm(Ax.double())) * float(torch.linalg.norm(y.double()))


# ------------------------------------------------------------------ filtered adjoint

@pytest.mark.parametrize("n,n_det,nv", [(16, 16, 9), (64, 80, 31), (128, 128, 180)])
def test_fbp_vs_oracle(n, n_det, nv):
    from oracle.grid import grid_fbp
    note(f"fbp n={n} n_det={n_det} nv={nv}")
    ang = special_angles(nv, 7) if nv != 180 else uniform_angles(nv)
    y = random_sinogram(71, nv, n_det)
    plan = Plan(n, ang, n_det)
    r = plan.fbp(to_dev(y)).cpu().numpy()
    assert rel(r, grid_fbp(y.astype(np.float64), ang, n)) < TOL_GRID


def test_fbp_reconstructs_gaussian():
    note("fbp gaussian")
    n = 256
    x = (gaussian_blob(n, 7.3, -5.1, 4.0) + 0.5 * gaussian_blob(n, -12.0, 9.0, 3.0)).astype(np.float32)
    ang = uniform_angles(2 * n)
    plan = Plan(n, ang, n)
    r = plan.fbp(plan.forward(to_dev(x))).cpu().numpy()
    xs = np.arange(n) - n / 2
    inside = np.sqrt(xs[None, :] ** 2 + xs[:, None] ** 2) < n / 2 - 2
    assert rel(r[inside], x[inside]) < 3e-4


# ------------------------------------------------------------------ kernel widths and the largest size

@pytest.mark.parametrize("W", [4, 8])
@pytest.mark.parametrize("n,n_det,nv", [(16, 16, 9), (64, 80, 31), (128, 128, 45)])
def test_other_kernel_widths_vs_oracle(W, n, n_det, nv):
    """W = 4 and W = 8 (the plan's other widths) against the oracle with the same W."""
    note(f"W={W} n={n} n_det={n_det} nv={nv}")
    ang = special_angles(nv, 3 * n + W)
    x = random_image(n + W, n)
    y = random_sinogram(n + W + 1, nv, n_det)
    plan = Plan(n, ang, n_det, W=W)
    yg = plan.forward(to_dev(x)).cpu().numpy()
    ag = plan.adjoint(to_dev(y)).cpu().numpy()
    assert rel(yg, grid_forward(x.astype(np.float64), ang, n_det, W=W)) < TOL_GRID
    assert rel(ag, grid_adjoint(y.astype(np.float64), ang, n, W=W)) < TOL_GRID


def test_largest_supported_size_vs_oracle():
    """n = n_det = 4096 (the largest FFT length; G = 8192) on a few views."""
    note("n=4096 nv=6")
    n, nv = 4096, 6
    ang = special_angles(nv, 11)
    x = random_image(4096, n)
    y = random_sinogram(4097, nv, n)
    plan = Plan(n, ang, n)
    yg = plan.forward(to_dev(x)).cpu().numpy()
    ag = plan.adjoint(to_dev(y)).cpu().numpy()
    assert rel(yg, grid_forward(x.astype(np.float64), ang, n)) < TOL_GRID
    assert rel(ag, grid_adjoint(y.astype(np.float64), ang, n)) < TOL_GRID


@pytest.mark.parametrize("kind", ["beyond_pi", "negative", "duplicated", "unsorted_wide"])
def test_unusual_angle_sets_vs_oracle(kind):
    """The header accepts any float64 angles in any order: angles in
    [pi, 2 pi), negative angles, repeated angles and an unsorted set spanning
    several turns all match O-grid (and O-exact) through the ABI."""
    note(f"angles {kind}")
    n, n_det, nv = 32, 40, 17
    rng = np.random.default_rng(7)
    if kind == "beyond_pi":
        ang = np.pi + rng.uniform(0, np.pi, nv)
        ang[0] = np.pi
        ang[1] = 1.5 * np.pi
    elif kind == "negative":
        ang = -rng.uniform(0, np.pi, nv)
        ang[0] = -np.pi / 2
    elif kind == "duplicated":
        base = rng.uniform(0, np.pi, 6)
        ang = np.concatenate([base, base, base[:5]])
        ang[0] = ang[6] = 0.0
    else:
        ang = rng.uniform(-3 * np.pi, 3 * np.pi, nv)
    x = random_image(91, n)
    y = random_sinogram(92, nv, n_det)
    plan = Plan(n, ang, n_det)
    yg = plan.forward(to_dev(x)).cpu().numpy()
    ag = plan.adjoint(to_dev(y)).cpu().numpy()
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    assert rel(yg, grid_forward(x64, ang, n_det)) < TOL_GRID
    assert rel(ag, grid_adjoint(y64, ang, n)) < TOL_GRID
    assert rel(yg, radon_exact(x64, ang, n_det)) < TOL_EXACT
    assert rel(ag, radon_exact_adjoint(y64, ang, n)) < TOL_EXACT
    if kind == "duplicated":
        # repeated views give identical rows
        assert np.array_equal(yg[0], yg[6]) and np.array_equal(yg[1], yg[7])


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_adjoint_propagates_nonfinite_input(bad):
    """A non-finite sinogram value reaches the adjoint image as non-finite
    values: the spreading's fixed-point sums do not turn it into finite
    numbers (which would hide a diverging solve)."""
    note(f"adjoint with a {bad} in the sinogram")
    n, nv = 128, 180
    plan = Plan(n, uniform_angles(nv), n)
    y = random_sinogram(93, nv, n)
    y[37, 61] = bad
    a = plan.adjoint(to_dev(y)).cpu().numpy()
    assert not np.isfinite(a).all()
    # the plan is unharmed: a finite sinogram afterwards gives the usual result
    y[37, 61] = 0.0
    a2 = plan.adjoint(to_dev(y)).cpu().numpy()
    assert rel(a2, grid_adjoint(y.astype(np.float64), uniform_angles(nv), n)) < TOL_GRID


def test_split_strips_repeat_bitwise():
    """Split strips (the dense centre) are summed by their last item in slot
    order: many repeated adjoints, interleaved with other plans' work, give
    the same bits."""
    note("split-strip sums, repeated")
    n, nv = 256, 360
    plan = Plan(n, uniform_angles(nv), n)
    other = Plan(64, uniform_angles(30), 64)
    assert plan.info()["n_slots"] > 0
    y = to_dev(random_sinogram(94, nv, n))
    y2 = to_dev(random_sinogram(95, 30, 64))
    a0 = plan.adjoint(y).clone()
    for _ in range(8):
        other.adjoint(y2)
        assert torch.equal(plan.adjoint(y), a0)
    assert rel(a0.cpu().numpy(), grid_adjoint(y.cpu().numpy().astype(np.float64), uniform_angles(nv), n)) < TOL_GRID


def test_adjoint_grid_high_dynamic_range():
    """The spreading's fixed-point scale is chosen per work item, from that
    item's own largest contribution. Ten views (in pairs, so no ray transform
    mixes a large and a small ray) are scaled by 1e6; grid regions that only
    the other views reach must still match the oracle to float32 accuracy
    relative to their own magnitude (a scale shared by all items would round
    them to about 2^-22 of the large views, i.e. errors of order 1e-1 there)."""
    note("adjoint grid, high dynamic range")
    n, n_det, nv = 128, 128, 180
    ang = uniform_angles(nv)
    y = random_sinogram(96, nv, n_det).astype(np.float64)
    y[:10] *= 1e6
    y32 = y.astype(np.float32)
    plan = Plan(n, ang, n_det)
    g = plan.debug_adjoint_grid(to_dev(y32)).cpu().numpy()
    gp = GridParams(n, n_det)
    G = gp.G
    u, v = polar_uv(ang, n_det, G)
    H = grid_spread(ray_spectrum(y32.astype(np.float64), n_det), u, v, gp)
    idx = (-np.arange(G)) % G
    ref = (0.5 * (H + np.conj(H[np.ix_(idx, idx)])))[:, : G // 2 + 1].T     # [mx][my]
    # the large views (angles below 9 degrees) lie within |v| <= 0.16 |u| + 3 of the u axis;
    # rows |v| >= G/4 are two tiles away from every item those views reach
    my = (np.arange(G) + G // 2) % G - G // 2
    far = np.abs(my) >= G // 4
    assert rel(g, ref) < TOL_GRID
    err_far = np.linalg.norm(g[:, far] - ref[:, far]) / np.linalg.norm(ref[:, far])
    note(f"far-region relative error {err_far:.2e}")
    assert err_far < TOL_GRID
