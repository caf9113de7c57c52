#!/usr/bin/env python3
"""Throughput of the MI355X Radon NUFFT: forward + adjoint pairs per second.

One step is one forward Radon transform and one adjoint of its result on the
full-size slice: a 2560 x 2560 float32 disk phantom (200 disks, radii 10-300
px, plus N(0, 1e-2^2) noise), 1024 views uniform in [0, pi), 2560 detector
bins, oversampling 2, Kaiser-Bessel width 6. The value is sinogram samples
through one forward+adjoint pair per second (Gsamples/s), inputs resident in
HBM. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 30] [--warmup 200]

Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Radon NUFFT fwd+adj Gsamples/s; solve time to fixed residual, warm vs cold"
N_IMG, N_VIEWS, N_DET, SIGMA, W = 2560, 1024, 2560, 2.0, 6
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_full_slice_2560.json")


def kernel_bytes(n: int, n_views: int, n_det: int):
    """Algorithmic HBM bytes per launch of each kernel (each array touched once).

    The grid is the Hermitian half plane, (n+1) x 2n complex64; T1 is the
    row-transform intermediate, (n+1) x n complex64.
    """
    G = 2 * n
    img = 4 * n * n
    t1 = 8 * (n + 1) * n
    grid = 8 * (n + 1) * G
    sino = 4 * n_views * n_det
    yh = 8 * n_views * (n_det // 2 + 1)
    xr = yh
    return {
        "F1_row_fft": img + t1,
        "F2_col_fft": t1 + grid,
        "F3_interp": grid + xr,
        "F4_ray_ifft": xr + sino,
        "A1_ray_fft": sino + yh,
        "A2_spread": yh + grid,
        "A2_reduce": 0,
        "A3_col_ifft": grid + t1,
        "A4_row_ifft": t1 + img,
    }


# the files that define the path's kernels and their launch shapes
KERNEL_SOURCES = ("fft_lds.hpp", "radon_kernels.hpp", "radon_multi.hpp", "radon_sort.hpp", "radon_fwd.hip",
                  "radon_adj.hip", "radon_api.hip")


def source_hash() -> str:
    """Hash of the kernel sources; counter-derived traffic is reported only
    while the kernels are the ones the counters were taken on."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1009_1380_amd")
    for name in KERNEL_SOURCES + ("../build.py",):
        with open(os.path.join(pkg, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def load_traffic(kernel: str, n_launch_bytes: int):
    """HBM bytes per launch from committed counter runs, if they are current."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_views_sample: int, dev=None):
    """Time the FP64 oracle (forward + adjoint) on a bounded sample: the same
    image and detector, every (1024/n_views_sample)-th view. With `dev`, the
    GPU path runs on the same input and geometry and its relative L2 error
    against the oracle's outputs is returned too (forward on the phantom;
    adjoint on the oracle's forward output rounded to float32)."""
    import numpy as np

    from oracle.grid import _WORKERS, grid_adjoint, grid_forward
    from radon_inputs import config2_phantom, uniform_angles

    x32 = config2_phantom(0, N_IMG)
    x = x32.astype(np.float64)
    ang = uniform_angles(N_VIEWS)[:: N_VIEWS // n_views_sample]
    t0 = time.perf_counter()
    y = grid_forward(x, ang, N_DET, SIGMA, W)
    t1 = time.perf_counter()
    y32 = y.astype(np.float32)
    a = grid_adjoint(y32.astype(np.float64), ang, N_IMG, SIGMA, W)
    t2 = time.perf_counter()
    samples = len(ang) * N_DET
    out = {
        "value": samples / (t2 - t0) / 1e9,
        "unit": "Gsamples/s",
        "cores": int(_WORKERS),
        "kind": "oracle",
        "host_cpu_count": os.cpu_count(),
        "cpu_model": cpu_model(),
        "sample": (f"FP64 O-grid forward+adjoint of the 2560^2 disk phantom on {len(ang)} of the "
                   f"1024 views x 2560 bins ({samples} samples): fwd {t1 - t0:.2f} s, "
                   f"adj {t2 - t1:.2f} s; scipy.fft with {_WORKERS} workers (the host share of one GPU "
                   f"is 16 threads), NumPy footprint sums"),
    }
    err = None
    if dev is not None:
        import torch

        from paper_1009_1380_amd import Plan

        plan = Plan(N_IMG, ang, N_DET, SIGMA, W)
        yg = plan.forward(torch.from_numpy(x32).to(dev)).cpu().numpy().astype(np.float64)
        ag = plan.adjoint(torch.from_numpy(y32).to(dev)).cpu().numpy().astype(np.float64)
        plan.close()
        err = {"fwd": float(np.linalg.norm(yg - y) / np.linalg.norm(y)),
               "adj": float(np.linalg.norm(ag - a) / np.linalg.norm(a)),
               "views": len(ang), "tolerance": 1e-5}
    return out, err


def copy_peak(dev, mib: int = 2048, reps: int = 10):
    """Device-to-device copy of a buffer much larger than the 256 MB last-level
    cache; bytes read + written per second (GB/s)."""
    import torch

    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2 * n * 4 / sec / 1e9


SOLVE_SNR_DB = 30.0     # noise level of the reduced-view data
SOLVE_OPT_TOL = 1e-3    # relative residual tolerance of the solve


def solve_times(dev, repeats: int = 3):
    """Reduced-view reconstruction: 1024^2 disk phantom, 128 views x 1024
    bins, ring gains N(1, 0.02^2), 30 dB noise. Basis-pursuit denoising with
    the ring filter, sigma at the noise level implied by the SNR
    (10^(-SNR/20) ||F b||), stopped when | ||r|| - sigma | <= 1e-3 ||r||.
    Cold start (x0 = 0) against a warm start from the filtered adjoint (its
    time included). Median wall time of `repeats` solves each."""
    import torch

    from paper_1009_1380_amd import Plan
    from radon_inputs import config4_problem

    _, b, ang = config4_problem(0)
    plan = Plan(1024, ang, 1024)
    bd = torch.from_numpy(b).to(dev)
    fbn = float(torch.linalg.norm(plan.ring_filter(bd).double()))
    sigma = 10.0 ** (-SOLVE_SNR_DB / 20.0) * fbn
    out = {"workload": "reduced-view reconstruction: 1024^2 disk phantom (60 disks, radii 8-128), "
                       "128 views x 1024 bins, exact line integrals, ring gains N(1,0.02^2), 30 dB noise; "
                       "min ||x||_1 s.t. ||F(Ax-b)|| <= sigma, sigma = 10^(-1.5) ||Fb||, "
                       "stop at relative residual error 1e-3",
           "sigma": sigma, "opt_tol": SOLVE_OPT_TOL}
    for name in ("cold", "warm_fbp"):
        runs = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x0 = plan.fbp(bd) if name == "warm_fbp" else None
            _, st = plan.solve_bpdn(bd, sigma, x0=x0, opt_tol=SOLVE_OPT_TOL, max_iter=5000)
            torch.cuda.synchronize()
            runs.append((time.perf_counter() - t0, st))
        runs.sort(key=lambda r: r[0])
        wall, st = runs[len(runs) // 2]
        out[name] = {"seconds": round(wall, 4), "iterations": st["iterations"],
                     "n_forward": st["n_forward"], "n_adjoint": st["n_adjoint"],
                     "rnorm_over_sigma": round(st["rnorm"] / sigma, 6), "x_l1": st["x_l1"],
                     "status": {0: "max_iter", 1: "bp", 2: "root"}.get(st["status"], st["status"])}
    out["warm_over_cold_time"] = round(out["warm_fbp"]["seconds"] / out["cold"]["seconds"], 3)
    return out


BATCH_SIZES = (512, 1024, 1536, 2048, 2560)
BATCH_VIEWS = (90, 180, 360, 720, 1024)


def batch_times(dev, n_slices: int = 64, repeats: int = 5, seed: int = 0, tune: bool = True):
    """Uneven slices: n_slices slices, side uniform in BATCH_SIZES, view count
    uniform in BATCH_VIEWS (angles uniform in [0, pi)), detector bins = side.
    One step = forward + adjoint of every slice. Three ways: per-slice calls
    back to back on one stream; the batch's two HIP graphs (forward, adjoint)
    with the default decomposition; the same with every distinct shape's
    decomposition chosen by the autotuner."""
    import numpy as np
    import torch

    from paper_1009_1380_amd import Batch, Plan, autotune
    from radon_inputs import random_image, uniform_angles

    rng = np.random.default_rng(seed)
    shapes = [(int(rng.choice(BATCH_SIZES)), int(rng.choice(BATCH_VIEWS))) for _ in range(n_slices)]
    imgs = [torch.from_numpy(random_image(seed + k, n)).to(dev) for k, (n, _) in enumerate(shapes)]
    sinos = [torch.empty((v, n), device=dev) for n, v in shapes]
    backs = [torch.empty((n, n), device=dev) for n, _ in shapes]
    samples = sum(n * v for n, v in shapes)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(repeats):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / repeats

    def run_modes(plans):
        def per_slice():
            for p, x, y, z in zip(plans, imgs, sinos, backs):
                p.forward(x, out=y, stream=stream)
                p.adjoint(y, out=z, stream=stream)
        batch = Batch(plans, n_branches=4)

        def graphs():
            batch.forward(imgs, sinos, stream=stream)
            batch.adjoint(sinos, backs, stream=stream)
        return timed(per_slice), timed(graphs)

    plans = [Plan(n, uniform_angles(v), n) for n, v in shapes]
    ms_slice, ms_graph = run_modes(plans)
    del plans

    def gs(ms):
        return round(samples / (ms * 1e-3) / 1e9, 3)
    out = {
        "workload": f"{n_slices} uneven slices: side uniform in {list(BATCH_SIZES)}, views uniform in "
                    f"{list(BATCH_VIEWS)}, detector bins = side; one step = forward + adjoint of every slice",
        "samples_per_step": samples,
        "per_slice_calls": {"ms_per_step": round(ms_slice, 3), "Gsamples_per_s": gs(ms_slice)},
        "graph_batch": {"ms_per_step": round(ms_graph, 3), "Gsamples_per_s": gs(ms_graph)},
    }
    if not tune:
        return out
    t0 = time.perf_counter()
    tuned = {}
    for n, v in sorted(set(shapes)):
        tuned[(n, v)] = autotune(n, uniform_angles(v), n, repeats=3, stream=stream)
    t_tune = time.perf_counter() - t0
    plans = [Plan(n, uniform_angles(v), n, tuning=tuned[(n, v)][0]) for n, v in shapes]
    ms_slice_t, ms_graph_t = run_modes(plans)
    del plans
    changed = sum(1 for k, (best, _, _) in tuned.items() if best != {"tile": 32, "a2_chunk": 512, "f3_chunk": 2048})

    out.update({
        "per_slice_calls_autotuned": {"ms_per_step": round(ms_slice_t, 3), "Gsamples_per_s": gs(ms_slice_t)},
        "graph_batch_autotuned": {"ms_per_step": round(ms_graph_t, 3), "Gsamples_per_s": gs(ms_graph_t)},
        "autotune": {"seconds": round(t_tune, 2), "shapes": len(tuned), "shapes_off_default": changed},
    })
    return out


def warmstart_times(pairs: int = 1024, epochs: int = 6, n_eval: int = 40):
    """Learned warm start on the 512^2, 90-view workload, reduced so the bench
    stays short (the full 2000-pair run is paper_1009_1380_amd.warmstart):
    pairs generated by the method, training, cold vs warm on held-out seeds.
    About 26 s on one MI355X; with 256 pairs, 4 epochs and 20 slices (8 s) the
    median warm/cold ratio moved between 0.81 and 0.96 from run to run."""
    import torch

    from paper_1009_1380_amd import WarmStartNet
    from paper_1009_1380_amd.warmstart import Problem, evaluate, generate_pairs, summarize, train

    prob = Problem(512, 90)
    t0 = time.perf_counter()
    xs, ts = generate_pairs(prob, range(pairs))
    net = WarmStartNet(8, 512, 512, seed=0)
    hist = train(net, xs, ts, epochs, 1e-3)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    net1 = WarmStartNet(1, 512, 512, seed=0)
    net1.set_params(net.get_params())
    rows = evaluate(prob, net1, range(10_000_000, 10_000_000 + n_eval))
    out = {"workload": f"512^2 random-disk slices, 90 views x 512 bins, 30 dB noise + ring gains; {pairs} "
                       f"method-generated training pairs, {epochs} epochs, {n_eval} held-out slices; basis pursuit to "
                       f"relative residual error 1e-3; warm time includes filtered adjoint + network",
           "prepare_seconds": round(t_prep, 1), "final_loss": hist[-1]}
    out.update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in summarize(rows).items()})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    # the clocks take a few tens of milliseconds of load to settle: after 5
    # warm-up pairs the first timed loop runs about 10% slow, after 100 or more
    # it matches the per-pair median of later loops
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-views", type=int, default=1024, help="views in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the reduced-view solve timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-slice batch timing")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the learned warm-start run")
    ap.add_argument("--no-autotune", action="store_true", help="batch timing without the autotuned half")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(slices are independent: each GPU would take its own slices, with no exchange)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: launched with WORLD_SIZE > 1; only one GPU is used", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1009_1380_amd import Plan
    from radon_inputs import config2_phantom, uniform_angles

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print("bench: building inputs and plan", file=sys.stderr, flush=True)
    x = torch.from_numpy(config2_phantom(0, N_IMG)).to(dev)
    ang = uniform_angles(N_VIEWS)
    t_plan0 = time.perf_counter()
    plan = Plan(N_IMG, ang, N_DET, SIGMA, W)
    t_plan = time.perf_counter() - t_plan0
    sino = torch.empty((N_VIEWS, N_DET), dtype=torch.float32, device=dev)
    back = torch.empty((N_IMG, N_IMG), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.forward(x, out=sino, stream=stream)
        plan.adjoint(sino, out=back, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps between events on the stream the kernels run on
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps

    # forward and adjoint separately
    def time_loop(fn, k):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    t_fwd = time_loop(lambda: plan.forward(x, out=sino, stream=stream), args.steps)
    t_adj = time_loop(lambda: plan.adjoint(sino, out=back, stream=stream), args.steps)

    # per-pair spread: at least 50 back-to-back pairs with an event between
    # consecutive pairs (warm cache, as in the solver loop)
    n_pairs = max(50, args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_pairs + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(n_pairs):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per_pair = [evs[i].elapsed_time(evs[i + 1]) for i in range(n_pairs)]
    pair_stats = {"pairs": n_pairs, "median_ms": round(float(np.median(per_pair)), 4),
                  "min_ms": round(float(np.min(per_pair)), 4), "max_ms": round(float(np.max(per_pair)), 4)}

    # cold last-level cache: a 1 GiB buffer is written before every pair (the
    # 256 MB cache then holds none of the pair's arrays); only the pair is timed
    flush = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(args.steps):
        flush.fill_(1.0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        torch.cuda.synchronize()
        cold.append(a.elapsed_time(b))
    del flush
    ms_cold = float(np.median(cold))
    copy_gbs = copy_peak(dev)

    # per-kernel durations: same steps with each launch bracketed by events
    plan.set_profiling(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.set_profiling(False)
    kbytes = kernel_bytes(N_IMG, N_VIEWS, N_DET)
    stages = {}
    for name, (ms, cnt) in st.items():
        if cnt:
            avg_us = 1e3 * ms / cnt
            gbs = kbytes[name] / (avg_us * 1e-6) / 1e9 if kbytes[name] else None
            stages[name] = {"avg_us": round(avg_us, 2), "launches": cnt,
                            "alg_bytes": kbytes[name], "alg_GBps": round(gbs, 1) if gbs else None}
    dominant = max(stages, key=lambda k: stages[k]["avg_us"] * stages[k]["launches"])
    d = stages[dominant]
    achieved = d["alg_bytes"] / (d["avg_us"] * 1e-6) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": dominant,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": load_traffic(dominant, d["alg_bytes"]),
        "copy_peak": round(copy_gbs, 1),
        "frac_of_copy_peak": round(achieved / copy_gbs, 4),
    }
    samples = N_VIEWS * N_DET
    value = samples / (ms_step * 1e-3) / 1e9
    pair_bytes = sum(kbytes[k] for k in kbytes)
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "full-size slice: 2560^2 disk phantom (200 disks, radii 10-300, +N(0,1e-2^2)), "
                        "1024 views in [0,pi) x 2560 bins, sigma=2, KB W=6; one step = forward + adjoint",
            "n": N_IMG, "n_views": N_VIEWS, "n_det": N_DET, "sigma": SIGMA, "W": W,
            "parallelism": "single GPU",
        },
        "t_fwd_ms": round(t_fwd, 4),
        "t_adj_ms": round(t_adj, 4),
        "wall_s_timed": round(wall, 4),
        "plan_s": round(t_plan, 3),
        "ms_per_pair_warm": pair_stats,
        "ms_per_step_cold_cache": round(ms_cold, 4),
        "copy_peak_GBps": round(copy_gbs, 1),
        # the bytes this design moves per pair (Hermitian half plane, each
        # array once per kernel that touches it) over the pair's time
        "pair_alg_bytes": pair_bytes,
        "pair_alg_GBps": round(pair_bytes / (ms_step * 1e-3) / 1e9, 1),
        "pair_frac_hbm_peak": round(pair_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "pair_frac_copy_peak": round(pair_bytes / (ms_step * 1e-3) / 1e9 / copy_gbs, 4),
        "pair_frac_hbm_peak_cold_cache": round(pair_bytes / (ms_cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        # the byte model of the full complex G x G grid (200 n^2 + 8 M per
        # pair), which this design does not move; kept for comparison only
        "full_grid_model": {
            "bytes": 200 * N_IMG * N_IMG + 8 * N_VIEWS * N_DET,
            "frac_hbm_peak": round((200 * N_IMG * N_IMG + 8 * N_VIEWS * N_DET) / (ms_step * 1e-3) / 8.0e12, 4),
        },
        "stages": stages,
        "roofline": roofline,
    }
    if args.calib_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings give
        # the scale from counter units to HBM bytes
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    def section(key, what, fn):
        # a secondary measurement that fails is reported in the line (and on
        # stderr) instead of losing the line
        print(f"bench: {what}", file=sys.stderr, flush=True)
        try:
            return fn()
        except Exception as e:  # noqa: BLE001
            print(f"bench: {key} failed: {e!r}", file=sys.stderr, flush=True)
            return {"error": repr(e)}

    if not args.no_solve:
        line["solve"] = section("solve", "timing the reduced-view solves", lambda: solve_times(dev))
    if not args.no_batch:
        line["batch"] = section("batch", "timing the uneven-slice batch",
                                lambda: batch_times(dev, tune=not args.no_autotune))
    if not args.no_warmstart:
        line["warmstart"] = section("warmstart", "learned warm start (reduced)", warmstart_times)
    if not args.no_cpu_baseline:
        res = section("cpu_baseline", "timing the CPU oracle sample", lambda: cpu_baseline(args.cpu_views, dev))
        if isinstance(res, tuple):
            line["cpu_baseline"], line["rel_l2_vs_ogrid"] = res
        else:
            line["cpu_baseline"], line["rel_l2_vs_ogrid"] = res, None
    else:
        line["cpu_baseline"] = None
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
