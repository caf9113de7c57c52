"""bench.py's host-side parts, without a GPU: the byte model of one pair and
the refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pair_bytes_at_the_full_size():
    """Each array touched once: image 26.2 MB, T1 52.5 MB, half-plane grid
    104.9 MB, ray spectra and sinogram 10.5 MB each; 744.8 MB per pair."""
    kb = bench.kernel_bytes(2560, 1024, 2560)
    n, G = 2560, 5120
    img, t1, grid = 4 * n * n, 8 * (n + 1) * n, 8 * (n + 1) * G
    spec, sino = 8 * 1024 * (2560 // 2 + 1), 4 * 1024 * 2560
    assert kb["F1_row_fft"] == kb["A4_row_ifft"] == img + t1
    assert kb["F2_col_fft"] == kb["A3_col_ifft"] == t1 + grid
    assert kb["F3_interp"] == kb["A2_spread"] == grid + spec
    assert kb["F4_ray_ifft"] == kb["A1_ray_fft"] == spec + sino
    assert kb["A2_reduce"] == 0
    assert sum(kb.values()) == 744767488


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == ""
