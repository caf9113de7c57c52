"""The ring filter entry point that allocates nothing (radon_ring_filter_noalloc)
against the allocating one (radon_ring_filter), through the C ABI: equal bit
for bit, and within the oracle's tolerance, on two calls in a row, the second
with a smaller plan (the static scratch array keeps the first call's contents)."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.solver import ring_filter  # noqa: E402
from radon_inputs import random_sinogram, uniform_angles  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1009_1380_amd import Plan  # noqa: E402
from paper_1009_1380_amd import radon as rb  # noqa: E402

DEV = "cuda:0"


def _sino(seed, nv, N):
    y = random_sinogram(seed, nv, N)
    y += np.tile(np.random.default_rng(seed + 1).normal(0, 0.3, N), (nv, 1)).astype(np.float32)
    return y


def _noalloc(plan, yd, out):
    st = torch.cuda.current_stream()
    rc = rb.lib().radon_ring_filter_noalloc(plan._h, ctypes.c_void_p(yd.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(st.cuda_stream))
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_ring_filter_matches_allocating_one(order):
    for k, (n, nv, N) in enumerate([(64, 45, 96), (32, 20, 48)]):
        print(f"noalloc ring filter call {k}: n={n} views={nv} n_det={N}", flush=True)
        sys.stdout.flush()
        y = _sino(100 + k, nv, N)
        plan = Plan(n, uniform_angles(nv), N)
        yd = torch.from_numpy(y).to(DEV)
        ref = plan.ring_filter(yd)
        out = torch.full_like(yd, float("nan"))
        assert _noalloc(plan, yd, out) == 0, rb.lib().radon_last_error()
        assert torch.equal(out, ref)
        o = ring_filter(y.astype(np.float64))
        assert np.linalg.norm(out.cpu().numpy() - o) <= 1e-6 * np.linalg.norm(o)
        plan.close()


def test_noalloc_ring_filter_rejects_null():
    plan = Plan(32, uniform_angles(20), 48)
    y = torch.zeros((20, 48), device=DEV)
    rc = rb.lib().radon_ring_filter_noalloc(plan._h, None, ctypes.c_void_p(y.data_ptr()), None)
    assert rc == rb.RADON_ERR_INVALID
    plan.close()
