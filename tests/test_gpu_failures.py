"""Failure paths of the C ABI on the GPU: device allocation failures while a
plan is built (forced from the host through the RADON_TEST_FAIL_ALLOC hook)
return RADON_ERR_OOM with a NULL plan and leave no device memory behind."""
import ctypes
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from radon_inputs import uniform_angles  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1009_1380_amd import Plan  # noqa: E402
from paper_1009_1380_amd import radon as rb  # noqa: E402


def _plan_raw(n, ang, n_det):
    h = ctypes.c_void_p(12345)
    a = np.ascontiguousarray(ang, dtype=np.float64)
    rc = rb.lib().radon_plan(ctypes.byref(h), n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(a),
                             n_det, 2.0, 6)
    return rc, h


def _sweep(n, ang):
    """Build the plan with allocation k failing, k = 1, 2, ... until it succeeds;
    returns the number of failures."""
    k, failures = 1, 0
    try:
        while True:
            print(f"plan with allocation {k} failing", flush=True)
            sys.stdout.flush()
            os.environ["RADON_TEST_FAIL_ALLOC"] = str(k)
            rc, h = _plan_raw(n, ang, n)
            if rc == rb.RADON_OK:
                rb.lib().radon_plan_destroy(h)
                return failures
            assert rc == rb.RADON_ERR_OOM, (k, rc, rb.lib().radon_last_error())
            assert h.value is None, "a failed plan must set *out = NULL"
            assert b"fail" in rb.lib().radon_last_error().lower()
            failures += 1
            k += 1
            assert k < 200
    finally:
        os.environ.pop("RADON_TEST_FAIL_ALLOC", None)


def test_plan_allocation_failures_are_clean():
    n, nv = 1024, 180
    ang = uniform_angles(nv)
    f1 = _sweep(n, ang)
    assert f1 >= 20   # every device buffer of the plan was made to fail once
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    f2 = _sweep(n, ang)
    assert f2 == f1
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    # a second sweep of failed plans (each holding up to tens of MB when it
    # failed) leaves the device's free memory where the first left it
    assert abs(free2 - free1) <= 2 * 1024 * 1024, (free1, free2)
    # and the library still works afterwards
    plan = Plan(n, ang, n)
    x = torch.ones((n, n), device="cuda:0")
    assert torch.isfinite(plan.forward(x)).all()
