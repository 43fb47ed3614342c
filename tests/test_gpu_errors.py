"""Failure handling on the GPU, forced from the host: device allocations made to
fail through the library's test hook (GBS_TEST_FAIL_ALLOC=1) must return
GBS_E_NOMEM with the caller's outputs untouched, leave the library usable, and
a context whose creation failed must leave nothing behind."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2010_15595_amd as gbs
from paper_2010_15595_amd import _lib, workloads

pytestmark = pytest.mark.gpu

NOMEM = -8


def _raw_lhaf(A):
    """gbs_lhaf through the C ABI with a sentinel in the output."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    N = A.shape[0]
    out = _lib.gbs_z(7.0, -7.0)
    rc = gbs.lib().gbs_lhaf(A.ctypes.data_as(ctypes.POINTER(_lib.gbs_z)), N, N, None, None, gbs.GBS_FP64,
                            ctypes.byref(out), None)
    return rc, complex(out.re, out.im)


def test_out_of_memory_paths(monkeypatch):
    gbs.finalize()
    # context creation: every allocation fails, nothing is left behind
    monkeypatch.setenv("GBS_TEST_FAIL_ALLOC", "1")
    assert gbs.lib().gbs_init(0) == NOMEM
    monkeypatch.delenv("GBS_TEST_FAIL_ALLOC")
    assert gbs.lib().gbs_init(0) == 0
    # a call whose workspace has to grow
    A = workloads.random_normal_symmetric(40, seed=5, scale=0.4)
    monkeypatch.setenv("GBS_TEST_FAIL_ALLOC", "1")
    rc, out = _raw_lhaf(A)
    assert rc == NOMEM and out == complex(7.0, -7.0)
    assert b"hipMalloc" in gbs.lib().gbs_last_error()
    # batch plan creation
    plan = ctypes.c_void_p(0x1234)
    dims = (ctypes.c_int32 * 3)(10, 20, 24)
    assert gbs.lib().gbs_batch_plan_create(dims, 3, gbs.GBS_FP64, 0, ctypes.byref(plan)) == NOMEM
    assert plan.value == 0x1234
    monkeypatch.delenv("GBS_TEST_FAIL_ALLOC")
    # the library works again
    rc, out = _raw_lhaf(A)
    assert rc == 0
    ref, ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
    ref = oracle.to_complex(ref)
    assert abs(out - ref) <= max(1e-10 * abs(ref), 2e-14 * float(ab))
    p = gbs.BatchPlan([10, 20, 24])
    p.close()
