"""The no-allocation entry point (gbs_lhaf_device_noalloc, through the C ABI)
against gbs_lhaf_device on the same device inputs: two calls in a row, the
second on a smaller input, FP64 and FP32-compensated, odd and empty inputs and
the argument checks.  Tolerance as for the other FP64 parity tests (reading
R6 of the design notes): both sides sum the same subset terms in a different
order, so |a - b| <= 2e-14 sum_S |t_S| (5e-6 sum_S |t_S| in FP32)."""
import numpy as np
import pytest

import paper_2010_15595_amd as gbs
from paper_2010_15595_amd import workloads

pytestmark = pytest.mark.gpu

NORMWISE = {gbs.GBS_FP64: 2e-14, gbs.GBS_FP32_COMP: 5e-6}


def _pair(A, prec):
    import torch

    dev = torch.device("cuda:0")
    At = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    o1 = torch.zeros(1, dtype=torch.complex128, device=dev)
    a1 = torch.zeros(1, dtype=torch.float64, device=dev)
    o2 = torch.full((1,), complex(np.nan, np.nan), dtype=torch.complex128, device=dev)
    a2 = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    gbs.lhaf_device(At, o1, a1, prec=prec)
    gbs.lhaf_device_noalloc(At, o2, a2, prec=prec)
    torch.cuda.synchronize()
    return complex(o1.cpu()[0]), float(a1.cpu()[0]), complex(o2.cpu()[0]), float(a2.cpu()[0])


def _check(tag, A, prec):
    ref, ab_ref, got, ab = _pair(A, prec)
    err = abs(got - ref)
    print(f"[noalloc {tag}] N={A.shape[0]} |diff|/sum|t| {err / max(ab_ref, 1e-300):.2e}", flush=True)
    assert ab == pytest.approx(ab_ref, rel=1e-12)
    assert err <= max(1e-10 * abs(ref), NORMWISE[prec] * ab_ref)


@pytest.fixture(scope="module", autouse=True)
def _init():
    gbs.init(0)


@pytest.mark.parametrize("prec", [gbs.GBS_FP64, gbs.GBS_FP32_COMP])
def test_two_calls_second_smaller(prec):
    for N in (50, 30):
        st = workloads.config3(N)
        A = gbs.expand(st["B"], st["gamma"], st["pattern"])
        _check(f"config3 prec={prec}", A, prec)


def test_odd_and_tiny_inputs():
    for N in (33, 7, 2, 1):
        _check("random", workloads.random_normal_symmetric(N, seed=300 + N, scale=0.5), gbs.GBS_FP64)


def test_empty_input():
    import torch

    dev = torch.device("cuda:0")
    A = torch.zeros((0, 0), dtype=torch.complex128, device=dev)
    out = torch.zeros(1, dtype=torch.complex128, device=dev)
    ab = torch.zeros(1, dtype=torch.float64, device=dev)
    gbs.lhaf_device_noalloc(A, out, ab)
    torch.cuda.synchronize()
    assert complex(out.cpu()[0]) == 1.0 and float(ab.cpu()[0]) == 1.0


def test_rejects_unsupported_requests():
    import torch

    dev = torch.device("cuda:0")
    A = torch.zeros((66, 66), dtype=torch.complex128, device=dev)
    out = torch.zeros(1, dtype=torch.complex128, device=dev)
    with pytest.raises(gbs.GbsError, match="TOO_LARGE"):
        gbs.lhaf_device_noalloc(A, out)
    with pytest.raises(gbs.GbsError, match="UNSUPPORTED"):
        gbs.lhaf_device_noalloc(A[:4, :4].contiguous(), out, prec=gbs.GBS_DD)
