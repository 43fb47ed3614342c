"""One GPU's share of the subset sum (gbs_lhaf_device_shard, through the C
ABI) and the host fold of the shard records (gbs_combine_partials).

G shards of one loop hafnian, run one after another on the one GPU and folded
in shard order, must give gbs_lhaf_device's result: bitwise for G = 1 (the
same partial records in the same reduction tree), and for G > 1 to the FP64
parity tolerance of the other tests (reading R6 of the design notes): the
same subset terms summed in a different grouping, so
|a - b| <= 2e-14 sum_S |t_S| (5e-6 sum_S |t_S| in FP32).  The N = 50
benchmark matrix split four ways meets the long-double oracle value under
the full-size gate."""
import os
import sys

import numpy as np
import pytest

import paper_2010_15595_amd as gbs
from paper_2010_15595_amd import workloads

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_lhaf_refs  # noqa: E402

pytestmark = pytest.mark.gpu

NORMWISE = {gbs.GBS_FP64: 2e-14, gbs.GBS_FP32_COMP: 5e-6}


@pytest.fixture(scope="module", autouse=True)
def _init():
    gbs.init(0)


def _whole(At, prec):
    import torch

    o = torch.zeros(1, dtype=torch.complex128, device=At.device)
    a = torch.zeros(1, dtype=torch.float64, device=At.device)
    gbs.lhaf_device(At, o, a, prec=prec)
    torch.cuda.synchronize()
    return complex(o.cpu()[0]), float(a.cpu()[0])


def _sharded(At, G, prec):
    import torch

    rec = torch.full((G, 5), np.nan, dtype=torch.float64, device=At.device)
    for g in range(G):
        gbs.lhaf_device_shard(At, rec[g], g, G, prec=prec)
    torch.cuda.synchronize()
    records = rec.cpu().numpy()
    assert np.all(np.isfinite(records))
    return gbs.combine_partials(records), records


def _dev(A):
    import torch

    return torch.from_numpy(np.ascontiguousarray(A)).to(torch.device("cuda:0"))


def _c3(N):
    st = workloads.config3(N)
    return gbs.expand(st["B"], st["gamma"], st["pattern"])


@pytest.mark.parametrize("prec", [gbs.GBS_FP64, gbs.GBS_FP32_COMP])
def test_one_shard_is_the_whole_sum_bitwise(prec):
    At = _dev(_c3(30))
    ref, ab_ref = _whole(At, prec)
    (val, ab), _ = _sharded(At, 1, prec)
    assert val == ref and ab == ab_ref


@pytest.mark.parametrize("prec", [gbs.GBS_FP64, gbs.GBS_FP32_COMP])
@pytest.mark.parametrize("G", [2, 3, 7])
def test_shards_fold_to_the_whole_sum(G, prec):
    for N in (36, 31):
        A = _c3(N) if N % 2 == 0 else workloads.random_normal_symmetric(N, seed=500 + N, scale=0.5)
        At = _dev(A)
        ref, ab_ref = _whole(At, prec)
        (val, ab), rec = _sharded(At, G, prec)
        err = abs(val - ref)
        print(f"[shard G={G} N={N} prec={prec}] |diff|/sum|t| {err / ab_ref:.2e}; "
              f"shares of sum|t| {np.round(rec[:, 4] / ab_ref, 3).tolist()}", flush=True)
        assert ab == pytest.approx(ab_ref, rel=1e-12)
        assert err <= max(1e-10 * abs(ref), NORMWISE[prec] * ab_ref)


def test_more_shards_than_subsets_of_a_class():
    # N = 4: two pairs, classes of 2 and 1 subsets.  Of 8 shards, shard 3 takes
    # rank 0 of the 1-subsets (ranks [2*3//8, 2*4//8) = [0, 1)) and shard 7 rank 1
    # of them and the one 2-subset; the other six are empty
    A = workloads.random_normal_symmetric(4, seed=41, scale=0.7)
    At = _dev(A)
    ref, ab_ref = _whole(At, gbs.GBS_FP64)
    (val, ab), rec = _sharded(At, 8, gbs.GBS_FP64)
    assert np.nonzero(rec[:, 4])[0].tolist() == [3, 7]
    assert abs(val - ref) <= 2e-14 * ab_ref and ab == pytest.approx(ab_ref, rel=1e-14)


def test_empty_matrix_goes_to_shard_zero():
    import torch

    At = torch.zeros((0, 0), dtype=torch.complex128, device=torch.device("cuda:0"))
    (val, ab), rec = _sharded(At, 3, gbs.GBS_FP64)
    assert val == 1.0 and ab == 1.0
    assert rec[0].tolist() == [1.0, 0.0, 0.0, 0.0, 1.0] and not rec[1:].any()


def test_benchmark_matrix_in_four_shards_against_long_double():
    """The N = 50 benchmark matrix, one quarter of every size class per shard
    (classes above 2^20 subsets still run in several launches), folded and
    compared with the stored long-double oracle value (gate of the full-size
    tests)."""
    N, re, im, ab_ref = make_lhaf_refs.load()["c3_50"]
    ref = complex(float(re), float(im))
    At = _dev(_c3(50))
    (val, ab), rec = _sharded(At, 4, gbs.GBS_FP64)
    err = abs(val - ref)
    print(f"[shard G=4 N=50] rel err {err / abs(ref):.2e}, |err|/sum|t| {err / float(ab_ref):.2e}; "
          f"shares of sum|t| {np.round(rec[:, 4] / float(ab_ref), 3).tolist()}", flush=True)
    assert ab == pytest.approx(float(ab_ref), rel=1e-12)
    assert err <= max(1e-10 * abs(ref), 2e-14 * float(ab_ref))


def test_rejects_bad_shards():
    import torch

    dev = torch.device("cuda:0")
    At = _dev(_c3(16))
    rec = torch.zeros(5, dtype=torch.float64, device=dev)
    for g, G in ((2, 2), (-1, 2), (0, 0), (0, 65537)):
        with pytest.raises(gbs.GbsError, match="E_ARG"):
            gbs.lhaf_device_shard(At, rec, g, G)
    with pytest.raises(gbs.GbsError, match="UNSUPPORTED"):
        gbs.lhaf_device_shard(At, rec, 0, 2, prec=gbs.GBS_DD)
