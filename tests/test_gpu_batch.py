"""Batched loop hafnians (persistent kernels captured in a HIP graph)
against single evaluations and the oracle, including graph replays."""
import numpy as np
import pytest

import os
import sys

import oracle
from paper_2010_15595_amd import workloads

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_lhaf_refs  # noqa: E402

pytestmark = pytest.mark.gpu

NORMWISE = 2e-14


@pytest.fixture(scope="module")
def gbs():
    import paper_2010_15595_amd as g

    g.init(0)
    return g


def _items(count, seed, lo=0, hi=28):
    r = np.random.default_rng(seed)
    dims = [int(x) for x in r.integers(lo, hi + 1, count)]
    mats = [workloads.random_normal_symmetric(N, seed=1000 * seed + i, scale=0.5) for i, N in enumerate(dims)]
    return dims, mats


def _run(gbs, plan, mats):
    import torch

    dev = torch.device("cuda:0")
    packed = torch.from_numpy(gbs.pack(mats)).to(dev)
    out = torch.zeros(len(mats), dtype=torch.complex128, device=dev)
    ab = torch.zeros(len(mats), dtype=torch.float64, device=dev)
    plan.run(packed, out, ab)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ab.cpu().numpy()


def test_batch_matches_single_evaluations_and_oracle(gbs):
    dims, mats = _items(40, seed=1)
    plan = gbs.BatchPlan(dims)
    info = plan.info()
    print(f"[batch] {info}", flush=True)
    got, ab = _run(gbs, plan, mats)
    worst = 0.0
    for i, A in enumerate(mats):
        single, d = gbs.lhaf(A, with_diag=True)
        assert abs(got[i] - single) <= NORMWISE * d["abs_sum"] + 1e-300, (i, dims[i])
        assert ab[i] == pytest.approx(d["abs_sum"], rel=1e-9)
        if dims[i] <= 20:
            ref = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
            assert abs(got[i] - ref) <= max(1e-10 * abs(ref), NORMWISE * ab[i])
            worst = max(worst, abs(got[i] - ref) / max(ab[i], 1e-300))
    print(f"[batch] worst normwise error vs oracle {worst:.2e}", flush=True)
    plan.close()


def test_graph_replays_are_identical(gbs):
    import torch

    dims, mats = _items(25, seed=2, lo=6, hi=30)
    plan = gbs.BatchPlan(dims)
    first, _ = _run(gbs, plan, mats)
    for rep in range(3):
        # eager work and synchronisation between replays
        x = torch.randn(1 << 16, device="cuda:0")
        _ = (x * x).sum().item()
        gbs.lhaf(mats[0])
        again, _ = _run(gbs, plan, mats)
        assert np.array_equal(again, first), f"replay {rep} differs"
    plan.close()


def test_batch_chain_like_patterns(gbs):
    """Items of the chain-like workload: expanded from one 100-mode state."""
    st = workloads.config4(count=48)
    mats = [gbs.expand(st["B"], st["gamma"], pat) for pat in st["patterns"]]
    dims = [a.shape[0] for a in mats]
    plan = gbs.BatchPlan(dims)
    got, ab = _run(gbs, plan, mats)
    for i, A in enumerate(mats):
        single, d = gbs.lhaf(A, with_diag=True)
        assert abs(got[i] - single) <= NORMWISE * d["abs_sum"], (i, dims[i])
    plan.close()


def test_batch_fp32_path(gbs):
    dims, mats = _items(20, seed=3, lo=4, hi=20)
    plan = gbs.BatchPlan(dims, prec=gbs.GBS_FP32_COMP)
    got, ab = _run(gbs, plan, mats)
    for i, A in enumerate(mats):
        ref = oracle.to_complex(oracle.lhaf_pt(A, prec="ld"))
        assert abs(got[i] - ref) <= 5e-6 * ab[i] + 1e-300, (i, dims[i])
    plan.close()


def test_batch_autotuned_plan(gbs):
    dims, mats = _items(30, seed=4, lo=10, hi=30)
    plan = gbs.BatchPlan(dims, autotune=True)
    info = plan.info()
    assert info["tile_subsets"] in (64, 128, 256, 1024, 4096, 16384, 65536)
    print(f"[batch autotune] tile {info['tile_subsets']}, {info['tune_ms']:.2f} ms", flush=True)
    got, _ = _run(gbs, plan, mats)
    for i, A in enumerate(mats):
        single, d = gbs.lhaf(A, with_diag=True)
        assert abs(got[i] - single) <= NORMWISE * d["abs_sum"]
    plan.close()


def test_batch_edge_items(gbs):
    """Empty, one-vertex and odd-dimension items; a batch with no items."""
    dims = [0, 1, 2, 3, 5, 0, 9, 14, 1]
    mats = [workloads.random_normal_symmetric(N, seed=70 + i, scale=0.7) for i, N in enumerate(dims)]
    plan = gbs.BatchPlan(dims)
    got, ab = _run(gbs, plan, mats)
    for i, A in enumerate(mats):
        ref = oracle.to_complex(oracle.lhaf_dp(A)) if dims[i] > 0 else 1.0
        assert abs(got[i] - ref) <= 1e-12 * max(1.0, abs(ref), ab[i]), (i, dims[i], got[i], ref)
    plan.close()
    empty = gbs.BatchPlan([])
    assert empty.info()["items"] == 0
    got, _ = _run(gbs, empty, [])
    assert got.shape == (0,)
    empty.close()


def test_batch_rejects_bad_dims(gbs):
    with pytest.raises(gbs.GbsError):
        gbs.BatchPlan([10, 70])


def test_batch_with_one_team_layout(gbs):
    """Batch tiles on the 8x4 grid with one 64-lane La Budde team (forced for
    every subset size it can hold) against single evaluations on the default
    grids: the team guard of the batch kernel must let these tiles through."""
    dims, mats = _items(24, seed=7, lo=18, hi=34)
    gbs.set_layout(0, 0, 3)
    try:
        plan = gbs.BatchPlan(dims)
        got, ab = _run(gbs, plan, mats)
        plan.close()
    finally:
        gbs.set_layout(0, 0, -1)
    for i, A in enumerate(mats):
        single, d = gbs.lhaf(A, with_diag=True)
        assert abs(got[i] - single) <= NORMWISE * d["abs_sum"], (i, dims[i])


def test_full_size_chain_workload(gbs):
    """The 4096-item chain-like workload the batch benchmark replays, in the
    same plan configuration: one item of every N in 22..36 and the eight
    largest against the long-double oracle (stored full sums, which run on the
    persistent kernels); sampled items against single evaluations, and the
    items with N <= 16 among them against the oracle."""
    st = workloads.config4(count=4096)
    mats = [gbs.expand(st["B"], st["gamma"], pat) for pat in st["patterns"]]
    dims = [a.shape[0] for a in mats]
    plan = gbs.BatchPlan(dims)
    got, ab = _run(gbs, plan, mats)
    plan.close()
    refs = make_lhaf_refs.load()
    picks = make_lhaf_refs.c4_picks(dims)
    assert sorted({dims[i] for i in picks}) == list(range(22, 37, 2))
    worst_ld = 0.0
    for i in picks:
        Nr, re, im, ab_ref = refs[f"c4_{i}"]
        assert Nr == dims[i]
        ref = complex(float(re), float(im))
        err = abs(got[i] - ref)
        assert ab[i] == pytest.approx(float(ab_ref), rel=1e-12), i
        assert err <= max(1e-10 * abs(ref), NORMWISE * float(ab_ref)), (i, dims[i], err / float(ab_ref))
        worst_ld = max(worst_ld, err / float(ab_ref))
    print(f"[batch 4096] {len(picks)} items N=22..36 vs long-double oracle: worst |err|/sum|t| {worst_ld:.2e}",
          flush=True)
    order = np.argsort(dims)
    pick = sorted(set([int(i) for i in order[-8:]] + [int(i) for i in order[:8]] +
                      [int(i) for i in np.random.default_rng(1).choice(len(mats), 16, replace=False)]))
    worst = 0.0
    for i in pick:
        single, d = gbs.lhaf(mats[i], with_diag=True)
        assert abs(got[i] - single) <= NORMWISE * d["abs_sum"], (i, dims[i])
        worst = max(worst, abs(got[i] - single) / d["abs_sum"])
        if dims[i] <= 16:
            ref = oracle.to_complex(oracle.lhaf_pt(mats[i], prec="ld"))
            assert abs(got[i] - ref) <= max(1e-10 * abs(ref), NORMWISE * ab[i]), (i, dims[i])
    print(f"[batch 4096] {len(pick)} sampled items, N {min(dims)}..{max(dims)}, worst |batch-single|/sum|t| "
          f"{worst:.2e}", flush=True)


def test_plan_survives_finalize(gbs):
    """A plan owns its copies of the library tables: run, gbs_finalize,
    gbs_init, run again gives identical results."""
    dims, mats = _items(12, seed=11, lo=10, hi=30)
    plan = gbs.BatchPlan(dims)
    first, _ = _run(gbs, plan, mats)
    gbs.finalize()
    gbs.init(0)
    again, _ = _run(gbs, plan, mats)
    plan.close()
    assert np.array_equal(first, again)
