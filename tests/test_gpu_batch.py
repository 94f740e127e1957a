"""GPU parity of batched multilevel coarsening (mis2_aggregate_batched): every
graph of a disjoint union must get, level by level, exactly the labels and
sizes the CPU oracle computes for that graph alone."""
import sys

import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_02934_amd import api
    return api.Context(0)


def _mixed():
    return [
        graphs.dropped_7pt(12, 0.1, seed=np.random.SeedSequence([2, 0])),
        graphs.star(300, 0),
        graphs.path(1500),
        (np.zeros(1, np.int64), np.zeros(0, np.int32)),  # a graph with no vertices
        graphs.edgeless(1),
        graphs.chung_lu(3000, 8.0, 2.1, 500, seed=4),
        graphs.grid3d_27pt(12, 12, 12),
        graphs.edgeless(1200),  # every vertex its own aggregate: stops after one level
        graphs.grid2d_5pt(40, 40),
        graphs.complete(40),
        graphs.cycle(777),
        graphs.grid3d_7pt(17, 13, 11),
    ]


def _union(gs):
    rp, c = graphs.disjoint_union(gs)
    voff = np.cumsum([0] + [g[0].size - 1 for g in gs]).astype(np.int64)
    return rp, c, voff


def _check(got, gs, stop, max_levels, seed, idx=None):
    idx = range(len(gs)) if idx is None else idx
    for i in idx:
        rp, c = gs[i]
        want = oracle.coarsen(rp, c, seed=seed, stop_below=stop, max_levels=max_levels)
        g = got[i]
        assert len(g) == len(want), (i, len(g), len(want))
        for lv, (a, b) in enumerate(zip(g, want)):
            assert (a["n"], a["nnz"], a["n_agg"]) == (b["n"], b["nnz"], b["n_agg"]), (i, lv)
            assert np.array_equal(a["agg"].cpu().numpy(), b["agg"]), (i, lv)


@pytest.mark.parametrize("stop,max_levels,seed", [(100, 64, 0), (50, 2, 3), (1, 64, 11),
                                                  (2000, 64, 0)])
def test_batched_mixed_graphs(ctx, stop, max_levels, seed):
    gs = _mixed()
    rp, c, voff = _union(gs)
    _say("batched mixed stop=%d max_levels=%d seed=%d" % (stop, max_levels, seed))
    got = ctx.aggregate_batched(rp, c, voff, seed=seed, stop_below=stop, max_levels=max_levels)
    _check(got, gs, stop, max_levels, seed)


def test_batched_level0_block_marks_graphs_without_levels(ctx):
    gs = [graphs.path(50), graphs.grid2d_5pt(30, 30), graphs.path(20)]
    rp, c, voff = _union(gs)
    out = ctx.aggregate_batched(rp, c, voff, seed=0, stop_below=100)
    assert [len(o) for o in out] == [0, len(oracle.coarsen(*gs[1], stop_below=100)), 0]
    _check(out, gs, 100, 64, 0)


def test_batched_single_graph_equals_coarsen(ctx):
    rp, c = graphs.grid3d_27pt(30, 29, 28)
    a = ctx.aggregate_batched(rp, c, np.array([0, rp.size - 1]), seed=5, stop_below=100)[0]
    b = ctx.coarsen(rp, c, seed=5, stop_below=100)
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert (x["n"], x["nnz"], x["n_agg"]) == (y["n"], y["nnz"], y["n_agg"])
        assert np.array_equal(x["agg"].cpu().numpy(), y["agg"].cpu().numpy())


def test_batched_no_graph_has_a_level(ctx):
    gs = [graphs.path(10), graphs.path(5)]
    rp, c, voff = _union(gs)
    assert ctx.aggregate_batched(rp, c, voff, stop_below=100) == [[], []]


def test_batched_subdomains_small(ctx):
    gs = graphs.batch_subdomains(num=48, lo=6, hi=20, seed=5)
    rp, c, voff = _union(gs)
    got = ctx.aggregate_batched(rp, c, voff, seed=0, stop_below=200)
    _check(got, gs, 200, 64, 0)


def test_batched_subdomains_full(ctx):
    # 512 dropped-edge 7-point subdomains of side 8..48, multilevel to < 1000
    # vertices in one batched call; every graph is checked against the
    # oracle run on that graph alone, level by level (about 15 s of CPU)
    gs = graphs.batch_subdomains(num=512, lo=8, hi=48, p_drop=0.1, seed=2)
    rp, c, voff = _union(gs)
    _say("C4 union n=%d nnz=%d" % (rp.size - 1, int(rp[-1])))
    got = ctx.aggregate_batched(rp, c, voff, seed=0, stop_below=1000)
    sizes = np.diff(voff)
    for i in range(len(gs)):
        assert (len(got[i]) == 0) == (sizes[i] < 1000), i
    _check(got, gs, 1000, 64, 0)
    _say("C4: all %d graphs equal the oracle, %d levels in all"
         % (len(gs), sum(len(g) for g in got)))
