"""GPU tests of the plan tuner (MIS2_OPT_AUTOTUNE): whatever plan it picks,
MIS-2 and aggregation stay bit-identical to the oracle; the tuned plan is
cached per graph class and device, and explicit plans bypass it."""
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
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_02934_amd import api as a
    return a


def _mis2_ok(c, rp, cc, seed, name):
    st, nr, it = c.mis2(rp, cc, seed)
    o = oracle.mis2_ex(rp, cc, seed)
    assert np.array_equal(st.cpu().numpy(), o["status"]), name
    assert it == o["n_iters"], name
    assert np.array_equal(c.last_trace(0), o["trace"][:, :2]), name


def _agg_ok(c, rp, cc, seed, name):
    agg, na = c.aggregate(rp, cc, seed)
    oa, ona = oracle.aggregate(rp, cc, seed)
    assert na == ona and np.array_equal(agg.cpu().numpy(), oa), name


CASES = [
    ("27-point 41x40x39", lambda: graphs.grid3d_27pt(41, 40, 39)),
    ("7-point 50^3", lambda: graphs.grid3d_7pt(50, 50, 50)),
    ("5-point 300x200", lambda: graphs.grid2d_5pt(300, 200)),
    ("Chung-Lu 60000", lambda: graphs.chung_lu(60000, 16.0, 2.1, 5000, seed=11)),
]


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_tuned_plan_matches_oracle(api, name):
    rp, cc = dict(CASES)[name]()
    c = api.Context(0)
    _mis2_ok(c, rp, cc, 2, name)
    p = c.last_plan()
    _say("%s: plan %s, tuning %s" % (name, p, c.last_tuning()))
    assert p["source"] in (1, 2)
    if p["source"] == 2:
        t = c.last_tuning()
        assert len(t) == 6 and all(r["ms"] > 0 for r in t)
        assert {r["lanes"] for r in t} == {1, 2, 4, 8, -2}
        # the last candidate is the fastest lane plan with the one-workgroup tail
        assert [r["tail"] for r in t] == [0] * 5 + [1]
    # the same graph again: the plan comes from the cache
    _agg_ok(c, rp, cc, 2, name)
    assert c.last_plan()["source"] == 1
    # another context on the device shares the class's plan
    d = api.Context(0)
    _mis2_ok(d, rp, cc, 5, name)
    q = d.last_plan()
    assert q["source"] == 1 and (q["lanes"], q["blocks"]) == (p["lanes"], p["blocks"])


def test_explicit_plans_and_small_graphs_skip_the_tuner(api):
    rp, cc = graphs.grid3d_27pt(30, 30, 30)
    c = api.Context(0, lanes=4)
    _mis2_ok(c, rp, cc, 0, "explicit")
    p = c.last_plan()
    assert (p["lanes"], p["source"], p["tail"]) == (4, 0, 0)
    off = api.Context(0, autotune=False)
    _mis2_ok(off, rp, cc, 0, "autotune off")
    assert off.last_plan()["source"] == 0
    small = api.Context(0)
    rp2, cc2 = graphs.grid2d_5pt(64, 64)  # 4096 vertices: below the tuner's size
    _mis2_ok(small, rp2, cc2, 0, "C1")
    assert small.last_plan()["source"] == 0


def test_tuned_batched_levels_match_oracle(api):
    gs = graphs.batch_subdomains(num=24, lo=10, hi=30, p_drop=0.1, seed=8)
    rp, cc = graphs.disjoint_union(gs)
    voff = np.cumsum([0] + [g[0].size - 1 for g in gs]).astype(np.int64)
    c = api.Context(0)
    got = c.aggregate_batched(rp, cc, voff, seed=0, stop_below=200)
    for i, (grp, gcol) in enumerate(gs):
        want = oracle.coarsen(grp, gcol, seed=0, stop_below=200)
        assert len(got[i]) == len(want), i
        for a, b in zip(got[i], want):
            assert (a["n"], a["nnz"], a["n_agg"]) == (b["n"], b["nnz"], b["n_agg"]), i
            assert np.array_equal(a["agg"].cpu().numpy(), b["agg"]), i


def test_lookup_only_never_tunes(api):
    # autotune = 2 takes a class's tuned plan when one exists, else the
    # degree rule, and never times candidates itself
    # every degree 2, n in [393216, 524288): a class no other test tunes (the
    # paths of the tuple-width tests sit at 2^12, 2^17 and 2^20)
    rp, cc = graphs.cycle(400_001)
    look = api.Context(0, autotune=2)
    _mis2_ok(look, rp, cc, 1, "lookup, new class")
    assert look.last_plan()["source"] == 0 and look.last_tuning() == []
    tuner = api.Context(0)
    _mis2_ok(tuner, rp, cc, 1, "tuning")
    p = tuner.last_plan()
    assert p["source"] in (1, 2)
    _agg_ok(look, rp, cc, 3, "lookup, tuned class")
    q = look.last_plan()
    assert q["source"] == 1 and (q["lanes"], q["blocks"]) == (p["lanes"], p["blocks"])
    with pytest.raises(Exception):
        api.Context(0, autotune=3)
