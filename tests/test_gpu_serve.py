"""GPU parity of the serving loop (mis2_server_*): jobs that arrive between
steps join the running union at level boundaries, and every job must still
get exactly the oracle's multilevel coarsening of its own graph."""
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


def _jobs():
    return [
        graphs.grid2d_5pt(70, 60),
        graphs.grid3d_27pt(14, 13, 12),
        graphs.chung_lu(6000, 10.0, 2.1, 800, seed=7),
        graphs.path(3000),
        graphs.edgeless(50),  # below stop_below: finishes at submit, no level
        graphs.dropped_7pt(16, 0.1, seed=np.random.SeedSequence([2, 7])),
        graphs.star(500, 3),
        graphs.cycle(2500),
        graphs.grid3d_7pt(20, 20, 9),
        graphs.chung_lu(9000, 16.0, 2.1, 2000, seed=8),
        graphs.complete(120),
        graphs.grid2d_5pt(33, 100),
    ]


def _check_job(levels, rp, c, stop):
    want = oracle.coarsen(rp, c, seed=0, stop_below=stop)
    assert len(levels) == len(want)
    for a, b in zip(levels, want):
        assert (a["n"], a["nnz"], a["n_agg"]) == (b["n"], b["nnz"], b["n_agg"])
        assert np.array_equal(a["agg"].cpu().numpy(), b["agg"])


def test_server_staggered_arrivals_match_oracle(api):
    jobs = _jobs()
    # room for a few jobs at a time, so later jobs queue and join mid-way
    srv = api.Server(max_vertices=20000, max_nnz=400000, max_graphs=4, seed=0, stop_below=100)
    done, steps, nxt = {}, 0, 0
    while len(done) < len(jobs):
        for _ in range(2):  # two arrivals per step
            if nxt < len(jobs):
                srv.submit(*jobs[nxt], tag=nxt)
                nxt += 1
        srv.step()
        steps += 1
        for r in srv.poll():
            done[r["tag"]] = r
        assert steps < 200
    _say("server: %d jobs in %d steps" % (len(jobs), steps))
    for t, (rp, c) in enumerate(jobs):
        assert not done[t]["truncated"]
        _check_job(done[t]["levels"], rp, c, 100)
    srv.close()


def test_server_all_at_once_equals_one_by_one(api):
    jobs = _jobs()[:6]
    a = api.Server(max_vertices=60000, max_nnz=1000000, max_graphs=16, seed=0, stop_below=100)
    for t, g in enumerate(jobs):
        a.submit(*g, tag=t)
    res_a = {}
    while a.step() > 0 or len(res_a) < len(jobs):
        for r in a.poll():
            res_a[r["tag"]] = r
    for t, (rp, c) in enumerate(jobs):
        _check_job(res_a[t]["levels"], rp, c, 100)
    a.close()


def test_server_rejects_oversized_and_truncates(api):
    from paper_2204_02934_amd._lib import Mis2Error
    srv = api.Server(max_vertices=5000, max_nnz=50000, max_graphs=2, seed=0, stop_below=100)
    with pytest.raises(Mis2Error):
        srv.submit(*graphs.grid2d_5pt(100, 100), tag=1)  # 10000 vertices > 5000
    rp, c = graphs.grid2d_5pt(40, 40)
    srv.submit(rp, c, tag=2, agg_cap=rp.size - 1)  # room for level 0 only
    while srv.step() > 0:
        pass
    (r,) = srv.poll()
    assert r["tag"] == 2 and r["truncated"] and len(r["levels"]) == 1
    want = oracle.coarsen(rp, c, seed=0, stop_below=100)[0]
    assert np.array_equal(r["levels"][0]["agg"].cpu().numpy(), want["agg"])
    srv.close()


def test_server_recipe_pool_matches_oracle(api):
    # the serving workload's own job mix: n log-uniform on [1e3, 1e7], 2D
    # 5-point / 3D 27-point / Chung-Lu 40/40/20, multilevel to < 1000
    # vertices.  The first 12 jobs of the seeded pool hold a 27-point job of
    # 1.6M vertices, a Chung-Lu job of 0.9M vertices with hubs of 14k
    # neighbours, and 5-point jobs of up to 0.87M vertices.  Capacity for
    # about two large jobs at a time, two arrivals per step: later jobs queue
    # and join the running union between levels.
    pool = graphs.serving_pool(12, seed=3)
    kinds = [k for k, _ in pool]
    sizes = [g[0].size - 1 for _, g in pool]
    assert any(k == "3d27" and n >= 1_000_000 for k, n in zip(kinds, sizes))
    assert any(k == "chunglu" and int(np.diff(g[0]).max()) >= 10_000 for k, g in pool)
    srv = api.Server(max_vertices=3_000_000, max_nnz=64_000_000, max_graphs=8, seed=0,
                     stop_below=1000)
    done, steps, nxt = {}, 0, 0
    while len(done) < len(pool):
        for _ in range(2):
            if nxt < len(pool):
                srv.submit(*pool[nxt][1], tag=nxt)
                nxt += 1
        srv.step()
        steps += 1
        for r in srv.poll():
            done[r["tag"]] = r
        assert steps < 400
    _say("server: %d recipe jobs (%d vertices) in %d steps" % (len(pool), sum(sizes), steps))
    for t, (kind, (rp, c)) in enumerate(pool):
        assert not done[t]["truncated"], t
        _say("job %d %s n=%d levels=%d" % (t, kind, rp.size - 1, len(done[t]["levels"])))
        _check_job(done[t]["levels"], rp, c, 1000)
    srv.close()
