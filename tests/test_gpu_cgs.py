"""GPU parity of cluster multicolor Gauss-Seidel (Algorithm 4, mis2_cgs_setup
and mis2_cgs_apply): the plan (clusters, colours, sweep order) must equal the
oracle's exactly, and so must x after forward and symmetric sweeps (each row
sums its entries in CSR order with separate roundings on both sides, and
clusters of one colour share no edge, so the parallel sweep is the
sequential one)."""
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


GRAPHS = {
    "grid27_20": lambda: graphs.grid3d_27pt(20, 19, 18),
    "grid7_30": lambda: graphs.grid3d_7pt(30, 30, 30),
    "grid2d": lambda: graphs.grid2d_5pt(61, 47),
    "chunglu_20k": lambda: graphs.chung_lu(20000, 10.0, 2.1, 1500, seed=6),
    "star300": lambda: graphs.star(300, 17),
    "path101": lambda: graphs.path(101),
    "edgeless50": lambda: graphs.edgeless(50),
    "union": lambda: graphs.disjoint_union([graphs.grid2d_5pt(10, 10), graphs.complete(9),
                                            graphs.edgeless(5), graphs.path(17)]),
    # the cluster sweep's batch limits: rows of exactly 64 entries (K65), rows
    # of 65 (K66, each a batch of its own) and 17 rows of 16 (K17: the first
    # batch holds exactly 256 entries, the last row starts a second)
    "cliques": lambda: graphs.disjoint_union([graphs.complete(65), graphs.complete(66),
                                              graphs.complete(17)]),
    # isolated vertices last: their CSR start is nnz, which no load may use
    "isolated_last": lambda: graphs.disjoint_union([graphs.grid2d_5pt(9, 7), graphs.edgeless(4)]),
}


def _plan_matches(plan, want, name):
    k, c = want["n_clusters"], want["n_colors"]
    assert plan.n_clusters == k and plan.n_colors == c, (name, plan.n_clusters, plan.n_colors)
    assert np.array_equal(plan.cluster.cpu().numpy()[:len(want["cluster"])], want["cluster"]), name
    assert np.array_equal(plan.cluster_color.cpu().numpy()[:k], want["cluster_color"]), name
    assert np.array_equal(plan.rows.cpu().numpy()[:len(want["rows"])], want["rows"]), name
    assert np.array_equal(plan.cluster_off.cpu().numpy()[:k + 1], want["cluster_off"]), name
    n = len(want["rows"])
    inv = np.empty(n, np.int32)
    inv[want["rows"]] = np.arange(n, dtype=np.int32)
    assert np.array_equal(plan.pos.cpu().numpy()[:n], inv), name
    assert np.array_equal(plan.color_off[:c + 1], want["color_off"]), name


@pytest.mark.parametrize("point", [False, True])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_cgs_plan_and_sweeps_match_oracle(ctx, name, point):
    import torch
    rp, cc = GRAPHS[name]()
    n = rp.size - 1
    _say("cgs", name, "point" if point else "cluster", n, int(rp[-1]))
    plan = ctx.cgs_setup(rp, cc, seed=2, point=point)
    want = oracle.cgs_plan(rp, cc, 2, point=point)
    _plan_matches(plan, want, name)
    val, diag = graphs.matrix_values(rp, cc, 1)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    dev = torch.device("cuda", 0)
    dval = torch.as_tensor(val if val.size else np.zeros(1), device=dev)
    ddiag = torch.as_tensor(diag, device=dev)
    db = torch.as_tensor(b, device=dev)
    for symmetric in (False, True):
        x = torch.as_tensor(x0.copy(), device=dev)
        ctx.cgs_apply(rp, cc, dval, ddiag, plan, db, x, sweeps=3, symmetric=symmetric)
        got = x.cpu().numpy()
        ref = oracle.cgs_apply(rp, cc, val, diag, want, b, x0, sweeps=3, symmetric=symmetric)
        assert np.array_equal(got, ref), (name, symmetric, np.max(np.abs(got - ref)))


def test_cgs_full_27_point_100_cube(ctx):
    import torch
    rp, cc = graphs.grid3d_27pt(100, 100, 100)
    n = rp.size - 1
    _say("cgs C2")
    plan = ctx.cgs_setup(rp, cc, seed=0)
    want = oracle.cgs_plan(rp, cc, 0)
    _plan_matches(plan, want, "C2")
    val, diag = graphs.matrix_values(rp, cc, 0)
    b = np.ones(n)
    dev = torch.device("cuda", 0)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    ctx.cgs_apply(rp, cc, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
                  plan, torch.as_tensor(b, device=dev), x, sweeps=1, symmetric=True)
    ref = oracle.cgs_apply(rp, cc, val, diag, want, b, np.zeros(n), sweeps=1, symmetric=True)
    assert np.array_equal(x.cpu().numpy(), ref)


def test_cgs_empty_graph(ctx):
    plan = ctx.cgs_setup(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert plan.n_clusters == 0 and plan.n_colors == 0


def test_cgs_validated_and_stale_workspace():
    # a validating context, a workspace full of 0xFF bytes before each setup,
    # and a larger graph after a smaller one: plans and sweeps stay exact
    import torch
    from paper_2204_02934_amd import api
    c = api.Context(0, validate=True)
    dev = torch.device("cuda", 0)
    for rp, cc in [graphs.grid2d_5pt(20, 17), graphs.chung_lu(5000, 8.0, 2.1, 600, seed=2),
                   graphs.grid3d_27pt(9, 9, 8)]:
        n = rp.size - 1
        for point in (False, True):
            if c._ws is not None:
                c._ws.fill_(0xFF)
            plan = c.cgs_setup(rp, cc, seed=5, point=point)
            want = oracle.cgs_plan(rp, cc, 5, point=point)
            _plan_matches(plan, want, "validated")
            val, diag = graphs.matrix_values(rp, cc, 3)
            b = np.linspace(-1.0, 1.0, n)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            c.cgs_apply(rp, cc, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
                        plan, torch.as_tensor(b, device=dev), x, sweeps=2, symmetric=True)
            ref = oracle.cgs_apply(rp, cc, val, diag, want, b, np.zeros(n), sweeps=2, symmetric=True)
            assert np.array_equal(x.cpu().numpy(), ref)


def test_cgs_rejects_bad_plans(ctx):
    import torch
    from paper_2204_02934_amd._lib import Mis2Error
    rp, cc = graphs.grid2d_5pt(8, 8)
    plan = ctx.cgs_setup(rp, cc)
    plan.c.n = 10  # not the graph's n
    dev = torch.device("cuda", 0)
    val, diag = graphs.matrix_values(rp, cc, 0)
    x = torch.zeros(64, dtype=torch.float64, device=dev)
    with pytest.raises(Mis2Error):
        ctx.cgs_apply(rp, cc, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
                      plan, torch.zeros(64, dtype=torch.float64, device=dev), x)
