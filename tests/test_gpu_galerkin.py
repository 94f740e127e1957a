"""GPU parity of the Galerkin coarse operator (mis2_galerkin): P^T A P of an
aggregation with the tentative prolongator, bit for bit against the oracle
(both sum over the fine rows in increasing id, diagonal first, then CSR
order, and divide once by sqrt(n_a * n_b)).  The aggregation and the
quotient graph come from the oracle, so only the operator is under test."""
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
    # coarse rows of up to about 3000 columns: past the LDS accumulators
    "chunglu_50k": lambda: graphs.chung_lu(50000, 16.0, 2.1, 3000, seed=5),
    "star300": lambda: graphs.star(300, 17),
    "path101": lambda: graphs.path(101),
    "edgeless50": lambda: graphs.edgeless(50),
    "er": lambda: graphs.erdos_renyi(1700, 0.004, seed=12),
    "union": lambda: graphs.disjoint_union([graphs.grid2d_5pt(10, 10), graphs.complete(9),
                                            graphs.edgeless(5), graphs.path(17)]),
}


def _run(ctx, rp, cc, val, diag, agg, na):
    import torch
    dev = torch.device("cuda", 0)
    crow, ccol = oracle.quotient(rp, cc, agg, na)
    cval, cdiag = ctx.galerkin(rp, cc, torch.as_tensor(val if val.size else np.zeros(1), device=dev),
                               torch.as_tensor(diag, device=dev), agg, crow, ccol)
    return crow, ccol, cval.cpu().numpy(), cdiag.cpu().numpy()


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_galerkin_matches_oracle(ctx, name):
    rp, cc = GRAPHS[name]()
    _say("galerkin", name, rp.size - 1, int(rp[-1]))
    for seed in (0, 3):
        val, diag = graphs.matrix_values(rp, cc, seed, shift=0.5)
        agg, na = oracle.aggregate(rp, cc, seed)
        crow, ccol, cval, cdiag = _run(ctx, rp, cc, val, diag, agg, na)
        _, _, wval, wdiag = oracle.galerkin(rp, cc, val, diag, agg, na, crow, ccol)
        assert np.array_equal(cval, wval), (name, seed, np.max(np.abs(cval - wval)))
        assert np.array_equal(cdiag, wdiag), (name, seed)


def test_identity_aggregation_copies_the_matrix(ctx):
    rp, cc = graphs.grid3d_27pt(12, 11, 10)
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, cc, 2)
    _, _, cval, cdiag = _run(ctx, rp, cc, val, diag, np.arange(n, dtype=np.int32), n)
    assert np.array_equal(cval, val) and np.array_equal(cdiag, diag)


def test_galerkin_full_27_point_100_cube(ctx):
    rp, cc = graphs.grid3d_27pt(100, 100, 100)
    _say("galerkin C2")
    val, diag = graphs.matrix_values(rp, cc, 0)
    agg, na = oracle.aggregate(rp, cc, 0)
    crow, ccol, cval, cdiag = _run(ctx, rp, cc, val, diag, agg, na)
    _, _, wval, wdiag = oracle.galerkin(rp, cc, val, diag, agg, na, crow, ccol)
    assert np.array_equal(cval, wval) and np.array_equal(cdiag, wdiag)


def test_galerkin_rejects_bad_labels_and_missing_couplings(ctx):
    import torch
    from paper_2204_02934_amd._lib import Mis2Error
    rp, cc = graphs.grid2d_5pt(9, 8)
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, cc, 1)
    agg, na = oracle.aggregate(rp, cc, 0)
    crow, ccol = oracle.quotient(rp, cc, agg, na)
    dev = torch.device("cuda", 0)
    dval, ddiag = torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev)
    bad = agg.copy()
    bad[5] = na
    with pytest.raises(Mis2Error):
        ctx.galerkin(rp, cc, dval, ddiag, bad, crow, ccol)
    bad[5] = -1
    with pytest.raises(Mis2Error):
        ctx.galerkin(rp, cc, dval, ddiag, bad, crow, ccol)
    # a coarse graph with no edges lacks every coupling between aggregates
    with pytest.raises(Mis2Error):
        ctx.galerkin(rp, cc, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
                     agg, np.zeros(na + 1, np.int64), np.zeros(0, np.int32))
    # and the context still works afterwards
    crow, ccol, cval, cdiag = _run(ctx, rp, cc, val, diag, agg, na)
    _, _, wval, wdiag = oracle.galerkin(rp, cc, val, diag, agg, na, crow, ccol)
    assert np.array_equal(cval, wval) and np.array_equal(cdiag, wdiag)


def test_galerkin_on_the_gpu_hierarchy(ctx):
    # the whole setup on the GPU: aggregation, quotient graph, operator
    import torch
    rp, cc = graphs.grid3d_7pt(24, 23, 22)
    dev = torch.device("cuda", 0)
    val, diag = graphs.matrix_values(rp, cc, 4)
    agg, na = ctx.aggregate(rp, cc, 0)
    crow, ccol = ctx.quotient(rp, cc, agg, na)
    cval, cdiag = ctx.galerkin(rp, cc, torch.as_tensor(val, device=dev),
                               torch.as_tensor(diag, device=dev), agg, crow, ccol)
    a = agg.cpu().numpy()
    _, _, wval, wdiag = oracle.galerkin(rp, cc, val, diag, a, na, crow.cpu().numpy(),
                                        ccol.cpu().numpy())
    assert np.array_equal(cval.cpu().numpy(), wval) and np.array_equal(cdiag.cpu().numpy(), wdiag)


def test_galerkin_validated_stale_workspace_and_sizes():
    # a validating context, a workspace of 0xFF bytes before each call, and
    # graphs of growing and shrinking size on one context
    import torch
    from paper_2204_02934_amd import api
    c = api.Context(0, validate=True)
    dev = torch.device("cuda", 0)
    for name in ("grid2d", "chunglu_50k", "path101", "grid27_20", "star300"):
        rp, cc = GRAPHS[name]()
        val, diag = graphs.matrix_values(rp, cc, 7)
        agg, na = oracle.aggregate(rp, cc, 1)
        crow, ccol = oracle.quotient(rp, cc, agg, na)
        if c._ws is not None:
            c._ws.fill_(0xFF)
        cval, cdiag = c.galerkin(rp, cc, torch.as_tensor(val if val.size else np.zeros(1), device=dev),
                                 torch.as_tensor(diag, device=dev), agg, crow, ccol)
        _, _, wval, wdiag = oracle.galerkin(rp, cc, val, diag, agg, na, crow, ccol)
        assert np.array_equal(cval.cpu().numpy(), wval), name
        assert np.array_equal(cdiag.cpu().numpy(), wdiag), name
