"""GPU parity of smoothed aggregation (mis2_smoothed): the prolongator
P = (I - omega D^-1 A) P_tent and the coarse operator P^T A P must equal the
CPU oracle's bit for bit (structure and values), on aggregations from the
oracle's Algorithm 3."""
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


CASES = {
    "grid2d_30x20": lambda: graphs.grid2d_5pt(30, 20),
    "grid27_14x13x12": lambda: graphs.grid3d_27pt(14, 13, 12),
    "grid7_20": lambda: graphs.grid3d_7pt(20, 20, 20),
    "chunglu_3000": lambda: graphs.chung_lu(3000, 8.0, 2.1, 300, seed=6),
    "union": lambda: graphs.disjoint_union([graphs.grid2d_5pt(9, 7), graphs.path(40),
                                            graphs.star(30, 2), graphs.complete(12)]),
    "edgeless40": lambda: graphs.edgeless(40),
    "complete20": lambda: graphs.complete(20),
}


def _check(ctx, rp, c, omega, seed, name):
    import torch
    dev = torch.device("cuda", 0)
    val, diag = graphs.matrix_values(rp, c, seed, shift=0.25)
    agg, na = oracle.aggregate(rp, c, 0)
    want = oracle.smoothed(rp, c, val, diag, agg, na, omega)
    (prow, pcol, pval), (crow, ccol, cval) = ctx.smoothed(
        rp, c, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
        agg, na, omega)
    got = [x.cpu().numpy() for x in (prow, pcol, pval, crow, ccol, cval)]
    for k, (g, w) in enumerate(zip(got, want)):
        assert g.shape == w.shape and np.array_equal(g, w), (name, k)
    return want


@pytest.mark.parametrize("omega", [2.0 / 3.0, 1.0])
@pytest.mark.parametrize("name", sorted(CASES))
def test_smoothed_matches_oracle(ctx, name, omega):
    rp, c = CASES[name]()
    _say("smoothed", name, rp.size - 1, omega)
    _check(ctx, rp, c, omega, 4, name)


def test_smoothed_27pt_40cube(ctx):
    rp, c = graphs.grid3d_27pt(40, 40, 40)
    w = _check(ctx, rp, c, 2.0 / 3.0, 1, "27-point 40^3")
    _say("27-point 40^3: P %d entries, coarse operator %d rows %d entries"
         % (w[1].size, w[3].size - 1, w[4].size))


def test_smoothed_rows_past_the_small_set(ctx):
    # a hub with 600 spokes of three vertices, each spoke its own aggregate:
    # the hub's row of P, the rows of A P next to it and the hub aggregate's
    # row of P^T A P hold more than 256 columns (the first, small-set pass
    # leaves them to the second); the other rows are small
    import torch
    k = 600
    u = np.concatenate([np.zeros(k, np.int64), 1 + 3 * np.arange(k), 2 + 3 * np.arange(k)])
    w = np.concatenate([1 + 3 * np.arange(k), 2 + 3 * np.arange(k), 3 + 3 * np.arange(k)])
    rp, c = graphs.from_edges(1 + 3 * k, u, w)
    agg = np.zeros(1 + 3 * k, np.int32)
    agg[1:] = 1 + np.repeat(np.arange(k), 3)
    na = k + 1
    val, diag = graphs.matrix_values(rp, c, 9, shift=0.25)
    want = oracle.smoothed(rp, c, val, diag, agg, na, 2.0 / 3.0)
    prow, pcol = want[0], want[1]
    assert prow[1] - prow[0] > 256  # the hub's row of P
    dev = torch.device("cuda", 0)
    (gp, gc, gv), (hp, hc, hv) = ctx.smoothed(rp, c, torch.as_tensor(val, device=dev),
                                              torch.as_tensor(diag, device=dev), agg, na,
                                              2.0 / 3.0)
    got = [x.cpu().numpy() for x in (gp, gc, gv, hp, hc, hv)]
    for i, (g, x) in enumerate(zip(got, want)):
        assert g.shape == x.shape and np.array_equal(g, x), i


def test_smoothed_rejects_labels_out_of_range(ctx):
    import torch
    from paper_2204_02934_amd._lib import Mis2Error
    rp, c = graphs.grid2d_5pt(10, 10)
    dev = torch.device("cuda", 0)
    val, diag = graphs.matrix_values(rp, c, 0)
    agg, na = oracle.aggregate(rp, c, 0)
    bad = agg.copy()
    bad[17] = na  # one past the last aggregate
    with pytest.raises(Mis2Error):
        ctx.smoothed(rp, c, torch.as_tensor(val, device=dev), torch.as_tensor(diag, device=dev),
                     bad, na, 0.5)
    # the context still works afterwards
    _check(ctx, rp, c, 0.5, 0, "after the error")
