"""GPU parity of Algorithm 2 (basic MIS-2 coarsening, mis2_aggregate_basic):
labels, aggregate count, root marks and the MIS-2's per-round sizes must
equal the CPU oracle's bit for bit."""
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


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _graphs():
    out = [("edgeless1", graphs.edgeless(1)), ("edgeless100", graphs.edgeless(100)),
           ("path2", graphs.path(2)), ("path101", graphs.path(101)), ("cycle64", graphs.cycle(64)),
           ("complete40", graphs.complete(40)), ("star70", graphs.star(70, 0)),
           ("star300", graphs.star(300, 17)), ("grid2d_ragged", graphs.grid2d_5pt(37, 29)),
           ("grid7_17", graphs.grid3d_7pt(17, 13, 11)), ("grid27_30", graphs.grid3d_27pt(30, 30, 30)),
           ("chunglu_50k", graphs.chung_lu(50000, 16.0, 2.1, 3000, seed=5)),
           ("dropped7_20", graphs.dropped_7pt(20, 0.1, seed=3)),
           ("union", graphs.disjoint_union([graphs.grid2d_5pt(10, 10), graphs.complete(9),
                                            graphs.edgeless(5), graphs.path(17)]))]
    rng = np.random.default_rng(19)
    for k in range(4):
        n = int(rng.integers(2, 3000))
        out.append(("er%d" % k, graphs.erdos_renyi(n, float(min(0.5, 8.0 / n)), seed=40 + k)))
    return out


GRAPHS = _graphs()


def _check(c, rp, cc, seed, name):
    agg, na, roots = c.aggregate_basic(rp, cc, seed, want_roots=True)
    d = oracle.aggregate_basic(rp, cc, seed, detail=True)
    assert na == d["n_agg"], (name, na, d["n_agg"])
    assert np.array_equal(roots.cpu().numpy(), d["roots"]), name
    assert np.array_equal(agg.cpu().numpy(), d["agg"]), name
    o = oracle.mis2_ex(rp, cc, seed)
    assert np.array_equal(c.last_trace(0), o["trace"][:, :2]), name


@pytest.mark.parametrize("name", [g[0] for g in GRAPHS])
def test_basic_parity(ctx, name):
    rp, cc = dict(GRAPHS)[name]
    _say("basic parity", name, rp.size - 1, int(rp[-1]))
    _check(ctx, rp, cc, 0, name)
    _check(ctx, rp, cc, 7, name)


@pytest.mark.parametrize("lanes", [-1, 1, 2, 8, 64])
def test_basic_lane_plans(api, lanes):
    # the join uses 4 lanes under the flat plan; chunglu_50k and star300 have
    # rows past every plan's whole-wavefront threshold
    for persistent in (False, True):
        c = api.Context(0, lanes=lanes, blocks=7, persistent=persistent)
        for name in ("chunglu_50k", "star300", "grid27_30", "er1"):
            rp, cc = dict(GRAPHS)[name]
            _check(c, rp, cc, 3, "%s L%d P%d" % (name, lanes, persistent))


def test_basic_empty_and_validated(api):
    c = api.Context(0, validate=True)
    agg, na = c.aggregate_basic(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert agg.numel() == 0 and na == 0
    rp, cc = graphs.grid2d_5pt(9, 9)
    _check(c, rp, cc, 0, "validated")


def test_basic_c2_full(ctx):
    rp, cc = graphs.grid3d_27pt(100, 100, 100)
    _say("basic C2", rp.size - 1, int(rp[-1]))
    _check(ctx, rp, cc, 0, "C2")


def test_basic_c3_full(ctx):
    rp, cc = graphs.chung_lu(4_000_000, 16.0, 2.1, 20000, seed=1)
    _say("basic C3", rp.size - 1, int(rp[-1]))
    _check(ctx, rp, cc, 0, "C3")
