"""Pins of the CPU oracle's basic MIS-2 coarsening (Algorithm 2, Section
III-B), by brute force from the algorithm's statement: the roots are the
MIS-2 of Luby's algorithm on G^2, each root's closed neighbourhood is one
aggregate, and every other vertex joins the smallest-id aggregate holding
one of its neighbours (the reading of "any neighbour")."""
import numpy as np

import oracle
from bruteforce import adjacency, check_basic_coarsening, luby_g2_hashed
from paper_2204_02934_amd import graphs


def _check(rp, c, seed=0):
    d = oracle.aggregate_basic(rp, c, seed, detail=True)
    roots = [int(v) for v in np.nonzero(d["roots"])[0]]
    want, _ = luby_g2_hashed(rp, c, seed)
    assert roots == want
    err = check_basic_coarsening(rp, c, d["agg"], d["n_agg"], roots)
    assert err is None, err
    return d


def test_basic_small_random_graphs():
    rng = np.random.default_rng(13)
    joined = 0
    for trial in range(120):
        n = int(rng.integers(1, 45))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.03, 0.35)), seed=900 + trial)
        joined += _check(rp, c, seed=trial % 3)["joined"]
    assert joined > 0  # the second loop ran


def test_basic_structured_and_power_law():
    for rp, c in [graphs.grid2d_5pt(13, 11), graphs.grid3d_7pt(6, 5, 4),
                  graphs.grid3d_27pt(5, 5, 5), graphs.path(37), graphs.cycle(29),
                  graphs.dropped_7pt(6, 0.1, seed=1), graphs.chung_lu(400, 6.0, 2.1, 80, seed=9)]:
        d = _check(rp, c)
        assert d["n_agg"] >= 1


def test_basic_special_cases():
    # complete graph and star: one root, one aggregate
    for rp, c in [graphs.complete(17), graphs.star(30, 0), graphs.star(30, 11)]:
        agg, na = oracle.aggregate_basic(rp, c)
        assert na == 1 and not agg.any()
    # edgeless: every vertex is its own aggregate
    agg, na = oracle.aggregate_basic(*graphs.edgeless(9))
    assert na == 9 and list(agg) == list(range(9))
    # empty graph
    agg, na = oracle.aggregate_basic(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert na == 0 and agg.size == 0


def test_basic_first_loop_is_phase_one_of_algorithm_3():
    # both algorithms start from the same MIS-2 and the same root numbering,
    # so the vertices aggregated in Algorithm 3's phase 1 carry the same
    # labels in both
    for rp, c in [graphs.grid2d_5pt(20, 17), graphs.chung_lu(600, 8.0, 2.1, 90, seed=4),
                  graphs.path(101)]:
        b = oracle.aggregate_basic(rp, c, 2, detail=True)
        a = oracle.aggregate(rp, c, 2, detail=True)
        assert np.array_equal(b["roots"], (a["roots"] == 1).astype(np.uint8))
        adj = adjacency(rp, c)
        first = np.zeros(rp.size - 1, bool)  # closed neighbourhoods of the roots
        for r in np.nonzero(b["roots"])[0]:
            first[list(adj[int(r)] | {int(r)})] = True
        assert np.array_equal(b["agg"][first], a["agg"][first])
        assert b["n_agg"] == a["n1"]
