"""Pins of the CPU oracle's MIS-2 aggregation (Algorithm 3, Section III-B) and
of the quotient graph / multilevel loop, by brute force from definitions."""
import numpy as np
import pytest

import oracle
from bruteforce import (adjacency, check_aggregation, check_mis2, luby_g2_hashed,
                        quotient_pairs)
from paper_2204_02934_amd import graphs


def _check(rp, c, seed=0):
    d = oracle.aggregate(rp, c, seed, detail=True)
    n = rp.size - 1
    roots1 = [int(v) for v in np.nonzero(d["roots"] == 1)[0]]
    roots2 = [int(v) for v in np.nonzero(d["roots"] == 2)[0]]
    # phase 1 roots: exactly the MIS-2 of G (brute force)
    want1, it1 = luby_g2_hashed(rp, c, seed)
    assert roots1 == want1 and d["iters1"] == it1
    # phase 2: MIS-2 of the subgraph induced by vertices outside phase-1
    # aggregates, same ids and iteration restarted at 0; accepted roots are
    # those with >= 2 unaggregated neighbours
    adj = adjacency(rp, c)
    lab1 = np.full(n, -1)
    for r in roots1:
        for u in adj[r] | {r}:
            lab1[u] = 1
    active = [bool(lab1[v] == -1) for v in range(n)]
    if any(active):
        m2, it2 = luby_g2_hashed(rp, c, seed, active=active)
    else:
        m2, it2 = [], 0
    assert d["m2"] == len(m2) and d["iters2"] == it2
    acc = [r for r in m2 if sum(1 for u in adj[r] if active[u]) >= 2]
    assert roots2 == acc
    err = check_aggregation(rp, c, d["agg"], d["n_agg"], roots1, roots2)
    assert err is None, err
    assert d["n_agg"] == len(roots1) + len(roots2)
    return d


def test_aggregate_small_random_graphs():
    rng = np.random.default_rng(3)
    for trial in range(120):
        n = int(rng.integers(1, 45))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.03, 0.35)), seed=500 + trial)
        _check(rp, c, seed=trial % 3)


def test_aggregate_structured():
    for rp, c in [graphs.grid2d_5pt(13, 11), graphs.grid3d_7pt(6, 5, 4),
                  graphs.grid3d_27pt(5, 5, 5), graphs.path(37), graphs.cycle(29),
                  graphs.dropped_7pt(6, 0.1, seed=1)]:
        d = _check(rp, c)
        assert d["joined"] + d["n1"] + d["n2"] <= rp.size - 1


def test_aggregate_power_law():
    rp, c = graphs.chung_lu(400, 6.0, 2.1, 80, seed=9)
    _check(rp, c, seed=1)


def test_aggregate_phase2_and_phase3_exercised():
    # a long path forces all three phases: spacing leaves gaps for phase 2
    # roots and for phase-3 joins
    seen = {"n2": 0, "joined": 0}
    for n in range(20, 120, 7):
        rp, c = graphs.path(n)
        d = _check(rp, c)
        seen["n2"] += d["n2"]
        seen["joined"] += d["joined"]
    rp, c = graphs.grid2d_5pt(30, 30)
    d = _check(rp, c)
    seen["n2"] += d["n2"]
    seen["joined"] += d["joined"]
    assert seen["n2"] > 0 and seen["joined"] > 0


@pytest.mark.parametrize("n", [1, 2, 6, 25])
def test_aggregate_complete_and_star(n):
    for rp, c in [graphs.complete(n), graphs.star(n, 0), graphs.star(n, n - 1)]:
        agg, na = oracle.aggregate(rp, c, 0)
        assert na == 1 and np.all(agg == 0)


@pytest.mark.parametrize("n", [0, 1, 9])
def test_aggregate_edgeless(n):
    rp, c = graphs.edgeless(n)
    agg, na = oracle.aggregate(rp, c, 0)
    assert na == n and list(agg) == list(range(n))


def test_aggregate_phase1_covers_mis2_neighbourhoods_on_grid():
    rp, c = graphs.grid2d_5pt(64, 64)
    d = oracle.aggregate(rp, c, 0, detail=True)
    st, _ = oracle.mis2(rp, c, 0)
    assert np.array_equal(d["roots"] == 1, st.astype(bool))
    assert check_mis2(adjacency(rp, c), list(np.nonzero(st)[0])) is None


def test_quotient_bruteforce():
    rng = np.random.default_rng(4)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.02, 0.3)), seed=trial)
        agg, na = oracle.aggregate(rp, c, 0)
        crp, cc = oracle.quotient(rp, c, agg, na)
        pairs = quotient_pairs(rp, c, agg)
        got = set()
        for a in range(na):
            row = list(cc[crp[a]:crp[a + 1]])
            assert row == sorted(set(row))          # ascending, no duplicates
            assert a not in row                      # no self-loops
            got |= {(a, int(x)) for x in row}
        assert got == pairs
        assert all((y, x) in got for x, y in got)   # symmetric


def test_quotient_of_grid_aggregates_is_connected_and_smaller():
    rp, c = graphs.grid3d_7pt(12, 12, 12)
    agg, na = oracle.aggregate(rp, c, 0)
    crp, cc = oracle.quotient(rp, c, agg, na)
    assert crp.size - 1 == na < rp.size - 1
    # breadth-first search over the coarse graph reaches every aggregate
    seen = {0}
    stack = [0]
    while stack:
        a = stack.pop()
        for x in cc[crp[a]:crp[a + 1]]:
            if int(x) not in seen:
                seen.add(int(x))
                stack.append(int(x))
    assert len(seen) == na


def test_coarsen_levels():
    rp, c = graphs.grid3d_7pt(20, 20, 20)
    levels = oracle.coarsen(rp, c, 0, stop_below=100)
    ns = [lv["n"] for lv in levels]
    assert ns[0] == 8000 and all(a > b for a, b in zip(ns, ns[1:]))
    assert levels[-1]["n_agg"] < 100 or levels[-1]["n_agg"] == levels[-1]["n"]
    for lv in levels:
        assert lv["n"] >= 100
    # each level's input is the previous level's quotient graph
    g = (rp, c)
    for lv in levels:
        assert g[0].size - 1 == lv["n"]
        g = oracle.quotient(g[0], g[1], lv["agg"], lv["n_agg"])


def test_coarsen_stops_without_progress():
    rp, c = graphs.edgeless(2000)
    levels = oracle.coarsen(rp, c, 0, stop_below=1000)
    assert len(levels) == 1 and levels[0]["n_agg"] == 2000


def test_coarsen_below_threshold_does_nothing():
    rp, c = graphs.grid2d_5pt(20, 20)
    assert oracle.coarsen(rp, c, 0, stop_below=1000) == []
