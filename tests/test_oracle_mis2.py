"""Pins of the CPU oracle's MIS-2 (Algorithm 1) against what the paper and the
mathematics fix: the Fig. 1 worked example, brute-force Luby on G^2
(Section IV, Lemma 2), the definitions (Section I), packing (Section V-C,
Eq. 1), closed-form special cases and Table III (soft)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from bruteforce import (adjacency, check_mis2, luby_g2, luby_g2_hashed, nbits,
                        prio_hash, tuple_of, within2)
from paper_2204_02934_amd import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- hash, packing
def test_xorshift_star_definition():
    # Section V-A: f is xorshift followed by a multiplicative LCG step; the
    # multiplier is Vigna's published constant, in both of its published forms.
    assert 0x2545F4914F6CDD1D == 2685821657736338717
    assert oracle.xorshift64star(0) == 0  # a zero state stays zero
    rng = np.random.default_rng(5)
    for x in rng.integers(0, 2**63, 200, dtype=np.uint64):
        x = int(x) * 2 + 1
        y = oracle.xorshift64star(x)
        # the multiplication is invertible modulo 2^64 (odd multiplier): undo it
        inv = pow(2685821657736338717, -1, 2**64)
        z = (y * inv) % 2**64
        # and each xorshift step is invertible: undo x ^= x >> 27, x ^= x << 25, x ^= x >> 12
        def unshr(v, s):
            r = v
            for _ in range(64 // s + 1):
                r = v ^ (r >> s)
            return r
        def unshl(v, s):
            r = v
            for _ in range(64 // s + 1):
                r = v ^ ((r << s) % 2**64)
            return r
        assert unshr(unshl(unshr(z, 27), 25), 12) == x


def test_hash_symmetric_and_seed_zero():
    # h(i, v) = f(f(i) xor f(v)) is symmetric in its arguments at seed 0
    for i, v in [(0, 1), (3, 7), (12345, 99), (2**40, 5)]:
        assert oracle.hash_priority(0, i, v) == oracle.hash_priority(0, v, i)
    # round 0 at seed 0: f(f(0) xor f(v)) = f(f(v))
    for v in range(50):
        assert oracle.hash_priority(0, 0, v) == oracle.xorshift64star(oracle.xorshift64star(v))
    # the seed enters as (seed << 32) xor iter
    assert oracle.hash_priority(3, 5, 11) == oracle.hash_priority(0, (3 << 32) ^ 5, 11)


def test_hash_matches_independent_python():
    rng = np.random.default_rng(0)
    for _ in range(300):
        s, i, v = (int(x) for x in rng.integers(0, 2**31, 3))
        assert oracle.hash_priority(s, i, v) == prio_hash(s, i, v)


@pytest.mark.parametrize("k", range(2, 31))
def test_id_bits_powers_of_two(k):
    # Eq. (1): b is the smallest integer with 2^b >= |V| + 2
    assert oracle.id_bits(2**k - 2) == k
    assert oracle.id_bits(2**k - 1) == k + 1
    assert oracle.id_bits(2**k) == k + 1
    assert oracle.id_bits(2**k - 3) == k


@pytest.mark.parametrize("b", range(1, 13))
def test_pack_exhaustive_small_b(b):
    # Section V-C: packed tuples are injective, ordered like (priority, id)
    # and never equal IN (0) or OUT (0xFFFFFFFF).  Exhaustive over ids and a
    # priority set that spans the field, including its extremes.
    n = 2**b - 2  # the largest |V| with this b
    pb = 32 - b
    prios = sorted(set([0, 1, 2, 3, (1 << pb) - 2, (1 << pb) - 1] +
                       [int(x) for x in np.random.default_rng(b).integers(0, 1 << pb, 30)]))
    vals = {}
    for p in prios:
        for v in range(n):
            t = oracle.pack(p, v, b)
            assert t not in (0, 0xFFFFFFFF)
            assert (p, v) not in vals
            vals[(p, v)] = t
    keys = sorted(vals)
    packed = [vals[k] for k in keys]
    assert packed == sorted(packed) and len(set(packed)) == len(packed)
    # the priority is taken modulo 2^(32-b): high hash bits are dropped
    assert oracle.pack((1 << pb) + 5, 3, b) == oracle.pack(5, 3, b)


def test_pack_no_priority_bits():
    assert oracle.pack(12345, 7, 32) == 8


# ----------------------------------------------------------------- Fig. 1
def _fig1():
    with open(os.path.join(GOLDEN, "fig1.json")) as f:
        return json.load(f)


def test_fig1_worked_example():
    g = _fig1()
    n = g["n"]
    e = np.array(g["edges"]) - 1
    rp, c = graphs.from_edges(n, e[:, 0], e[:, 1])
    b = oracle.id_bits(n)
    prio = np.zeros((len(g["rounds"]), n), np.uint64)
    for r, rd in enumerate(g["rounds"]):
        for lab, (p, idv) in rd["refresh_row"].items():
            assert int(lab) == idv
            prio[r, int(lab) - 1] = p
    o = oracle.mis2_ex(rp, c, prio=prio, history=4)
    assert o["n_iters"] == g["iterations"]
    assert sorted(np.nonzero(o["status"])[0] + 1) == g["result"]

    def unpack(t):
        if t == 0xFFFFFFFF:
            return "OUT"
        if t == 0:
            return "IN"
        return [t >> b, t & ((1 << b) - 1)]

    for r, rd in enumerate(g["rounds"]):
        for lab, want in rd["refresh_row"].items():
            assert unpack(int(o["T"][r, int(lab) - 1])) == want
        for lab, want in rd["refresh_column"].items():
            assert unpack(int(o["M"][r, int(lab) - 1])) == want, (r, lab)
        for lab in rd["decide_in"]:
            assert o["D"][r, lab - 1] == 0
        for lab in rd["decide_out"]:
            assert o["D"][r, lab - 1] == 0xFFFFFFFF
        decided_now = set(rd["decide_in"]) | set(rd["decide_out"])
        for lab in rd["refresh_row"]:
            if int(lab) not in decided_now:
                assert o["D"][r, int(lab) - 1] not in (0, 0xFFFFFFFF)


def test_fig1_open_neighbourhood_would_differ():
    # The figure fixes the closed-neighbourhood reading: with adj(v) open,
    # vertex 1 would see only (3,2) and M_1 would not be (1,1).
    g = _fig1()
    t = {int(k): tuple(v) for k, v in g["rounds"][0]["refresh_row"].items()}
    m1 = tuple(g["rounds"][0]["refresh_column"]["1"])
    assert t[2] != m1 and min(t[1], t[2]) == m1


# ----------------------------------------------------------------- brute force
def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        if es:
            u, v = zip(*es)
        else:
            u, v = [], []
        yield graphs.from_edges(n, list(u), list(v))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_bruteforce_all_small_graphs(n):
    for rp, c in _all_graphs(n):
        for seed in (0, 1):
            st, it = oracle.mis2(rp, c, seed)
            want, rounds = luby_g2_hashed(rp, c, seed)
            assert list(np.nonzero(st)[0]) == want
            assert it == rounds


def test_bruteforce_six_vertex_sample():
    gen = _all_graphs(6)
    for k, (rp, c) in enumerate(gen):
        if k % 7:
            continue
        st, it = oracle.mis2(rp, c, 0)
        want, rounds = luby_g2_hashed(rp, c, 0)
        assert list(np.nonzero(st)[0]) == want and it == rounds


def test_bruteforce_injected_priorities_with_ties_in_priority():
    # Narrow random priorities (many equal priorities): the id breaks ties.
    rng = np.random.default_rng(11)
    for trial in range(150):
        n = int(rng.integers(2, 25))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.05, 0.5)), seed=trial)
        prio = rng.integers(0, 4, size=(64, n)).astype(np.uint64)
        o = oracle.mis2_ex(rp, c, prio=prio)
        adj = adjacency(rp, c)
        want, rounds = luby_g2(n, adj, lambda r, v: (int(prio[r, v]), v))
        assert list(np.nonzero(o["status"])[0]) == want
        assert o["n_iters"] == rounds


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_random_graphs(seed):
    rng = np.random.default_rng(100 + seed)
    for trial in range(25):
        n = int(rng.integers(7, 41))
        p = float(rng.uniform(0.02, 0.4))
        rp, c = graphs.erdos_renyi(n, p, seed=1000 * seed + trial)
        st, it = oracle.mis2(rp, c, seed)
        want, rounds = luby_g2_hashed(rp, c, seed)
        assert list(np.nonzero(st)[0]) == want
        assert it == rounds


def test_bruteforce_induced_subgraph():
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(3, 35))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.05, 0.4)), seed=trial)
        active = (rng.random(n) < 0.6).astype(np.uint8)
        o = oracle.mis2_ex(rp, c, seed=0, active=active)
        want, rounds = luby_g2_hashed(rp, c, 0, active=list(active.astype(bool)))
        assert list(np.nonzero(o["status"])[0]) == want
        assert o["n_iters"] == rounds
        assert check_mis2(adjacency(rp, c), want, list(active.astype(bool))) is None


def test_validity_medium_graphs():
    for k, (rp, c) in enumerate([graphs.erdos_renyi(300, 0.02, 1),
                                 graphs.random_regular_ish(800, 6, 2),
                                 graphs.grid2d_5pt(23, 17),
                                 graphs.grid3d_27pt(7, 6, 5),
                                 graphs.chung_lu(2000, 8.0, 2.1, 300, seed=3)]):
        st, _ = oracle.mis2(rp, c, k)
        assert check_mis2(adjacency(rp, c), list(np.nonzero(st)[0])) is None


# ----------------------------------------------------------------- special cases
@pytest.mark.parametrize("n", [1, 2, 5, 30])
def test_complete_graph_single_root(n):
    rp, c = graphs.complete(n)
    st, it = oracle.mis2(rp, c, 0)
    b = nbits(n)
    t0 = [tuple_of(prio_hash(0, 0, v), v, n) for v in range(n)]
    assert list(np.nonzero(st)[0]) == [int(np.argmin([t[0] * 2**b + t[1] for t in t0]))]
    assert it == (1 if n == 1 else 2)


@pytest.mark.parametrize("n", [2, 3, 9, 40])
def test_star_single_root(n):
    for center in (0, n - 1):
        rp, c = graphs.star(n, center)
        st, _ = oracle.mis2(rp, c, 0)
        assert st.sum() == 1


@pytest.mark.parametrize("n", [0, 1, 7, 100])
def test_edgeless_all_in_one_round(n):
    rp, c = graphs.edgeless(n)
    st, it = oracle.mis2(rp, c, 0)
    assert st.sum() == n
    assert it == (1 if n else 0)


@pytest.mark.parametrize("n", list(range(1, 30)) + [200, 1001])
def test_path_bounds(n):
    rp, c = graphs.path(n)
    st, _ = oracle.mis2(rp, c, 0)
    k = int(st.sum())
    # each member covers at most 5 path vertices within distance 2, and members
    # are at least 3 apart
    assert -(-n // 5) <= k <= -(-n // 3)
    if n <= 3:
        assert k == 1


def test_grid_density_bounds():
    rp, c = graphs.grid2d_5pt(64, 64)
    k = int(oracle.mis2(rp, c, 0)[0].sum())
    assert 4096 / 13 <= k <= 4096 / 5 + 64
    rp, c = graphs.grid3d_27pt(20, 20, 20)
    k = int(oracle.mis2(rp, c, 0)[0].sum())
    assert 8000 / 125 <= k <= 8000 / 27 + 3 * 20 * 20


def test_disjoint_union_equals_masked_components():
    parts = [graphs.erdos_renyi(40, 0.1, 1), graphs.grid2d_5pt(6, 7), graphs.path(13)]
    rp, c = graphs.disjoint_union(parts)
    n = rp.size - 1
    whole = oracle.mis2_ex(rp, c, seed=4)
    acc = np.zeros(n, np.uint8)
    iters = 0
    off = 0
    for prp, _ in parts:
        m = prp.size - 1
        act = np.zeros(n, np.uint8)
        act[off:off + m] = 1
        o = oracle.mis2_ex(rp, c, seed=4, active=act)
        acc |= o["status"]
        iters = max(iters, o["n_iters"])
        off += m
    assert np.array_equal(acc, whole["status"])
    assert iters == whole["n_iters"]


def test_worklist_invariants_on_trace():
    rp, c = graphs.grid3d_27pt(12, 11, 10)
    o = oracle.mis2_ex(rp, c, seed=0)
    tr = o["trace"]
    assert tr[0, 0] == tr[0, 1] == rp.size - 1
    assert tr[0, 2] == tr[0, 3] == rp[-1]
    assert np.all(np.diff(tr[:, 0]) < 0)      # every round decides something
    assert np.all(np.diff(tr[:, 1]) <= 0)
    assert np.all(tr[:, 0] <= tr[:, 1])       # worklist1 stays inside worklist2


def test_worklist_free_equivalence():
    """Worklists only avoid work (Section V-B): recomputing every vertex in
    every round, with numpy, gives the same set and round count."""
    OUT = np.uint32(0xFFFFFFFF)
    for rp, c in [graphs.grid3d_7pt(15, 14, 13), graphs.chung_lu(3000, 10.0, 2.1, 400, seed=8)]:
        n = rp.size - 1
        b = nbits(n)
        deg = np.diff(rp)
        starts = rp[:-1] + np.arange(n)
        cc = np.empty(rp[-1] + n, np.int64)
        cc[starts] = np.arange(n)
        m = np.ones(cc.size, bool)
        m[starts] = False
        cc[m] = c
        T = np.zeros(n, np.uint32)
        und = np.ones(n, bool)
        r = 0
        while und.any():
            for v in np.nonzero(und)[0]:
                p, _ = tuple_of(prio_hash(0, r, int(v)), int(v), n)
                T[v] = (p << b) | (int(v) + 1)
            M = np.minimum.reduceat(T[cc], starts)
            M[M == 0] = OUT
            g = M[cc]
            anyout = np.logical_or.reduceat(g == OUT, starts)
            alleq = np.logical_and.reduceat(g == np.repeat(T, deg + 1), starts)
            T = np.where(und & anyout, OUT, np.where(und & ~anyout & alleq, 0, T)).astype(np.uint32)
            und = (T != 0) & (T != OUT)
            r += 1
        st, it = oracle.mis2(rp, c, 0)
        assert np.array_equal(st.astype(bool), T == 0) and it == r


def test_seed_changes_result_deterministically():
    rp, c = graphs.grid2d_5pt(40, 40)
    a0, _ = oracle.mis2(rp, c, 0)
    a0b, _ = oracle.mis2(rp, c, 0)
    a1, _ = oracle.mis2(rp, c, 1)
    assert np.array_equal(a0, a0b)
    assert not np.array_equal(a0, a1)


# ----------------------------------------------------------------- Table III (soft)
def test_table3_soft():
    with open(os.path.join(GOLDEN, "table3.json")) as f:
        t = json.load(f)
    for row in t["rows"]:
        nx, ny, nz = row["grid"]
        if nx * ny * nz > 250000:
            continue  # the large rows run in the slow test below
        gen = graphs.grid3d_7pt if row["problem"] == "laplace" else graphs.elasticity3d
        rp, c = gen(nx, ny, nz)
        assert rp.size - 1 == row["n"]
        st, it = oracle.mis2(rp, c, 0)
        assert abs(int(st.sum()) - row["mis2"]) <= 0.05 * row["mis2"]
        assert abs(it - row["iters"]) <= 2


@pytest.mark.slow
def test_table3_soft_large():
    with open(os.path.join(GOLDEN, "table3.json")) as f:
        t = json.load(f)
    for row in t["rows"]:
        nx, ny, nz = row["grid"]
        if nx * ny * nz <= 250000:
            continue
        gen = graphs.grid3d_7pt if row["problem"] == "laplace" else graphs.elasticity3d
        rp, c = gen(nx, ny, nz)
        st, it = oracle.mis2(rp, c, 0)
        assert abs(int(st.sum()) - row["mis2"]) <= 0.05 * row["mis2"]
        assert abs(it - row["iters"]) <= 2


def test_within2_helper_sanity():
    rp, c = graphs.path(5)
    adj = adjacency(rp, c)
    assert within2(adj, 0) == {1, 2}
    assert within2(adj, 2) == {0, 1, 3, 4}
