"""GPU checks of the compacted Refresh Column rows: a tuple that is OUT stays
OUT (Algorithm 1 never refreshes a decided vertex), so dropping OUT
neighbours from the long rows Refresh Column keeps cannot change any
minimum.  Results must equal the oracle's with and without compaction, and
the entries a compacting sweep visits must be exactly what the rewrite rule
leaves (counted here from the oracle's history)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs

pytestmark = pytest.mark.gpu

OUT = 0xFFFFFFFF
COMPACT_FROM = 2  # first round whose Refresh Column writes compacted rows (unmasked runs)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_02934_amd import api as a
    return a


GRAPHS = {
    "grid27_30": lambda: graphs.grid3d_27pt(30, 30, 30),
    "chunglu_50k": lambda: graphs.chung_lu(50000, 16.0, 2.1, 3000, seed=5),
    "dropped7_20": lambda: graphs.dropped_7pt(20, 0.1, seed=3),
    "grid2d_ragged": lambda: graphs.grid2d_5pt(37, 29),
    "star300": lambda: graphs.star(300, 17),
}


def _heavy_threshold(lanes):
    # rows longer than this are streamed by the whole wavefront (and only
    # those are rewritten in compacted form); -2: the staged sweeps' LDS slot
    if lanes == -2:
        return 32
    return 1024 if lanes >= 64 else 32 * lanes


def _mis2_matches(c, rp, cc, seed, name):
    st, nr, it = c.mis2(rp, cc, seed)
    o = oracle.mis2_ex(rp, cc, seed)
    assert np.array_equal(st.cpu().numpy(), o["status"]), name
    assert it == o["n_iters"], name
    assert np.array_equal(c.last_trace(0), o["trace"][:, :2]), name


def _agg_matches(c, rp, cc, seed, name):
    agg, na = c.aggregate(rp, cc, seed)
    oa, ona = oracle.aggregate(rp, cc, seed)
    assert na == ona and np.array_equal(agg.cpu().numpy(), oa), name


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_compaction_on_and_off_match_oracle(api, name):
    rp, cc = GRAPHS[name]()
    _say("compaction on/off", name, rp.size - 1, int(rp[-1]))
    # compaction runs only on graphs with rows past the cooperative
    # threshold (4 lanes per row here: 128 entries)
    long_rows = int(np.diff(rp).max()) > _heavy_threshold(4)
    on, off = api.Context(0, lanes=4), api.Context(0, lanes=4, compact=False)
    for seed in (0, 9):
        _mis2_matches(on, rp, cc, seed, name)
        rounds = len(on.last_trace(0))
        modes = [r["compact"] for r in on.last_sweeps() if r["kind"] == 0]
        assert modes == [0 if r < COMPACT_FROM or not long_rows else 1 if r == COMPACT_FROM
                         else 2 for r in range(rounds)], (name, modes)
        _mis2_matches(off, rp, cc, seed, name)
        assert all(r["compact"] == 0 for r in off.last_sweeps())
        _agg_matches(on, rp, cc, seed, name)
        # the phase-2 (masked) run compacts from its first round
        p2 = [r["compact"] for r in on.last_sweeps() if r["kind"] == 0 and r["phase"] == 1]
        assert p2 == ([1] + [2] * (len(p2) - 1) if p2 and long_rows else [0] * len(p2)), \
            (name, p2)
        _agg_matches(off, rp, cc, seed, name)


@pytest.mark.parametrize("lanes", [-2, 1, 2, 4, 8, 16, 64])
def test_compaction_every_lane_plan(api, lanes):
    # chunglu_50k has rows past every lane plan's cooperative threshold, so
    # the whole-wavefront rewrite of long rows runs too
    for persistent in (False, True):
        c = api.Context(0, lanes=lanes, blocks=7, persistent=persistent)
        for name in ("chunglu_50k", "grid27_30", "star300"):
            rp, cc = GRAPHS[name]()
            _mis2_matches(c, rp, cc, 4, "%s L%d P%d" % (name, lanes, persistent))
            _agg_matches(c, rp, cc, 4, "%s L%d P%d" % (name, lanes, persistent))


def test_flat_sweeps_do_not_compact(api):
    c = api.Context(0, lanes=-1)
    rp, cc = GRAPHS["grid27_30"]()
    _mis2_matches(c, rp, cc, 0, "flat")
    assert all(r["compact"] == 0 for r in c.last_sweeps())


def test_compaction_needs_workspace_room(api):
    import ctypes
    import torch
    from paper_2204_02934_amd import _lib
    rp, cc = GRAPHS["chunglu_50k"]()
    c = api.Context(0)
    n, nnz = rp.size - 1, int(rp[-1])
    small = c.workspace_bytes(n, _lib.MIS2_OP_MIS2)
    big = c.workspace_bytes(n, _lib.MIS2_OP_MIS2, nnz)
    assert big > small
    g, keep = c.graph(rp, cc)
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    o = oracle.mis2_ex(rp, cc, 0)
    for size, want in ((small, 0), (big, 2)):
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        assert c.lib.mis2_set_workspace(c.ptr, ctypes.c_void_p(ws.data_ptr()), size) == 0
        rc = c.lib.mis2_run(c.ptr, ctypes.byref(g), 0, ctypes.c_void_p(st.data_ptr()), None, None,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        assert np.array_equal(st.cpu().numpy(), o["status"])
        assert max(r["compact"] for r in c.last_sweeps()) == want
        assert c.lib.mis2_set_workspace(c.ptr, None, 0) == 0
        del ws


@pytest.mark.parametrize("lanes", [1, 4, -2])
@pytest.mark.parametrize("name", ["grid27_30", "chunglu_50k", "dropped7_20"])
def test_compacted_sweeps_visit_exactly_the_live_neighbours(api, name, lanes):
    # Refresh Column of round r reads, for each v of worklist2, the whole
    # CSR row unless the row is longer than the cooperative threshold and
    # r > COMPACT_FROM: then it reads the row as last rewritten, i.e. the
    # neighbours whose tuple was not OUT at the last Refresh Column that
    # found the row (as then stored) longer than the threshold.
    rp, cc = GRAPHS[name]()
    n = rp.size - 1
    thr = _heavy_threshold(lanes)
    o = oracle.mis2_ex(rp, cc, 0, history=64)
    assert o["n_iters"] <= 64
    T, M = o["T"], o["M"]
    deg = np.diff(rp).astype(np.int64)
    src = np.repeat(np.arange(n), deg)
    length = deg.copy()  # length of each row as the next sweep reads it
    want, wwant = [], []
    for r in range(o["n_iters"]):
        wl2 = np.ones(n, bool) if r == 0 else (M[r - 1] != OUT)
        want.append(int(length[wl2].sum()))
        wwant.append(0)
        if r >= COMPACT_FROM:
            live = np.bincount(src, weights=(T[r][cc] != OUT), minlength=n).astype(np.int64)
            rewrite = wl2 & (length > thr)
            length = np.where(rewrite, live, length)
            wwant[-1] = int(live[rewrite].sum())
    c = api.Context(0, account=True, lanes=lanes)
    c.mis2(rp, cc, 0)
    got = [r["edges"] for r in c.last_sweeps() if r["kind"] == 0]
    assert got == want, (name, got, want)
    written = [r["written"] for r in c.last_sweeps() if r["kind"] == 0]
    assert written == wwant, (name, written, wwant)
    # and the uncompacted run visits the whole rows of worklist2
    d = api.Context(0, account=True, compact=False, lanes=lanes)
    d.mis2(rp, cc, 0)
    full = [r["edges"] for r in d.last_sweeps() if r["kind"] == 0]
    assert full == [int(deg[np.ones(n, bool) if r == 0 else (M[r - 1] != OUT)].sum())
                    for r in range(o["n_iters"])]


@pytest.mark.parametrize("lanes", [4, -2])
def test_stale_workspace_contents_do_not_matter(api, lanes):
    # Lanes past a row's end must not gather through entries of the
    # compacted array that this run never wrote (here vertex 0's row, short,
    # so entry 0 keeps whatever the workspace held): fill the workspace with
    # 0xFF bytes (index -1) before each call.  A star after each random graph
    # supplies the long row that turns compaction on.
    from paper_2204_02934_amd import _lib
    rng = np.random.default_rng(9)
    gs = []
    for k in range(6):
        n = int(rng.integers(2, 3000))
        gs.append(graphs.disjoint_union([graphs.erdos_renyi(n, float(min(0.5, 8.0 / n)), seed=k),
                                         graphs.star(300, 5)]))
    gs.append(GRAPHS["chunglu_50k"]())
    c = api.Context(0, lanes=lanes)
    for i, (rp, cc) in enumerate(gs):
        n, nnz = rp.size - 1, int(rp[-1])
        c.ensure_workspace(n, _lib.MIS2_OP_AGGREGATE, nnz)
        c._ws.fill_(0xFF)
        _mis2_matches(c, rp, cc, 0, "stale %d" % i)
        assert max(r["compact"] for r in c.last_sweeps()) == 2
        c._ws.fill_(0xFF)
        _agg_matches(c, rp, cc, 0, "stale %d" % i)
