"""GPU parity of mis2_run_ablation (Algorithm 1 with the optimizations of
Section V taken away, Fig. 2 and Table I): for every combination of flags,
status, round count and per-round worklist sizes equal the oracle's with the
same priority choice.  Worklists, tuple packing and lanes per row change
the work done, not the result (nor the per-round sizes)."""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs

pytestmark = pytest.mark.gpu

FIXED, XOR, NOWL, UNPACKED, ONE_LANE, SIMPLE = 1, 2, 4, 8, 16, 32


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_02934_amd import api
    return api.Context(0)


def _pflags(flags):
    return (oracle.PRIO_FIXED if flags & FIXED else 0) | (oracle.PRIO_XORSHIFT if flags & XOR else 0)


GRAPHS = {
    "grid27_20": lambda: graphs.grid3d_27pt(20, 19, 18),
    "chunglu_20k": lambda: graphs.chung_lu(20000, 12.0, 2.1, 1500, seed=6),
    "star300": lambda: graphs.star(300, 17),
    "path101": lambda: graphs.path(101),
    "edgeless50": lambda: graphs.edgeless(50),
    "er": lambda: graphs.erdos_renyi(1700, 0.004, seed=12),
    "union": lambda: graphs.disjoint_union([graphs.grid2d_5pt(10, 10), graphs.complete(9),
                                            graphs.edgeless(5), graphs.path(17)]),
}


def _check(ctx, rp, cc, seed, flags, name):
    st, nr, it = ctx.mis2_ablation(rp, cc, seed, flags)
    ost, oit, otr = oracle.mis2_ablation(rp, cc, seed, _pflags(flags))
    assert np.array_equal(st.cpu().numpy(), ost), (name, flags)
    assert it == oit and nr == int(ost.sum()), (name, flags, it, oit)
    assert np.array_equal(ctx.last_trace(0), otr[:, :2]), (name, flags)


ALL_FLAG_SETS = [sum(c) for k in range(0, 6) for c in itertools.combinations(
    (FIXED, XOR, NOWL, UNPACKED, ONE_LANE, SIMPLE), k)]


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_ablation_every_flag_combination(ctx, name):
    rp, cc = GRAPHS[name]()
    _say("ablation", name, rp.size - 1, int(rp[-1]))
    for flags in ALL_FLAG_SETS:
        _check(ctx, rp, cc, 3, flags, name)


def test_ablation_empty_graph(ctx):
    st, nr, it = ctx.mis2_ablation(np.zeros(1, np.int64), np.zeros(0, np.int32), 0,
                                   FIXED | NOWL | UNPACKED)
    assert st.numel() == 0 and nr == 0 and it == 0


def test_ablation_rejects_unknown_flags(ctx):
    from paper_2204_02934_amd._lib import Mis2Error
    rp, cc = graphs.path(10)
    with pytest.raises(Mis2Error):
        ctx.mis2_ablation(rp, cc, 0, 64)


@pytest.mark.parametrize("flags", [FIXED | NOWL | UNPACKED, NOWL | UNPACKED, UNPACKED, SIMPLE,
                                   ONE_LANE, XOR])
def test_ablation_ladder_on_the_27_point_100_cube(ctx, flags):
    rp, cc = graphs.grid3d_27pt(100, 100, 100)
    _say("ablation C2 flags", flags)
    _check(ctx, rp, cc, 0, flags, "C2")
