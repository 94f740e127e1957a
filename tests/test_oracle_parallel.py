"""The OpenMP build of the oracle (used only to time it on every host core)
gives the sequential build's results bit for bit: the three phase loops of
Algorithm 1 it runs in parallel are pure maps (Section III-A)."""
import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs


@pytest.fixture(scope="module")
def omp_lib():
    try:
        return oracle.build_oracle(parallel=True)
    except Exception as e:  # pragma: no cover - a compiler without OpenMP
        pytest.skip("no OpenMP build: %s" % e)


GRAPHS = {
    "27pt": lambda: graphs.grid3d_27pt(24, 22, 20),
    "5pt": lambda: graphs.grid2d_5pt(150, 130),
    "chung_lu": lambda: graphs.chung_lu(30000, 16.0, 2.1, 2000, seed=7),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_parallel_oracle_identical(omp_lib, name, monkeypatch):
    rp, c = GRAPHS[name]()
    want = oracle.mis2_ex(rp, c, 3)
    want_agg = oracle.aggregate(rp, c, 3, detail=True)
    monkeypatch.setenv("OMP_NUM_THREADS", "4")
    with oracle.use_library(omp_lib):
        got = oracle.mis2_ex(rp, c, 3)
        got_agg = oracle.aggregate(rp, c, 3, detail=True)
    assert np.array_equal(got["status"], want["status"])
    assert got["n_iters"] == want["n_iters"]
    assert np.array_equal(got["trace"], want["trace"])
    assert np.array_equal(got_agg["agg"], want_agg["agg"])
    assert got_agg["n_agg"] == want_agg["n_agg"]
    assert np.array_equal(got_agg["trace2"], want_agg["trace2"])
