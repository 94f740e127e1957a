"""GPU test of mis2_run_noalloc, the MIS-2 entry point that allocates nothing
(its workspace is the library's static device scratch): called through the C
ABI, its status, root count and round count must equal mis2_run's bit for
bit, on calls in a row with shrinking inputs (the scratch keeps the previous
call's contents)."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2204_02934_amd import graphs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_02934_amd import _lib, api
    return torch, _lib, api


def _device_graph(torch, api, g):
    rp, c = api.as_device_csr(g[0], g[1], torch.device("cuda", 0))
    return rp, c, int(g[0][-1])


def test_noalloc_equals_mis2_run_on_calls_in_a_row(env):
    torch, _lib, api = env
    ctx = api.Context(0)
    cases = [
        ("27-point 60x50x40", graphs.grid3d_27pt(60, 50, 40)),
        ("5-point 50x50 (smaller)", graphs.grid2d_5pt(50, 50)),
        ("Chung-Lu 30000, hubs", graphs.chung_lu(30000, 16.0, 2.1, 3000, seed=5)),
        ("path 7 (smaller again)", graphs.path(7)),
    ]
    for name, g in cases:
        rp, c, nnz = _device_graph(torch, api, g)
        n = rp.numel() - 1
        _say("noalloc vs mis2_run: %s n=%d nnz=%d" % (name, n, nnz))
        want, nr_w, ni_w = ctx.mis2(rp, c, seed=3, nnz=nnz)
        status = torch.full((n,), 0xAB, dtype=torch.uint8, device=rp.device)
        nr, ni = ctx.mis2_noalloc(rp, c, status, seed=3, nnz=nnz)
        torch.cuda.synchronize()
        assert (nr, ni) == (nr_w, ni_w), name
        assert torch.equal(status, want), name


def test_noalloc_repeat_is_identical(env):
    torch, _lib, api = env
    ctx = api.Context(0)
    rp, c, nnz = _device_graph(torch, api, graphs.grid3d_7pt(40, 40, 40))
    n = rp.numel() - 1
    outs = []
    for _ in range(3):
        st = torch.zeros(n, dtype=torch.uint8, device=rp.device)
        outs.append((ctx.mis2_noalloc(rp, c, st, seed=0, nnz=nnz), st))
    for (k, st) in outs[1:]:
        assert k == outs[0][0] and torch.equal(st, outs[0][1])


def test_noalloc_rejects_sizes_beyond_the_scratch(env):
    torch, _lib, api = env
    lib = _lib.load()
    ctx = api.Context(0)
    max_n = ctypes.c_int64(0)
    assert lib.mis2_run_noalloc_max_n(ctypes.byref(max_n)) == _lib.MIS2_OK
    assert max_n.value >= 1_000_000  # room for the 100^3 grids
    small = torch.zeros(16, dtype=torch.int64, device="cuda")
    status = torch.zeros(16, dtype=torch.uint8, device="cuda")
    g = _lib.Mis2Graph(max_n.value + 1, 0, small.data_ptr(), 0)
    nr, ni = ctypes.c_int64(0), ctypes.c_int32(0)
    rc = lib.mis2_run_noalloc(ctx.ptr, ctypes.byref(g), ctypes.c_uint64(0),
                              ctypes.c_void_p(status.data_ptr()), ctypes.byref(nr),
                              ctypes.byref(ni), None)
    assert rc == _lib.MIS2_ENOSPACE
    assert b"static scratch" in lib.mis2_last_error(ctx.ptr)
    prof = api.Context(0, profile=True)
    rp, c, nnz = _device_graph(torch, api, graphs.path(10))
    st = torch.zeros(10, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.Mis2Error):
        prof.mis2_noalloc(rp, c, st, nnz=nnz)
