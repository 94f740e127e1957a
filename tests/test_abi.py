"""The C-ABI library builds, loads and exports every symbol include/mis2.h
declares; host-only entry points work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mis2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mis2_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("mis2_run", "mis2_aggregate", "mis2_create", "mis2_workspace_bytes"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2204_02934_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def test_workspace_bytes_host_only():
    from paper_2204_02934_amd import _lib
    lib = _lib.load()
    b = ctypes.c_size_t(0)
    assert lib.mis2_workspace_bytes(1000, _lib.MIS2_OP_MIS2, ctypes.byref(b)) == 0
    small = b.value
    assert small >= 24 * 1000
    assert lib.mis2_workspace_bytes(1000, _lib.MIS2_OP_AGGREGATE, ctypes.byref(b)) == 0
    assert b.value > small
    assert lib.mis2_workspace_bytes(-1, 0, ctypes.byref(b)) == _lib.MIS2_EINVAL
    assert lib.mis2_workspace_bytes(10, 7, ctypes.byref(b)) == _lib.MIS2_EINVAL


def test_null_context_is_rejected():
    from paper_2204_02934_amd import _lib
    lib = _lib.load()
    assert lib.mis2_set_option(None, 0, 1) == _lib.MIS2_EINVAL
    assert lib.mis2_last_error(None) == b"null context"
    lib.mis2_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2204_02934_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


def test_host_only_size_queries_of_batching_and_serving():
    from paper_2204_02934_amd import _lib
    lib = _lib.load()
    b = ctypes.c_size_t(0)
    assert lib.mis2_batch_workspace_bytes(4, 1000, 5000, ctypes.byref(b)) == 0
    coarsen = ctypes.c_size_t(0)
    assert lib.mis2_coarsen_workspace_bytes(1000, 5000, ctypes.byref(coarsen)) == 0
    assert b.value > coarsen.value  # the union needs the coarsening workspace and more
    assert lib.mis2_batch_workspace_bytes(-1, 1000, 5000, ctypes.byref(b)) == _lib.MIS2_EINVAL
    assert lib.mis2_server_bytes(1000, 5000, 8, ctypes.byref(b)) == 0 and b.value > 0
    assert lib.mis2_server_bytes(0, 5000, 8, ctypes.byref(b)) == _lib.MIS2_EINVAL
    assert lib.mis2_server_bytes(1000, 5000, 0, ctypes.byref(b)) == _lib.MIS2_EINVAL


def test_null_server_is_rejected():
    from paper_2204_02934_amd import _lib
    lib = _lib.load()
    assert lib.mis2_server_last_error(None) == b"null server"
    assert lib.mis2_server_step(None, None, None) == _lib.MIS2_EINVAL
    k = ctypes.c_int32(0)
    assert lib.mis2_server_poll(None, None, 0, ctypes.byref(k)) == _lib.MIS2_EINVAL
    lib.mis2_server_destroy(None)
    out = ctypes.c_void_p()
    # a null arena is rejected before any device is touched
    assert lib.mis2_server_create(ctypes.byref(out), 0, None, 0, 1000, 5000, 8, 0, 100,
                                  4) == _lib.MIS2_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stderr + r.stdout)


def test_serving_pool_recipe():
    import sys
    sys.path.insert(0, ROOT)
    import bench
    pool = bench.c5_pool(6, n_hi=20000)
    assert len(pool) == 6
    for kind, (rp, c) in pool:
        assert kind in ("2d5", "3d27", "chunglu")
        assert rp.size >= 2 and int(rp[-1]) == c.size
