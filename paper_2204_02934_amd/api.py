"""Python binding of the MIS-2 library: argument marshalling only.

PyTorch provides device memory (inputs, outputs, workspace) and the HIP
stream; every step of the computation runs in libmis2.so's kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Mis2Error, Mis2Graph


def _check(lib, ctx, rc):
    if rc != _lib.MIS2_OK:
        msg = lib.mis2_last_error(ctx)
        raise Mis2Error(rc, msg.decode() if msg else "")


def _stream_ptr(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def as_device_csr(row_ptr, col, device="cuda"):
    """(row_ptr int64, col int32) as contiguous tensors on `device`."""
    rp = torch.as_tensor(np.asarray(row_ptr) if not torch.is_tensor(row_ptr) else row_ptr)
    cc = torch.as_tensor(np.asarray(col) if not torch.is_tensor(col) else col)
    rp = rp.to(device=device, dtype=torch.int64).contiguous()
    cc = cc.to(device=device, dtype=torch.int32).contiguous()
    if cc.numel() == 0:
        cc = torch.zeros(1, dtype=torch.int32, device=device)  # a valid pointer
    return rp, cc


class Context:
    """One mis2_ctx bound to a GPU, with a torch-allocated workspace that grows
    on demand (allocation happens outside the library calls)."""

    def __init__(self, device=None, validate=False, lanes=0, blocks=0, profile=False,
                 account=False, persistent=False, compact=True, autotune=True, tail=-1,
                 queue_depth=0):
        self.lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.ptr = ctypes.c_void_p()
        _check(self.lib, None, self.lib.mis2_create(ctypes.byref(self.ptr), self.device.index or 0))
        self._ws = None
        self.set_option(_lib.MIS2_OPT_VALIDATE, int(validate))
        self.set_option(_lib.MIS2_OPT_LANES_PER_ROW, lanes)
        self.set_option(_lib.MIS2_OPT_GRID_BLOCKS, blocks)
        self.set_option(_lib.MIS2_OPT_PROFILE, int(profile))
        self.set_option(_lib.MIS2_OPT_ACCOUNT, int(account))
        self.set_option(_lib.MIS2_OPT_PERSISTENT, int(persistent))
        self.set_option(_lib.MIS2_OPT_COMPACT, int(compact))
        self.set_option(_lib.MIS2_OPT_AUTOTUNE, int(autotune))
        self.set_option(_lib.MIS2_OPT_TAIL, int(tail))
        self.set_option(_lib.MIS2_OPT_QUEUE_DEPTH, int(queue_depth))

    def __del__(self):
        lib = getattr(self, "lib", None)
        if lib is not None and getattr(self, "ptr", None):
            lib.mis2_destroy(self.ptr)
            self.ptr = None

    def set_option(self, option, value):
        _check(self.lib, self.ptr, self.lib.mis2_set_option(self.ptr, option, int(value)))

    def workspace_bytes(self, n, op, nnz=None):
        """mis2_workspace_bytes, or with nnz mis2_workspace_bytes_csr (room for
        the compacted adjacency as well)."""
        b = ctypes.c_size_t(0)
        if nnz is None:
            rc = self.lib.mis2_workspace_bytes(int(n), op, ctypes.byref(b))
        else:
            rc = self.lib.mis2_workspace_bytes_csr(int(n), int(nnz), op, ctypes.byref(b))
        _check(self.lib, self.ptr, rc)
        return b.value

    def ensure_workspace(self, n, op, nnz=None):
        need = self.workspace_bytes(n, op, nnz)
        if self._ws is None or self._ws.numel() < need:
            # torch's caching allocator returns 512-byte aligned blocks
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            _check(self.lib, self.ptr, self.lib.mis2_set_workspace(
                self.ptr, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel()))
        return self._ws

    def graph(self, row_ptr, col, nnz=None):
        rp, cc = as_device_csr(row_ptr, col, self.device)
        n = rp.numel() - 1
        if nnz is None:
            nnz = int(rp[-1].item())
        return Mis2Graph(n, nnz, rp.data_ptr(), cc.data_ptr()), (rp, cc)

    def mis2(self, row_ptr, col, seed=0, stream=None, nnz=None):
        """Algorithm 1.  Returns (status uint8[n] on the GPU, n_roots, n_iters)."""
        g, keep = self.graph(row_ptr, col, nnz)
        self.ensure_workspace(g.n, _lib.MIS2_OP_MIS2, g.nnz)
        status = torch.empty(max(g.n, 1), dtype=torch.uint8, device=self.device)
        nr, ni = ctypes.c_int64(0), ctypes.c_int32(0)
        rc = self.lib.mis2_run(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed),
                               ctypes.c_void_p(status.data_ptr()), ctypes.byref(nr),
                               ctypes.byref(ni), _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        return status[:g.n], nr.value, ni.value

    def mis2_noalloc(self, row_ptr, col, status, seed=0, stream=None, nnz=None):
        """Algorithm 1 through mis2_run_noalloc: the library's static device
        scratch is the workspace and the call allocates nothing; the caller
        passes the uint8 status tensor (>= n entries).  Returns (n_roots,
        n_iters)."""
        g, keep = self.graph(row_ptr, col, nnz)
        if g.n > 0 and (status.dtype != torch.uint8 or status.numel() < g.n or
                        status.device != self.device):
            raise ValueError("status must be a uint8 tensor of >= n entries on " + str(self.device))
        nr, ni = ctypes.c_int64(0), ctypes.c_int32(0)
        rc = self.lib.mis2_run_noalloc(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed),
                                       ctypes.c_void_p(status.data_ptr()), ctypes.byref(nr),
                                       ctypes.byref(ni), _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        return nr.value, ni.value

    def aggregate(self, row_ptr, col, seed=0, stream=None, nnz=None, want_roots=False):
        """Algorithm 3.  Returns (agg int32[n] on the GPU, n_agg) or, with
        want_roots, (agg, n_agg, roots uint8[n])."""
        g, keep = self.graph(row_ptr, col, nnz)
        self.ensure_workspace(g.n, _lib.MIS2_OP_AGGREGATE, g.nnz)
        agg = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        roots = torch.empty(max(g.n, 1), dtype=torch.uint8, device=self.device) if want_roots else None
        na = ctypes.c_int64(0)
        rc = self.lib.mis2_aggregate(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed),
                                     ctypes.c_void_p(agg.data_ptr()), ctypes.byref(na),
                                     ctypes.c_void_p(roots.data_ptr() if roots is not None else 0),
                                     _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        if want_roots:
            return agg[:g.n], na.value, roots[:g.n]
        return agg[:g.n], na.value

    def cgs_setup(self, row_ptr, col, seed=0, point=False, stream=None, nnz=None):
        """Algorithm 4's setup (mis2_cgs_setup): returns a CgsPlan holding the
        device arrays cluster, cluster_color, rows, pos, cluster_off and the host
        colour offsets."""
        g, keep = self.graph(row_ptr, col, nnz)
        b = ctypes.c_size_t(0)
        _check(self.lib, self.ptr, self.lib.mis2_cgs_workspace_bytes(g.n, g.nnz, ctypes.byref(b)))
        self._ensure_bytes(b.value)
        n = g.n
        dev = self.device
        plan = CgsPlan(n, dev)
        rc = self.lib.mis2_cgs_setup(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed), int(point),
                                     ctypes.byref(plan.c), _stream_ptr(stream, dev))
        _check(self.lib, self.ptr, rc)
        plan.keep = keep
        return plan

    def cgs_apply(self, row_ptr, col, val, diag, plan, b, x, sweeps=1, symmetric=False,
                  stream=None, nnz=None):
        """sweeps applications of Algorithm 4 to x (float64 CUDA tensor, in
        place) for the matrix with off-diagonal values val and diagonal diag."""
        g, keep = self.graph(row_ptr, col, nnz)
        tensors = [val, diag, b, x]
        for t in tensors:
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        rc = self.lib.mis2_cgs_apply(self.ptr, ctypes.byref(g), ctypes.c_void_p(val.data_ptr()),
                                     ctypes.c_void_p(diag.data_ptr()), ctypes.byref(plan.c),
                                     ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     int(sweeps), int(symmetric), _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        return x

    def mis2_ablation(self, row_ptr, col, seed=0, flags=0, stream=None, nnz=None):
        """Algorithm 1 with Section V's optimizations taken away (MIS2_ABL_*
        flags).  Returns (status uint8[n] on the GPU, n_roots, n_iters)."""
        g, keep = self.graph(row_ptr, col, nnz)
        b = ctypes.c_size_t(0)
        _check(self.lib, self.ptr,
               self.lib.mis2_ablation_workspace_bytes(g.n, int(flags), ctypes.byref(b)))
        self._ensure_bytes(max(b.value, self.workspace_bytes(g.n, _lib.MIS2_OP_MIS2, g.nnz)))
        status = torch.empty(max(g.n, 1), dtype=torch.uint8, device=self.device)
        nr, ni = ctypes.c_int64(0), ctypes.c_int32(0)
        rc = self.lib.mis2_run_ablation(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed), int(flags),
                                        ctypes.c_void_p(status.data_ptr()), ctypes.byref(nr),
                                        ctypes.byref(ni), _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        return status[:g.n], nr.value, ni.value

    def aggregate_basic(self, row_ptr, col, seed=0, stream=None, nnz=None, want_roots=False):
        """Algorithm 2 (basic MIS-2 coarsening).  Returns (agg int32[n] on the
        GPU, n_agg) or, with want_roots, (agg, n_agg, roots uint8[n])."""
        g, keep = self.graph(row_ptr, col, nnz)
        self.ensure_workspace(g.n, _lib.MIS2_OP_AGGREGATE, g.nnz)
        agg = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.device)
        roots = torch.empty(max(g.n, 1), dtype=torch.uint8, device=self.device) if want_roots else None
        na = ctypes.c_int64(0)
        rc = self.lib.mis2_aggregate_basic(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed),
                                           ctypes.c_void_p(agg.data_ptr()), ctypes.byref(na),
                                           ctypes.c_void_p(roots.data_ptr() if roots is not None else 0),
                                           _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        if want_roots:
            return agg[:g.n], na.value, roots[:g.n]
        return agg[:g.n], na.value

    def _ensure_bytes(self, need):
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            _check(self.lib, self.ptr, self.lib.mis2_set_workspace(
                self.ptr, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel()))

    def quotient(self, row_ptr, col, agg, n_agg, stream=None, nnz=None):
        """Coarse (quotient) graph of an aggregation: (row_ptr int64[n_agg+1],
        col int32[coarse nnz]) on the GPU."""
        g, keep = self.graph(row_ptr, col, nnz)
        self.ensure_workspace(g.n, _lib.MIS2_OP_COARSEN)
        agg = torch.as_tensor(agg).to(device=self.device, dtype=torch.int32).contiguous()
        crow = torch.empty(n_agg + 1, dtype=torch.int64, device=self.device)
        ccol = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=self.device)
        cnnz = ctypes.c_int64(0)
        rc = self.lib.mis2_quotient(self.ptr, ctypes.byref(g), ctypes.c_void_p(agg.data_ptr()),
                                    int(n_agg), ctypes.c_void_p(crow.data_ptr()),
                                    ctypes.c_void_p(ccol.data_ptr()), ctypes.byref(cnnz),
                                    _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep
        return crow, ccol[:cnnz.value]

    def galerkin(self, row_ptr, col, val, diag, agg, crow, ccol, stream=None, nnz=None):
        """Galerkin coarse operator P^T A P of an aggregation (mis2_galerkin)
        with the tentative prolongator P[i][agg i] = 1/sqrt(|agg i|): returns
        (off-diagonal values in the coarse graph's CSR order, diagonal), float64
        on the GPU.  (crow, ccol) is the quotient graph, as from quotient()."""
        g, keep = self.graph(row_ptr, col, nnz)
        cg, ckeep = self.graph(crow, ccol)
        for t in (val, diag):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        agg = torch.as_tensor(agg).to(device=self.device, dtype=torch.int32).contiguous()
        b = ctypes.c_size_t(0)
        _check(self.lib, self.ptr, self.lib.mis2_galerkin_workspace_bytes(g.n, cg.n, ctypes.byref(b)))
        self._ensure_bytes(b.value)
        cval = torch.empty(max(cg.nnz, 1), dtype=torch.float64, device=self.device)
        cdiag = torch.empty(max(cg.n, 1), dtype=torch.float64, device=self.device)
        rc = self.lib.mis2_galerkin(self.ptr, ctypes.byref(g), ctypes.c_void_p(val.data_ptr()),
                                    ctypes.c_void_p(diag.data_ptr()), ctypes.c_void_p(agg.data_ptr()),
                                    ctypes.byref(cg), ctypes.c_void_p(cval.data_ptr()),
                                    ctypes.c_void_p(cdiag.data_ptr()), _stream_ptr(stream, self.device))
        _check(self.lib, self.ptr, rc)
        del keep, ckeep
        return cval[:cg.nnz], cdiag[:cg.n]

    def smoothed(self, row_ptr, col, val, diag, agg, n_agg, omega, stream=None, nnz=None):
        """Smoothed aggregation (mis2_smoothed): the prolongator
        P = (I - omega D^-1 A) P_tent and the coarse operator P^T A P.  Returns
        ((prow, pcol, pval), (crow, ccol, cval)), CSR arrays on the GPU."""
        g, keep = self.graph(row_ptr, col, nnz)
        for t in (val, diag):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        agg = torch.as_tensor(agg).to(device=self.device, dtype=torch.int32).contiguous()
        n = g.n
        prow = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        crow = torch.empty(max(n_agg, 0) + 1, dtype=torch.int64, device=self.device)
        p_cap = max(n + g.nnz, 1)  # P row i holds at most deg(i) + 1 entries
        pcol = torch.empty(p_cap, dtype=torch.int32, device=self.device)
        pval = torch.empty(p_cap, dtype=torch.float64, device=self.device)
        # A_c's size is known only after its count pass: start from the size
        # the last call on a graph of this shape needed, if any
        caps = self.__dict__.setdefault("_smoothed_caps", {})
        c_cap = max(min(n_agg * n_agg, 32 * n_agg), caps.get((n, g.nnz, int(n_agg)), 0), 1)
        ccol = torch.empty(c_cap, dtype=torch.int32, device=self.device)
        cval = torch.empty(c_cap, dtype=torch.float64, device=self.device)
        pn, cn, need = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_size_t(0)
        for _ in range(6):
            rc = self.lib.mis2_smoothed(
                self.ptr, ctypes.byref(g), ctypes.c_void_p(val.data_ptr()),
                ctypes.c_void_p(diag.data_ptr()), ctypes.c_void_p(agg.data_ptr()), int(n_agg),
                ctypes.c_double(omega), ctypes.c_void_p(prow.data_ptr()),
                ctypes.c_void_p(pcol.data_ptr()), ctypes.c_void_p(pval.data_ptr()), p_cap,
                ctypes.c_void_p(crow.data_ptr()), ctypes.c_void_p(ccol.data_ptr()),
                ctypes.c_void_p(cval.data_ptr()), c_cap, ctypes.byref(pn), ctypes.byref(cn),
                ctypes.byref(need), _stream_ptr(stream, self.device))
            if rc != _lib.MIS2_ENOSPACE:
                break
            if need.value:
                self._ensure_bytes(need.value)
            elif cn.value > c_cap:
                c_cap = cn.value
                ccol = torch.empty(c_cap, dtype=torch.int32, device=self.device)
                cval = torch.empty(c_cap, dtype=torch.float64, device=self.device)
            else:
                break
        _check(self.lib, self.ptr, rc)
        caps[(n, g.nnz, int(n_agg))] = cn.value
        del keep
        return ((prow, pcol[:pn.value], pval[:pn.value]),
                (crow, ccol[:cn.value], cval[:cn.value]))

    def coarsen(self, row_ptr, col, seed=0, stop_below=1000, max_levels=64, stream=None, nnz=None):
        """Multilevel coarsening: list of per-level dicts {n, nnz, n_agg, agg
        (int32 labels on the GPU)}."""
        g, keep = self.graph(row_ptr, col, nnz)
        b = ctypes.c_size_t(0)
        _check(self.lib, self.ptr, self.lib.mis2_coarsen_workspace_bytes(g.n, g.nnz, ctypes.byref(b)))
        self._ensure_bytes(b.value)
        cap = max(2 * g.n, 1)
        agg = torch.empty(cap, dtype=torch.int32, device=self.device)
        ln = (ctypes.c_int64 * max(max_levels, 1))()
        lz = (ctypes.c_int64 * max(max_levels, 1))()
        la = (ctypes.c_int64 * max(max_levels, 1))()
        nl = ctypes.c_int32(0)
        while True:
            rc = self.lib.mis2_coarsen(self.ptr, ctypes.byref(g), ctypes.c_uint64(seed),
                                       int(stop_below), int(max_levels),
                                       ctypes.c_void_p(agg.data_ptr()), agg.numel(), ln, lz, la,
                                       ctypes.byref(nl), _stream_ptr(stream, self.device))
            if rc == _lib.MIS2_ENOSPACE and b"agg_cap" in self.lib.mis2_last_error(self.ptr):
                agg = torch.empty(2 * agg.numel(), dtype=torch.int32, device=self.device)
                continue
            break
        _check(self.lib, self.ptr, rc)
        del keep
        out, off = [], 0
        for i in range(nl.value):
            out.append({"n": ln[i], "nnz": lz[i], "n_agg": la[i], "agg": agg[off:off + ln[i]]})
            off += ln[i]
        return out

    def aggregate_batched(self, row_ptr, col, vtx_off, seed=0, stop_below=1000, max_levels=64,
                          stream=None, nnz=None):
        """Multilevel coarsening of every graph of a disjoint union in one call
        (mis2_aggregate_batched).  vtx_off: host int64[G + 1] vertex offsets of
        the graphs in the union.  Returns, per graph, the list of its levels as
        dicts {n, nnz, n_agg, agg (int32 graph-local labels on the GPU)}."""
        g, keep = self.graph(row_ptr, col, nnz)
        voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
        G = voff.size - 1
        b = ctypes.c_size_t(0)
        _check(self.lib, self.ptr,
               self.lib.mis2_batch_workspace_bytes(G, g.n, g.nnz, ctypes.byref(b)))
        self._ensure_bytes(b.value)
        cap = max(2 * g.n, 1)
        agg = torch.empty(cap, dtype=torch.int32, device=self.device)
        k = max(max_levels, 1) * max(G, 1)
        ln = (ctypes.c_int64 * k)()
        lz = (ctypes.c_int64 * k)()
        la = (ctypes.c_int64 * k)()
        nl = (ctypes.c_int32 * max(G, 1))()
        vo = voff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        while True:
            rc = self.lib.mis2_aggregate_batched(self.ptr, ctypes.byref(g), G, vo,
                                                 ctypes.c_uint64(seed), int(stop_below),
                                                 int(max_levels), ctypes.c_void_p(agg.data_ptr()),
                                                 agg.numel(), ln, lz, la, nl,
                                                 _stream_ptr(stream, self.device))
            if rc == _lib.MIS2_ENOSPACE and b"agg_cap" in self.lib.mis2_last_error(self.ptr):
                agg = torch.empty(2 * agg.numel(), dtype=torch.int32, device=self.device)
                continue
            break
        _check(self.lib, self.ptr, rc)
        del keep
        out = [[] for _ in range(G)]
        off = 0
        for lv in range(max(nl[i] for i in range(G)) if G else 0):
            for i in range(G):
                if lv == 0:
                    n_i = int(voff[i + 1] - voff[i])
                    if nl[i] > 0:
                        out[i].append({"n": ln[i], "nnz": lz[i], "n_agg": la[i],
                                       "agg": agg[off + int(voff[i]):off + int(voff[i + 1])]})
                    continue
                if nl[i] > lv:
                    e = lv * G + i
                    out[i].append({"n": ln[e], "nnz": lz[e], "n_agg": la[e],
                                   "agg": agg[off:off + ln[e]]})
                    off += ln[e]
            if lv == 0:
                off += g.n
        return out

    def last_trace(self, phase=0, cap=4096):
        """Per-round (|worklist1|, |worklist2|) of the last call, int64[rounds, 2]."""
        buf = (ctypes.c_int64 * (2 * cap))()
        r = ctypes.c_int32(0)
        _check(self.lib, self.ptr, self.lib.mis2_last_trace(self.ptr, phase, buf, cap, ctypes.byref(r)))
        k = min(r.value, cap)
        return np.ctypeslib.as_array(buf)[:2 * k].reshape(k, 2).copy()


    def last_plan(self):
        """Plan of the last call: {lanes (-2 = staged sweeps), blocks, tail (1
        = last rounds in one workgroup), source (0 = options or the degree
        rule, 1 = tuned plan from the cache, 2 = tuned during the call)}."""
        a, b, t, c = (ctypes.c_int32(0) for _ in range(4))
        _check(self.lib, self.ptr, self.lib.mis2_last_plan(self.ptr, ctypes.byref(a), ctypes.byref(b),
                                                           ctypes.byref(t), ctypes.byref(c)))
        return {"lanes": a.value, "blocks": b.value, "tail": t.value, "source": c.value}

    def last_tuning(self, cap=64):
        """Candidate plans the last tuning on this context timed: list of
        {lanes, blocks, ms}."""
        buf = (_lib.Mis2TuneRecord * cap)()
        k = ctypes.c_int32(0)
        _check(self.lib, self.ptr, self.lib.mis2_last_tuning(self.ptr, buf, cap, ctypes.byref(k)))
        return [{"lanes": buf[i].lanes, "blocks": buf[i].blocks, "tail": buf[i].tail,
                 "ms": buf[i].ms} for i in range(min(k.value, cap))]

    def last_sweeps(self, cap=8192):
        """Sweep launches of the last call: list of dicts (kind 0 = Refresh
        Column, 1 = Decide Set; edges / ms are -1 unless accounting /
        profiling is on; compact as mis2_sweep_record.compact)."""
        buf = (_lib.Mis2SweepRecord * cap)()
        k = ctypes.c_int32(0)
        _check(self.lib, self.ptr, self.lib.mis2_last_sweeps(self.ptr, buf, cap, ctypes.byref(k)))
        out = []
        for i in range(min(k.value, cap)):
            r = buf[i]
            out.append({"kind": r.kind, "phase": r.phase, "round": r.round, "lanes": r.lanes,
                        "rows": r.rows, "rows_out": r.rows_out, "edges": r.edges, "ms": r.ms,
                        "compact": r.compact, "written": r.written})
        return out


class CgsPlan:
    """The arrays of a mis2_cgs_plan (device tensors and host colour offsets)."""

    def __init__(self, n, device):
        m = max(n, 1)
        self.cluster = torch.empty(m, dtype=torch.int32, device=device)
        self.cluster_color = torch.empty(m, dtype=torch.int32, device=device)
        self.rows = torch.empty(m, dtype=torch.int32, device=device)
        self.pos = torch.empty(m, dtype=torch.int32, device=device)
        self.cluster_off = torch.empty(n + 1, dtype=torch.int64, device=device)
        self.color_off = np.zeros(n + 1, np.int64)
        self.c = _lib.Mis2CgsPlan()
        self.c.n = n
        self.c.cluster = self.cluster.data_ptr()
        self.c.cluster_color = self.cluster_color.data_ptr()
        self.c.rows = self.rows.data_ptr()
        self.c.pos = self.pos.data_ptr()
        self.c.cluster_off = self.cluster_off.data_ptr()
        self.c.color_off = self.color_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    @property
    def n_clusters(self):
        return self.c.n_clusters

    @property
    def n_colors(self):
        return self.c.n_colors


class Server:
    """A mis2_server: continuous batching of multilevel coarsening jobs.  The
    arena is one torch allocation sized for the given union capacities."""

    def __init__(self, max_vertices, max_nnz, max_graphs=1024, seed=0, stop_below=1000,
                 max_levels=_lib.MIS2_SERVE_MAX_LEVELS, device=None):
        self.lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        b = ctypes.c_size_t(0)
        rc = self.lib.mis2_server_bytes(int(max_vertices), int(max_nnz), int(max_graphs),
                                        ctypes.byref(b))
        if rc != _lib.MIS2_OK:
            raise Mis2Error(rc, "bad server capacities")
        self.arena = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.ptr = ctypes.c_void_p()
        rc = self.lib.mis2_server_create(ctypes.byref(self.ptr), self.device.index or 0,
                                         ctypes.c_void_p(self.arena.data_ptr()), b.value,
                                         int(max_vertices), int(max_nnz), int(max_graphs),
                                         ctypes.c_uint64(seed), int(stop_below), int(max_levels))
        if rc != _lib.MIS2_OK:
            raise Mis2Error(rc, "mis2_server_create failed")
        self._jobs = {}  # tag -> (graph tensors, agg tensor), kept alive until polled
        self._copy_stream = None  # uploads of host CSRs
        self._uploads = []        # their events, waited for by the next step

    def _check(self, rc):
        if rc != _lib.MIS2_OK:
            msg = self.lib.mis2_server_last_error(self.ptr)
            raise Mis2Error(rc, msg.decode() if msg else "")

    def submit(self, row_ptr, col, tag, agg_cap=None, nnz=None):
        """Queue one coarsening job (device or host CSR); its labels land in a
        device int32 tensor returned by poll().  A host CSR is copied to the
        GPU on a side stream, so the copy overlaps the level running on the
        server's stream; the next step() waits for it before it admits jobs."""
        if not torch.is_tensor(row_ptr) or row_ptr.device.type != "cuda":
            rp_h = torch.as_tensor(np.asarray(row_ptr), dtype=torch.int64)
            cc_h = torch.as_tensor(np.asarray(col), dtype=torch.int32)
            if cc_h.numel() == 0:
                cc_h = torch.zeros(1, dtype=torch.int32)
            if self._copy_stream is None:
                self._copy_stream = torch.cuda.Stream(device=self.device)
            with torch.cuda.stream(self._copy_stream):
                rp = rp_h.pin_memory().to(self.device, non_blocking=True)
                cc = cc_h.pin_memory().to(self.device, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self._copy_stream)
            self._uploads.append(ev)
            if nnz is None:
                nnz = int(rp_h[-1])
        else:
            rp, cc = as_device_csr(row_ptr, col, self.device)
        n = rp.numel() - 1
        if nnz is None:
            nnz = int(rp[-1].item())
        cap = max(2 * n, 1) if agg_cap is None else agg_cap
        agg = torch.empty(cap, dtype=torch.int32, device=self.device)
        g = Mis2Graph(n, nnz, rp.data_ptr(), cc.data_ptr())
        self._check(self.lib.mis2_server_submit(self.ptr, ctypes.byref(g),
                                                ctypes.c_void_p(agg.data_ptr()), cap, int(tag)))
        self._jobs[int(tag)] = (rp, cc, agg)

    def step(self, stream=None):
        """One admission + level step; returns the number of jobs still queued
        or coarsening."""
        if self._uploads:
            st = stream if stream is not None else torch.cuda.current_stream(self.device)
            for ev in self._uploads:
                st.wait_event(ev)
            self._uploads = []
        k = ctypes.c_int32(0)
        self._check(self.lib.mis2_server_step(self.ptr, _stream_ptr(stream, self.device),
                                              ctypes.byref(k)))
        return k.value

    def poll(self, cap=4096):
        """Finished jobs: list of dicts {tag, levels: [{n, nnz, n_agg, agg}], truncated}."""
        buf = (_lib.Mis2JobResult * cap)()
        k = ctypes.c_int32(0)
        self._check(self.lib.mis2_server_poll(self.ptr, buf, cap, ctypes.byref(k)))
        out = []
        for i in range(k.value):
            r = buf[i]
            _, _, agg = self._jobs.pop(int(r.tag))
            levels, off = [], 0
            for lv in range(r.n_levels):
                levels.append({"n": r.level_n[lv], "nnz": r.level_nnz[lv],
                               "n_agg": r.level_nagg[lv], "agg": agg[off:off + r.level_n[lv]]})
                off += r.level_n[lv]
            out.append({"tag": r.tag, "levels": levels, "truncated": bool(r.truncated)})
        return out

    def close(self):
        if self.ptr:
            self.lib.mis2_server_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device=None):
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def mis2(row_ptr, col, seed=0, stream=None):
    """Deterministic MIS-2 (Algorithm 1): (status, n_roots, n_iters)."""
    return default_context().mis2(row_ptr, col, seed, stream)


def aggregate(row_ptr, col, seed=0, stream=None):
    """MIS-2 aggregation (Algorithm 3): (agg_id, n_agg)."""
    return default_context().aggregate(row_ptr, col, seed, stream)
