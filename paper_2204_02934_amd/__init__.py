"""Deterministic distance-2 maximal independent set (MIS-2) and MIS-2 aggregation
on AMD MI355X (gfx950), after Kelley & Rajamanickam, arXiv 2204.02934.

The computation runs in libmis2.so (hand-written HIP kernels behind the C ABI
of include/mis2.h); this package binds it for PyTorch tensors.  `graphs`
builds seeded synthetic inputs.  The binding is imported lazily so that the
generators work on machines without a GPU.
"""


def __getattr__(name):
    if name in ("Context", "mis2", "aggregate", "default_context", "as_device_csr"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
