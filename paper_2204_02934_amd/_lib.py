"""ctypes loader for libmis2.so (the C ABI in include/mis2.h).

There is no fallback: if the HIP library is missing, loading raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmis2.so")

MIS2_OK = 0
MIS2_EINVAL = -1
MIS2_EGRAPH = -2
MIS2_ENOSPACE = -3
MIS2_EHIP = -4
MIS2_EINTERNAL = -5

MIS2_OP_MIS2 = 0
MIS2_OP_AGGREGATE = 1
MIS2_OP_COARSEN = 2

MIS2_OPT_VALIDATE = 0
MIS2_OPT_LANES_PER_ROW = 1
MIS2_OPT_GRID_BLOCKS = 2
MIS2_OPT_PROFILE = 3
MIS2_OPT_ACCOUNT = 4
MIS2_OPT_PERSISTENT = 5
MIS2_OPT_COMPACT = 6
MIS2_OPT_AUTOTUNE = 7
MIS2_OPT_TAIL = 8
MIS2_OPT_QUEUE_DEPTH = 9
MIS2_ABL_FIXED_PRIORITY = 1
MIS2_ABL_XORSHIFT = 2
MIS2_ABL_NO_WORKLISTS = 4
MIS2_ABL_UNPACKED = 8
MIS2_ABL_ONE_LANE = 16
MIS2_ABL_SIMPLE = 32
MIS2_LANES_STAGED = -2

# Every symbol include/mis2.h declares.
EXPORTS = (
    "mis2_create", "mis2_destroy", "mis2_last_error", "mis2_set_option",
    "mis2_workspace_bytes", "mis2_workspace_bytes_csr", "mis2_set_workspace", "mis2_run",
    "mis2_last_trace", "mis2_aggregate", "mis2_aggregate_basic", "mis2_last_sweeps",
    "mis2_run_ablation", "mis2_ablation_workspace_bytes", "mis2_cgs_workspace_bytes",
    "mis2_cgs_setup", "mis2_cgs_apply",
    "mis2_quotient", "mis2_galerkin_workspace_bytes", "mis2_galerkin", "mis2_coarsen_workspace_bytes",
    "mis2_coarsen", "mis2_batch_workspace_bytes", "mis2_aggregate_batched",
    "mis2_server_bytes", "mis2_server_create", "mis2_server_destroy", "mis2_server_last_error",
    "mis2_server_submit", "mis2_server_step", "mis2_server_poll",
    "mis2_run_noalloc", "mis2_run_noalloc_max_n", "mis2_last_plan", "mis2_last_tuning",
    "mis2_smoothed",
)

MIS2_SERVE_MAX_LEVELS = 32


class Mis2Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class Mis2CgsPlan(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_clusters", ctypes.c_int64),
                ("n_colors", ctypes.c_int32), ("cluster", ctypes.c_void_p),
                ("cluster_color", ctypes.c_void_p), ("rows", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("cluster_off", ctypes.c_void_p), ("color_off", ctypes.POINTER(ctypes.c_int64))]


class Mis2SweepRecord(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("phase", ctypes.c_int32), ("round", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("rows", ctypes.c_int64), ("rows_out", ctypes.c_int64),
                ("edges", ctypes.c_int64), ("ms", ctypes.c_float), ("compact", ctypes.c_int32),
                ("written", ctypes.c_int64)]


class Mis2TuneRecord(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("blocks", ctypes.c_int32), ("tail", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class Mis2JobResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("truncated", ctypes.c_int32),
                ("level_n", ctypes.c_int64 * MIS2_SERVE_MAX_LEVELS),
                ("level_nnz", ctypes.c_int64 * MIS2_SERVE_MAX_LEVELS),
                ("level_nagg", ctypes.c_int64 * MIS2_SERVE_MAX_LEVELS)]


class Mis2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mis2 error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Load libmis2.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmis2.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2204_02934_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    gp = ctypes.POINTER(Mis2Graph)
    sig = {
        "mis2_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int]),
        "mis2_destroy": (None, [vp]),
        "mis2_last_error": (ctypes.c_char_p, [vp]),
        "mis2_set_option": (ctypes.c_int, [vp, ctypes.c_int, i64]),
        "mis2_workspace_bytes": (ctypes.c_int, [i64, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_workspace_bytes_csr": (ctypes.c_int, [i64, i64, ctypes.c_int,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_set_workspace": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "mis2_run": (ctypes.c_int, [vp, gp, u64, vp, ctypes.POINTER(i64), ctypes.POINTER(i32), vp]),
        "mis2_run_noalloc": (ctypes.c_int, [vp, gp, u64, vp, ctypes.POINTER(i64),
                                            ctypes.POINTER(i32), vp]),
        "mis2_run_noalloc_max_n": (ctypes.c_int, [ctypes.POINTER(i64)]),
        "mis2_last_trace": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(i64), i32,
                                           ctypes.POINTER(i32)]),
        "mis2_aggregate": (ctypes.c_int, [vp, gp, u64, vp, ctypes.POINTER(i64), vp, vp]),
        "mis2_aggregate_basic": (ctypes.c_int, [vp, gp, u64, vp, ctypes.POINTER(i64), vp, vp]),
        "mis2_cgs_workspace_bytes": (ctypes.c_int, [i64, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_cgs_setup": (ctypes.c_int, [vp, gp, u64, ctypes.c_int, ctypes.POINTER(Mis2CgsPlan),
                                          vp]),
        "mis2_cgs_apply": (ctypes.c_int, [vp, gp, vp, vp, ctypes.POINTER(Mis2CgsPlan), vp, vp,
                                          i32, ctypes.c_int, vp]),
        "mis2_run_ablation": (ctypes.c_int, [vp, gp, u64, ctypes.c_int, vp, ctypes.POINTER(i64),
                                             ctypes.POINTER(i32), vp]),
        "mis2_ablation_workspace_bytes": (ctypes.c_int, [i64, ctypes.c_int,
                                                         ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_smoothed": (ctypes.c_int, [vp, gp, vp, vp, vp, i64, ctypes.c_double, vp, vp, vp,
                                         i64, vp, vp, vp, i64, ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t),
                                         vp]),
        "mis2_last_plan": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                          ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "mis2_last_tuning": (ctypes.c_int, [vp, ctypes.POINTER(Mis2TuneRecord), i32,
                                            ctypes.POINTER(i32)]),
        "mis2_last_sweeps": (ctypes.c_int, [vp, ctypes.POINTER(Mis2SweepRecord), i32,
                                            ctypes.POINTER(i32)]),
        "mis2_quotient": (ctypes.c_int, [vp, gp, vp, i64, vp, vp, ctypes.POINTER(i64), vp]),
        "mis2_galerkin_workspace_bytes": (ctypes.c_int, [i64, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_galerkin": (ctypes.c_int, [vp, gp, vp, vp, vp, gp, vp, vp, vp]),
        "mis2_coarsen_workspace_bytes": (ctypes.c_int, [i64, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_coarsen": (ctypes.c_int, [vp, gp, u64, i64, i32, vp, i64, ctypes.POINTER(i64),
                                        ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i32), vp]),
        "mis2_server_bytes": (ctypes.c_int, [i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_server_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t,
                                              i64, i64, i32, u64, i64, i32]),
        "mis2_server_destroy": (None, [vp]),
        "mis2_server_last_error": (ctypes.c_char_p, [vp]),
        "mis2_server_submit": (ctypes.c_int, [vp, gp, vp, i64, i64]),
        "mis2_server_step": (ctypes.c_int, [vp, vp, ctypes.POINTER(i32)]),
        "mis2_server_poll": (ctypes.c_int, [vp, ctypes.POINTER(Mis2JobResult), i32,
                                            ctypes.POINTER(i32)]),
        "mis2_batch_workspace_bytes": (ctypes.c_int, [i32, i64, i64,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
        "mis2_aggregate_batched": (ctypes.c_int, [vp, gp, i32, ctypes.POINTER(i64), u64, i64, i32,
                                                  vp, i64, ctypes.POINTER(i64),
                                                  ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                  ctypes.POINTER(i32), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
