"""ctypes declarations of the C ABI in include/etest.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetest.so")

OK, EINVAL, ENONFINITE, ENOMEM, EDEVICE, EBUSY, ENOTFOUND = range(7)
PREC_F64, PREC_F32, PREC_BF16_REFINED = 0, 1, 2
ED, MMD = 0, 1
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENONFINITE", 3: "ENOMEM", 4: "EDEVICE", 5: "EBUSY",
                6: "ENOTFOUND"}

c_i32, c_i64, c_u64, c_dbl, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_void_p)


class Result(ctypes.Structure):
    _fields_ = [("statistic", c_dbl), ("threshold", c_dbl), ("p_value", c_dbl),
                ("count_ge", c_i64), ("B", c_i64), ("n_refined", c_i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CrossResult(ctypes.Structure):
    _fields_ = [("statistic", c_dbl), ("sigma", c_dbl), ("z", c_dbl), ("p_value", c_dbl),
                ("n_refined", c_i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("prec", c_i32), ("nx", c_i64), ("ny", c_i64), ("p", c_i64),
                ("B", c_i64), ("seed", c_u64), ("gamma", c_dbl), ("X", c_vp), ("Y", c_vp),
                ("perm_stats", c_vp)]


class HsicRequest(ctypes.Structure):
    _fields_ = [("prec", c_i32), ("reserved", c_i32), ("n", c_i64), ("p", c_i64), ("q", c_i64),
                ("B", c_i64), ("seed", c_u64), ("gamma_x", c_dbl), ("gamma_y", c_dbl),
                ("X", c_vp), ("Y", c_vp), ("perm_stats", c_vp)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", c_i64), ("max_resident", c_i32), ("max_queue", c_i32),
                ("chunk_updates", c_i64)]


# (name, restype, argtypes) for every function the header declares
SIGNATURES = [
    ("ed_test", c_i32, [c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_u64, c_i32, c_vp,
                        ctypes.POINTER(Result)]),
    ("mmd_test", c_i32, [c_vp, c_i64, c_vp, c_i64, c_i64, c_dbl, c_i64, c_u64, c_i32, c_vp,
                         ctypes.POINTER(Result)]),
    ("ed_test_f64", c_i32, [c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_u64, c_vp,
                            ctypes.POINTER(Result)]),
    ("mmd_test_f64", c_i32, [c_vp, c_i64, c_vp, c_i64, c_i64, c_dbl, c_i64, c_u64, c_vp,
                             ctypes.POINTER(Result)]),
    ("etest_run", c_i32, [ctypes.POINTER(Request), c_vp, ctypes.POINTER(Result)]),
    ("etest_cross", c_i32, [ctypes.POINTER(Request), c_vp, ctypes.POINTER(CrossResult)]),
    ("etest_standard", c_i32, [ctypes.POINTER(Request), c_vp, ctypes.POINTER(Result)]),
    ("etest_hsic", c_i32, [ctypes.POINTER(HsicRequest), c_vp, ctypes.POINTER(Result)]),
    ("etest_permutations", c_i32, [c_i64, c_u64, c_i64, c_i64, c_vp, c_vp]),
    ("etest_precomputed", c_i32, [ctypes.POINTER(Request), c_vp, ctypes.POINTER(Result)]),
    ("etest_precomputed_dense", c_i32, [ctypes.POINTER(Request), c_vp, ctypes.POINTER(Result)]),
    ("ed_test_async", c_i32, [ctypes.POINTER(Request), c_vp, c_vp]),
    ("mmd_test_async", c_i32, [ctypes.POINTER(Request), c_vp, c_vp]),
    ("etest_run_async_noalloc", c_i32, [ctypes.POINTER(Request), c_vp, c_vp]),
    ("etest_batch", c_i32, [ctypes.POINTER(Request), c_i64, c_vp, ctypes.POINTER(Result)]),
    ("etest_batch_async", c_i32, [ctypes.POINTER(Request), c_i64, c_vp, c_vp]),
    ("etest_membership", c_i32, [c_i64, c_i64, c_u64, c_i64, c_i64, c_vp, c_vp]),
    ("etest_blocks", c_i32, [ctypes.POINTER(Request), c_vp, c_vp, c_vp, c_vp]),
    ("etest_perm_stats_from_membership", c_i32, [ctypes.POINTER(Request), c_vp, c_i64, c_vp,
                                                 c_vp, ctypes.POINTER(Result)]),
    ("etest_server_create", c_i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(c_vp)]),
    ("etest_server_submit", c_i32, [c_vp, ctypes.POINTER(Request), ctypes.POINTER(c_u64)]),
    ("etest_server_poll", c_i32, [c_vp, c_u64, ctypes.POINTER(Result)]),
    ("etest_server_wait", c_i32, [c_vp, c_u64, ctypes.POINTER(Result)]),
    ("etest_server_stats", c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                   ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    ("etest_server_destroy", c_i32, [c_vp]),
    ("etest_last_error", ctypes.c_char_p, []),
    ("etest_footprint", c_i32, [ctypes.POINTER(Request), ctypes.POINTER(c_i64)]),
    ("etest_validate", c_i32, [ctypes.POINTER(Request)]),
    ("etest_profile_enable", c_i32, [c_i32]),
    ("etest_profile_read", c_i32, [ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64), c_i32]),
    ("etest_tune_set", c_i32, [c_i32, c_i64, c_i64, c_i32, c_i32]),
    ("etest_tune_clear", c_i32, []),
    ("etest_tune_set_gram", c_i32, [c_i32, c_i64, c_i64, c_i32]),
]

STAGES = ["staging", "blocks", "splits", "sums", "centring", "resampling", "finalize"]

_lib = None


class EtestError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def load():
    """Load the in-tree HIP library; there is no fallback if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libetest.so is not built (run paper_2406_06488_amd/build.py); "
                               "this package has no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise EtestError(status, load().etest_last_error().decode())
    return status
