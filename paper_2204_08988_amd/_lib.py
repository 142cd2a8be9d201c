"""ctypes declarations of the C ABI in include/dpmm.h.

Loads paper_2204_08988_amd/libdpmm.so (built in-tree by build.py).  There is
no fallback: if the library is missing or does not load, every entry point
raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpmm.so")

DPMM_OK = 0
STATUS = {0: "DPMM_OK", -1: "DPMM_E_ARG", -2: "DPMM_E_SHAPE", -3: "DPMM_E_CAPACITY",
          -4: "DPMM_E_NUMERIC", -5: "DPMM_E_DEVICE", -6: "DPMM_E_OOM", -7: "DPMM_E_STATE"}
GAUSSIAN, MULTINOMIAL, POISSON = 0, 1, 2
FP32, BF16, BF16X3 = 0, 1, 2
MERGE_PAPER, MERGE_INVERSE_SPLIT = 0, 1

# every symbol include/dpmm.h declares
EXPORTS = [
    "dpmm_create", "dpmm_destroy", "dpmm_last_error", "dpmm_status_string", "dpmm_init_labels",
    "dpmm_set_state", "dpmm_get_state", "dpmm_set_params", "dpmm_get_params", "dpmm_set_stats",
    "dpmm_get_stats", "dpmm_loglik", "dpmm_sample_labels", "dpmm_suffstats", "dpmm_sample_params",
    "dpmm_split_merge", "dpmm_step", "dpmm_mlp_n_params", "dpmm_mlp_set_weights", "dpmm_mlp_get_weights",
    "dpmm_mlp_forward", "dpmm_mlp_grad", "dpmm_mlp_adam_step", "dpmm_set_features", "dpmm_learned_move",
    "dpmm_mlp_train", "dpmm_mlp_training_set", "dpmm_suffstats_static", "dpmm_nmi", "dpmm_fit",
    "dpmm_save_checkpoint", "dpmm_load_checkpoint",
]


class Config(ctypes.Structure):
    _fields_ = [
        ("family", ctypes.c_int32), ("d", ctypes.c_int32), ("k_max", ctypes.c_int32),
        ("burn_out", ctypes.c_int32), ("alpha", ctypes.c_double), ("kappa", ctypes.c_double),
        ("nu", ctypes.c_double), ("m", ctypes.POINTER(ctypes.c_double)),
        ("psi", ctypes.POINTER(ctypes.c_double)), ("beta", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("merge_form", ctypes.c_int32),
        ("learned", ctypes.c_int32), ("gamma_shape", ctypes.POINTER(ctypes.c_double)),
        ("gamma_rate", ctypes.POINTER(ctypes.c_double)), ("sparse", ctypes.c_int32),
    ]


class CSR(ctypes.Structure):
    """dpmm_csr: count rows in compressed sparse rows (device arrays)."""
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("nnz", ctypes.c_int64)]


class IterInfo(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("splits", ctypes.c_int32), ("merges", ctypes.c_int32),
        ("removed", ctypes.c_int32), ("logpost", ctypes.c_double), ("ms_params", ctypes.c_float),
        ("ms_labels", ctypes.c_float), ("ms_sort", ctypes.c_float), ("ms_stats", ctypes.c_float),
        ("ms_splitmerge", ctypes.c_float), ("learned_kind", ctypes.c_int32),
        ("learned_accepted", ctypes.c_int32), ("ms_learned", ctypes.c_float),
        ("ms_label_kernel", ctypes.c_float),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LearnedInfo(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("k1", ctypes.c_int32), ("k2", ctypes.c_int32),
        ("accepted", ctypes.c_int32), ("skipped", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("n_a", ctypes.c_int64), ("n_b", ctypes.c_int64), ("log_target", ctypes.c_double),
        ("log_q_part", ctypes.c_double), ("log_h", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class FitOptions(ctypes.Structure):
    _fields_ = [
        ("t0", ctypes.c_uint32), ("iters", ctypes.c_int32), ("train_every", ctypes.c_int32),
        ("train_until", ctypes.c_int32), ("train_steps", ctypes.c_int32), ("train_batch", ctypes.c_int32),
        ("train_lr", ctypes.c_float), ("reserved", ctypes.c_int32),
    ]


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2204_08988_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)
    sig = {
        "dpmm_create": ([ctypes.POINTER(Config), vp, ctypes.POINTER(vp)], i32),
        "dpmm_destroy": ([vp], None),
        "dpmm_last_error": ([vp], ctypes.c_char_p),
        "dpmm_status_string": ([i32], ctypes.c_char_p),
        "dpmm_init_labels": ([vp, i64, vp, vp], i32),
        "dpmm_set_state": ([vp, i32, ctypes.POINTER(i32)], i32),
        "dpmm_get_state": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "dpmm_set_params": ([vp, i32, dp, dp, dp], i32),
        "dpmm_get_params": ([vp, dp, dp, dp], i32),
        "dpmm_set_stats": ([vp, i32, vp], i32),
        "dpmm_get_stats": ([vp, vp], i32),
        "dpmm_loglik": ([vp, vp, i64, vp], i32),
        "dpmm_sample_labels": ([vp, vp, i64, u32, vp, vp], i32),
        "dpmm_suffstats": ([vp, vp, i64, vp, vp], i32),
        "dpmm_suffstats_static": ([vp, vp, i64, vp, vp], i32),
        "dpmm_nmi": ([vp, vp, i64, dp], i32),
        "dpmm_fit": ([vp, vp, i64, ctypes.POINTER(FitOptions), vp, vp, ctypes.POINTER(IterInfo), dp], i32),
        "dpmm_save_checkpoint": ([vp, ctypes.c_char_p, i64, u32, vp, vp], i32),
        "dpmm_load_checkpoint": ([vp, ctypes.c_char_p, i64, ctypes.POINTER(u32), vp, vp], i32),
        "dpmm_sample_params": ([vp, u32], i32),
        "dpmm_split_merge": ([vp, vp, i64, u32, vp, vp, ctypes.POINTER(IterInfo)], i32),
        "dpmm_step": ([vp, vp, i64, u32, vp, vp, ctypes.POINTER(IterInfo)], i32),
        "dpmm_mlp_n_params": ([vp], i64),
        "dpmm_mlp_set_weights": ([vp, dp], i32),
        "dpmm_mlp_get_weights": ([vp, dp], i32),
        "dpmm_mlp_forward": ([vp, vp, i64, vp], i32),
        "dpmm_mlp_grad": ([vp, vp, vp, i64, dp, dp], i32),
        "dpmm_mlp_adam_step": ([vp, vp, vp, i64, ctypes.c_float, dp], i32),
        "dpmm_set_features": ([vp, vp, i64, vp, i32, i32, vp, vp, i64, ctypes.POINTER(i64)], i32),
        "dpmm_learned_move": ([vp, vp, i64, u32, vp, vp, vp, ctypes.POINTER(LearnedInfo)], i32),
        "dpmm_mlp_train": ([vp, vp, i64, vp, vp, i32, i32, ctypes.c_float, dp], i32),
        "dpmm_mlp_training_set": ([vp, vp, i64, vp, vp, vp, vp, vp, i64, ctypes.POINTER(i64)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class DpmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def nmi(a, b):
    """Normalised mutual information of two host labelings (dpmm_nmi)."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32).ravel()
    b = np.ascontiguousarray(b, dtype=np.int32).ravel()
    if a.size != b.size:
        raise ValueError("label vectors differ in length")
    out = ctypes.c_double()
    s = lib().dpmm_nmi(a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p), a.size,
                       ctypes.byref(out))
    if s != DPMM_OK:
        raise DpmmError(s, "dpmm_nmi")
    return out.value
