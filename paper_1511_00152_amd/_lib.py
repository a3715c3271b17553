"""ctypes binding of libpds.so (the C ABI in include/pds.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Importing this module fails loudly when the library has not been
built; there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpds.so")

PDS_OK = 0
PDS_E_ARG = -1
PDS_E_UNSUPPORTED = -2
PDS_E_M = -3
PDS_E_WORKSPACE = -4
PDS_E_HIP = -5

PDS_F64 = 0
PDS_F32 = 1
PDS_SPLIT_BF16 = 2

PDS_GRAM_AUTO = 0
PDS_GRAM_DENSE = 1
PDS_GRAM_SPARSE = 2

PDS_TRANSFORM_HADAMARD = 0
PDS_TRANSFORM_DCT = 1
PDS_DCT_MAX_P = 8192

PDS_OP_COMPRESS = 0
PDS_OP_COVARIANCE = 1
PDS_OP_KMEANS = 2
PDS_OP_KMEANS2 = 3
PDS_OP_MEAN = 4
PDS_OP_KMEANSPP = 5
PDS_OP_KMEANS_BEST = 6
PDS_OP_KMEANS_RUN = 7
PDS_EXPLAINED_WS_BYTES = 16384
PDS_NOALLOC_SCRATCH_BYTES = 64 << 20

# every entry point declared in include/pds.h
EXPORTS = (
    "pds_plan_create", "pds_plan_create_dct", "pds_plan_transform", "pds_plan_destroy", "pds_plan_set_gram", "pds_plan_gram", "pds_signs", "pds_workspace_size", "pds_covariance_acc_size",
    "pds_compress", "pds_covariance", "pds_kmeans_step", "pds_kmeans_run", "pds_kmeans_step_noalloc", "pds_unmix", "pds_kmeans_2pass", "pds_sample_mean", "pds_explained_variance", "pds_kmeanspp", "pds_kmeans_best", "pds_pad_rows", "pds_profile_enable", "pds_profile_report",
    "pds_last_error", "pds_version",
    "pds_row_moments", "pds_frob_diff", "pds_msel_workspace_size", "pds_msel_label", "pds_msel_features",
    "pds_mlp_param_count", "pds_mlp_forward", "pds_mlp_backward", "pds_mlp_adam", "pds_mlp_pack_bf16",
    "pds_msel_predict",
    "pds_batch_create", "pds_batch_destroy", "pds_batch_workspace_size", "pds_batch_bind", "pds_batch_compress",
    "pds_batch_init_centers", "pds_batch_kmeans", "pds_batch_autotune", "pds_batch_info",
)


class PdsBatchDesc(ctypes.Structure):
    """pds_batch_desc (include/pds.h)."""
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("ldx", ctypes.c_int64), ("p", ctypes.c_int32),
                ("m", ctypes.c_int32), ("K", ctypes.c_int32), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("vals", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("centers", ctypes.c_void_p),
                ("centers_alt", ctypes.c_void_p), ("assign", ctypes.c_void_p), ("objective", ctypes.c_void_p)]

PDS_FROB_WS_BYTES = 4096


class PdsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().pds_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpds.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    u64 = ctypes.c_uint64
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    st = ctypes.c_int
    L.pds_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, u64, i32]
    L.pds_plan_create_dct.argtypes = [ctypes.POINTER(P), i64, i64, u64, i32]
    L.pds_plan_transform.argtypes = [P, ctypes.POINTER(i32)]
    L.pds_plan_destroy.argtypes = [P]
    L.pds_plan_set_gram.argtypes = [P, i32]
    L.pds_plan_gram.argtypes = [P, i64, ctypes.POINTER(i32)]
    L.pds_signs.argtypes = [P, P]
    L.pds_workspace_size.argtypes = [P, i32, i64, i32, ctypes.POINTER(sz)]
    L.pds_covariance_acc_size.argtypes = [P, ctypes.POINTER(sz)]
    L.pds_compress.argtypes = [P, P, i64, i64, u64, P, P, P, sz, P]
    L.pds_covariance.argtypes = [P, P, P, i64, P, i32, i64, P, P, sz, P]
    L.pds_kmeans_step.argtypes = [P, P, P, i64, i32, P, P, P, P, P, sz, P]
    L.pds_kmeans_run.argtypes = [P, P, P, i64, i32, i32, P, P, P, P, P, sz, P]
    L.pds_kmeans_step_noalloc.argtypes = [P, P, P, i64, i32, P, P, P, P, P]
    L.pds_unmix.argtypes = [P, P, i32, P, P]
    L.pds_kmeans_2pass.argtypes = [P, P, i64, i64, i32, P, P, P, P, P, sz, P]
    L.pds_sample_mean.argtypes = [P, P, P, i64, P, i32, i64, P, P, sz, P]
    L.pds_kmeanspp.argtypes = [P, P, P, i64, i32, i32, P, P, P, sz, P]
    L.pds_kmeans_best.argtypes = [P, P, P, i64, i32, i32, i32, P, P, P, P, P, sz, P]
    L.pds_pad_rows.argtypes = [P, i32, i64, i64, i64, P, i64, P]
    L.pds_explained_variance.argtypes = [P, i32, P, i32, i64, i64, i64, P, P, sz, P]
    L.pds_profile_enable.argtypes = [i32]
    L.pds_profile_report.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    f32 = ctypes.c_float
    f64 = ctypes.c_double
    L.pds_row_moments.argtypes = [P, i64, i64, i64, P, P]
    L.pds_frob_diff.argtypes = [P, P, i64, P, P, sz, P]
    L.pds_msel_workspace_size.argtypes = [P, i64, ctypes.POINTER(sz)]
    L.pds_msel_label.argtypes = [P, P, i64, i64, f64, P, P, P, sz, P]
    L.pds_msel_features.argtypes = [P, P, i64, i64, i64, f64, P, P, sz, P]
    L.pds_mlp_param_count.argtypes = []
    L.pds_mlp_forward.argtypes = [P, P, P, P, i64, P, P, P]
    L.pds_mlp_backward.argtypes = [P, P, P, P, i64, f32, P, sz, P, P, P]
    L.pds_mlp_adam.argtypes = [P, P, P, P, i32, f32, f32, f32, f32, P]
    L.pds_mlp_pack_bf16.argtypes = [P, P, P]
    L.pds_msel_predict.argtypes = [P, P, P, P, i64, f32, f32, f32, P, P]
    L.pds_batch_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(PdsBatchDesc), i32, i32]
    L.pds_batch_destroy.argtypes = [P]
    L.pds_batch_workspace_size.argtypes = [P, ctypes.POINTER(sz)]
    L.pds_batch_bind.argtypes = [P, P, sz, P]
    L.pds_batch_compress.argtypes = [P, P]
    L.pds_batch_init_centers.argtypes = [P, P]
    L.pds_batch_kmeans.argtypes = [P, P]
    L.pds_batch_autotune.argtypes = [P, P]
    L.pds_batch_info.argtypes = [P, ctypes.c_char_p, sz]
    L.pds_last_error.restype = ctypes.c_char_p
    L.pds_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("pds_last_error", "pds_version"):
            f.restype = st
    _lib = L
    return L


def check(status, where):
    if status != PDS_OK:
        raise PdsError(status, where)
