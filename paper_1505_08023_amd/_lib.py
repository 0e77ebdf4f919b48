"""ctypes declarations of the C ABI in include/mfe.h (argument marshalling only).

Every name here is the C entry point of the same name.  Loading fails loudly
when libmfe.so has not been built: there is no fallback path.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfe.so")

MFE_OK, MFE_NOT_CONVERGED = 0, 1
MFE_EINVAL, MFE_ENOMEM, MFE_EHIP, MFE_EBREAKDOWN, MFE_EUNSUPPORTED = -1, -2, -3, -4, -5
MFE_CSR, MFE_BCRS13 = 1, 2
MFE_F64, MFE_F32 = 1, 2
MFE_MIXED_WARM, MFE_MIXED_KEEP_DIRECTION = 1, 2

STATUS_NAMES = {0: "MFE_OK", 1: "MFE_NOT_CONVERGED", -1: "MFE_EINVAL", -2: "MFE_ENOMEM",
                -3: "MFE_EHIP", -4: "MFE_EBREAKDOWN", -5: "MFE_EUNSUPPORTED"}

c_int, c_i32, c_i64, c_dbl, c_vp, c_size = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t)


class mfe_cg_stats(ctypes.Structure):
    _fields_ = [("status", c_i32), ("iterations", c_i32), ("outer", c_i32), ("spmv_count", c_i32),
                ("rel_res_recurrence", c_dbl), ("rel_res_true", c_dbl), ("seconds", c_dbl),
                ("guess_rejected", c_i32), ("reserved_", c_i32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


mfe_alloc_fn = ctypes.CFUNCTYPE(c_vp, c_size, c_vp)
mfe_free_fn = ctypes.CFUNCTYPE(None, c_vp, c_vp)

PP = ctypes.POINTER(c_vp)

# name -> (restype, argtypes)
SIGNATURES = {
    "mfe_last_error": (ctypes.c_char_p, []),
    "mfe_version": (c_int, []),
    "mfe_ctx_create": (c_int, [c_int, c_vp, mfe_alloc_fn, mfe_free_fn, c_vp, PP]),
    "mfe_ctx_destroy": (c_int, [c_vp]),
    "mfe_problem_create": (c_int, [c_vp, c_int, c_int, c_int, c_vp, c_vp, c_int, c_int, PP]),
    "mfe_problem_from_csr": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_int, c_int, PP]),
    "mfe_problem_from_csr_host": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_int, c_int, PP]),
    "mfe_problem_export_csr_host": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mfe_rhs": (c_int, [c_vp, c_vp]),
    "mfe_problem_set_bc": (c_int, [c_vp, c_vp, c_vp]),
    "mfe_problem_info": (c_int, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "mfe_problem_csr_layout": (c_int, [c_vp] + [ctypes.POINTER(c_i64)] * 3),
    "mfe_problem_csr_groups": (c_int, [c_vp] + [ctypes.POINTER(c_i64)] * 4),
    "mfe_problem_bcrs13_layout": (c_int, [c_vp] + [ctypes.POINTER(c_i64)] * 4),
    "mfe_batch_bcrs13_layout": (c_int, [c_vp] + [ctypes.POINTER(c_i64)] * 4),
    "mfe_problem_export_csr": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mfe_problem_export_bcrs13": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "mfe_problem_destroy": (c_int, [c_vp]),
    "mfe_spmv": (c_int, [c_vp, c_int, c_vp, c_vp]),
    "mfe_spmv_f32": (c_int, [c_vp, c_int, c_vp, c_vp]),
    "mfe_spmv_dot": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mfe_spmv_dot_noalloc": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp]),
    "mfe_dot": (c_int, [c_vp, c_i64, c_vp, c_vp, ctypes.POINTER(c_dbl)]),
    "mfe_cg_mixed_warm": (c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_int, c_int, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_cg_mixed_ex": (c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_int, c_int, c_int, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_prolong_trilinear": (c_int, [c_vp, c_int, c_int, c_int, c_vp, c_int, c_vp, c_vp]),
    "mfe_stream_probe": (c_int, [c_vp, c_int, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "mfe_cg": (c_int, [c_vp, c_int, c_vp, c_dbl, c_int, c_vp, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_spmv_dot_f32": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mfe_cg_warm": (c_int, [c_vp, c_int, c_vp, c_dbl, c_int, c_vp, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_cg_single_reduction": (c_int, [c_vp, c_int, c_vp, c_dbl, c_int, c_vp, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_cg_jacobi": (c_int, [c_vp, c_int, c_vp, c_dbl, c_int, c_vp, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_verify_series": (c_int, [c_vp, c_vp, c_dbl, c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                                  ctypes.POINTER(ctypes.c_int64)]),
    "mfe_cg_mixed": (c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_int, c_int, ctypes.POINTER(mfe_cg_stats)]),
    "mfe_batch_create": (c_int, [c_vp, c_int, c_vp, c_vp, c_int, c_int, PP]),
    "mfe_batch_destroy": (c_int, [c_vp]),
    "mfe_batch_from_problems": (c_int, [c_vp, c_int, c_vp, c_int, c_int, PP]),
    "mfe_cg_batched": (c_int, [c_vp, c_int, c_vp, c_int, c_vp, c_dbl, c_int, c_int, c_vp]),
    "mfe_batch_info": (c_int, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_vp]),
    "mfe_batch_export_csr": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "mfe_batch_set_bc": (c_int, [c_vp, c_vp, c_vp]),
    "mfe_batch_autotune": (c_int, [c_vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "mfe_batch_cg": (c_int, [c_vp, c_int, c_vp, c_dbl, c_int, c_vp]),
    "mfe_batch_cg_mixed": (c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_int, c_int, c_vp]),
    "mfe_batch_cg_mixed_ex": (c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_int, c_int, c_int, c_vp]),
    "mfe_net_create": (c_int, [c_vp, c_int, c_int, PP]),
    "mfe_net_destroy": (c_int, [c_vp]),
    "mfe_net_num_params": (c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "mfe_net_set_params": (c_int, [c_vp, c_vp]),
    "mfe_net_get_params": (c_int, [c_vp, c_vp]),
    "mfe_net_forward": (c_int, [c_vp, c_int, c_vp, c_vp]),
    "mfe_net_loss_grad": (c_int, [c_vp, c_int, c_vp, c_vp, ctypes.POINTER(c_dbl), c_vp]),
    "mfe_net_loss_grad_energy": (c_int, [c_vp, c_vp, c_int, c_int, c_vp, c_vp, ctypes.POINTER(c_dbl), c_vp]),
    "mfe_net_set_grad": (c_int, [c_vp, c_vp]),
    "mfe_net_adam_step": (c_int, [c_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "mfe_net_predict_x0": (c_int, [c_vp, c_vp, c_vp]),
    "mfe_conv3d_bf16": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_vp]),
    "mfe_conv3d_dgrad_bf16": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp, c_vp]),
    "mfe_conv3d_wgrad_bf16": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_vp]),
}

_lib = None


def load():
    """Load libmfe.so and declare every entry point.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1505_08023_amd.build` "
                           "(the HIP library is the only implementation; there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MfeError(RuntimeError):
    def __init__(self, code, where):
        msg = load().mfe_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, where, ok=(MFE_OK,)):
    if code not in ok:
        raise MfeError(code, where)
    return code


def __getattr__(name):
    # mfe_* names resolve to the C entry points
    if name.startswith("mfe_") and name in SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
