"""ctypes binding of libosvmbe.so (include/osv.h).  Argument marshalling only:
every step of the hot path runs in the HIP library.  Importing this module on a
machine without the built library raises; there is no fallback path."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libosvmbe.so")

OSV_OK, OSV_E_ARG, OSV_E_HIP, OSV_E_NOMEM = 0, -1, -2, -3
OSV_E_NOT_CONVERGED, OSV_E_NONFINITE, OSV_E_STATE, OSV_E_DOMAIN = -4, -5, -6, -7
OSV_FP64, OSV_MIXED = 0, 1
OSV_SEL_DISTANCE, OSV_SEL_OVERLAP, OSV_SEL_FULL = 0, 1, 2
OSV_DT_F64, OSV_DT_F32 = 0, 1
OSV_MAX_DOMAIN = 100
OSV_NOALLOC_MAX_WEAK = 1 << 20
TUNING_KEYS = {"gemm_ks": (8, 16, 32), "prep_nt_small": (128, 256), "prep_nt_mid": (256, 512, 1024),
               "prep_nt_big": (512, 1024), "cpl_split": (0, 64), "solve_split": (0, 1)}

EXPORTS = ["osv_build_pairs", "osv_query", "osv_solve_clusters", "osv_energy", "osv_weak_pairs",
           "osv_weak_pairs_noalloc", "osv_generate_osvs", "osv_high_order_correction",
           "osv_response_layout", "osv_response", "osv_weak_response", "osv_correction_stats",
           "osv_generation_stats",
           "osv_set_tuning", "osv_get_tuning", "osv_load_tuning", "osv_build_pairs_exact",
           "osv_densities",
           "osv_plan_clusters", "osv_destroy", "osv_status_string", "osv_last_error",
           "osv_stage_times", "osv_stage_flops", "osv_release_cached_memory", "osv_cached_bytes"]


class OsvSystem(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int32), ("nvir", ctypes.c_int32), ("naux", ctypes.c_int32),
                ("r", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("C_dtype", ctypes.c_int32), ("eps_vir", ctypes.c_void_p),
                ("F_occ", ctypes.c_void_p), ("centroid", ctypes.c_void_p)]


class OsvSelect(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("cut2", ctypes.c_double), ("cut3", ctypes.c_double),
                ("l2b", ctypes.c_double), ("l3b", ctypes.c_double), ("tau_S", ctypes.c_double)]


class OsvCounts(ctypes.Structure):
    _fields_ = [("n1b", ctypes.c_int64), ("n2b", ctypes.c_int64), ("n3b", ctypes.c_int64),
                ("n_clusters", ctypes.c_int64), ("n_pair_blocks", ctypes.c_int64),
                ("n_domains", ctypes.c_int64), ("n_couplings", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class OsvSolveInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("max_residual", ctypes.c_double),
                ("converged", ctypes.c_int32), ("n_not_converged", ctypes.c_int64)]


class OSVError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load the built library (raises if it is missing: no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2106_06149_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.osv_build_pairs.argtypes = [ctypes.POINTER(OsvSystem), ctypes.POINTER(OsvSelect), i32, vp,
                                    ctypes.POINTER(vp)]
    lib.osv_build_pairs.restype = ctypes.c_int
    lib.osv_build_pairs_exact.argtypes = [ctypes.POINTER(OsvSystem), vp, ctypes.POINTER(OsvSelect), i32, vp,
                                          ctypes.POINTER(vp)]
    lib.osv_build_pairs_exact.restype = ctypes.c_int
    lib.osv_query.argtypes = [vp, ctypes.POINTER(OsvCounts)]
    lib.osv_query.restype = ctypes.c_int
    lib.osv_solve_clusters.argtypes = [vp, dbl, i32, vp, ctypes.POINTER(OsvSolveInfo)]
    lib.osv_solve_clusters.restype = ctypes.c_int
    lib.osv_energy.argtypes = [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp]
    lib.osv_energy.restype = ctypes.c_int
    lib.osv_densities.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.osv_densities.restype = ctypes.c_int
    lib.osv_weak_pairs.argtypes = [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64), vp, vp]
    lib.osv_weak_pairs.restype = ctypes.c_int
    lib.osv_weak_pairs_noalloc.argtypes = [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64), vp, vp]
    lib.osv_weak_pairs_noalloc.restype = ctypes.c_int
    lib.osv_generate_osvs.argtypes = [i32, i32, i32, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp]
    lib.osv_generate_osvs.restype = ctypes.c_int
    lib.osv_high_order_correction.argtypes = [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                              ctypes.POINTER(dbl), vp]
    lib.osv_high_order_correction.restype = ctypes.c_int
    lib.osv_response_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), vp, vp]
    lib.osv_response_layout.restype = ctypes.c_int
    lib.osv_response.argtypes = [vp, vp, vp, vp]
    lib.osv_response.restype = ctypes.c_int
    lib.osv_weak_response.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
    lib.osv_weak_response.restype = ctypes.c_int
    lib.osv_correction_stats.argtypes = [vp, vp]
    lib.osv_correction_stats.restype = ctypes.c_int
    lib.osv_generation_stats.argtypes = [vp]
    lib.osv_generation_stats.restype = ctypes.c_int
    lib.osv_set_tuning.argtypes = [ctypes.c_char_p, i32]
    lib.osv_set_tuning.restype = ctypes.c_int
    lib.osv_get_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    lib.osv_get_tuning.restype = ctypes.c_int
    lib.osv_load_tuning.argtypes = [ctypes.c_char_p]
    lib.osv_load_tuning.restype = ctypes.c_int
    lib.osv_plan_clusters.argtypes = [i32, vp, ctypes.POINTER(OsvSelect), ctypes.POINTER(OsvCounts),
                                      vp, vp, i64]
    lib.osv_plan_clusters.restype = ctypes.c_int
    lib.osv_destroy.argtypes = [vp]
    lib.osv_destroy.restype = None
    lib.osv_status_string.argtypes = [ctypes.c_int]
    lib.osv_status_string.restype = ctypes.c_char_p
    lib.osv_last_error.argtypes = [vp]
    lib.osv_last_error.restype = ctypes.c_char_p
    lib.osv_stage_times.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.osv_stage_times.restype = ctypes.c_int
    lib.osv_stage_flops.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.osv_stage_flops.restype = ctypes.c_int
    lib.osv_release_cached_memory.argtypes = [i32]
    lib.osv_release_cached_memory.restype = ctypes.c_int
    lib.osv_cached_bytes.argtypes = [i32]
    lib.osv_cached_bytes.restype = ctypes.c_int64
    _lib = lib
    return lib


def check(status, ctx=None):
    if status != OSV_OK:
        lib = load()
        msg = lib.osv_last_error(ctx).decode()
        raise OSVError(status, f"{lib.osv_status_string(status).decode()}: {msg}")
