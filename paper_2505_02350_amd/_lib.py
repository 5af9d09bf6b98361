"""ctypes binding of the C ABI declared in ``include/erbf.h``.

Argument marshalling only: every step of the computation runs in the HIP
library ``liberbf.so``.  Torch tensors supply device memory and streams.
Loading fails loudly when the library has not been built.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liberbf.so")

MAX_LEVELS = 8

ERBF_OK = 0
ERBF_ERR_INVALID_ARG = -1
ERBF_ERR_HIP = -2
ERBF_ERR_WORKSPACE = -3
ERBF_ERR_CAPACITY = -4
ERBF_ERR_UNSUPPORTED = -5
ERBF_ERR_STATE = -6

FLAG_BUCKET_OVERFLOW = 1

MODE_FIXED, MODE_DYNAMIC, MODE_L2 = 0, 1, 2
WEIGHT_SIGNED_SQUARE, WEIGHT_LINEAR = 0, 1
ORIENT_QUATERNION, ORIENT_EULER = 0, 1
VARIANT_FWD_PERSISTENT, VARIANT_BWD_PERSISTENT, VARIANT_FUSED, N_VARIANTS = 1, 2, 4, 8
ABI_VERSION = 7


class ErbfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"erbf error {code}: {msg}")
        self.code = code


class ShapeDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("level_n", ctypes.c_int32 * MAX_LEVELS),
                ("m_cap", ctypes.c_int32), ("level_samples", ctypes.c_int32 * MAX_LEVELS)]


class Config(ctypes.Structure):
    _fields_ = [("n_shapes", ctypes.c_int32), ("shapes", ctypes.POINTER(ShapeDesc)),
                ("pair_cap", ctypes.c_int64), ("cull_k", ctypes.c_float),
                ("weight_map", ctypes.c_int32), ("orientation", ctypes.c_int32), ("batch_cap", ctypes.c_int32)]


class Level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("axis", ctypes.c_void_p), ("target", ctypes.c_void_p),
                ("sdf", ctypes.c_void_p), ("active_bits", ctypes.c_void_p), ("samples", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("m_dev", ctypes.c_void_p)]


class LossCfg(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("lambda_", ctypes.c_float), ("lambda_dev", ctypes.c_void_p),
                ("l1_active", ctypes.c_int32), ("tau1", ctypes.c_float), ("tau2", ctypes.c_float),
                ("tau_m", ctypes.c_float), ("l1_active_dev", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("L2", ctypes.c_double), ("L1", ctypes.c_double), ("loss", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("n_idall", ctypes.c_int64),
                ("P_fwd", ctypes.c_int64), ("P_bwd", ctypes.c_int64), ("n_bucket_pairs", ctypes.c_int64),
                ("max_abs_E", ctypes.c_float), ("m", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("P_fwd_total", ctypes.c_int64), ("P_bwd_total", ctypes.c_int64),
                ("calls", ctypes.c_int64)]


class AdamCfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("lr_dev", ctypes.c_void_p), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("hold_dev", ctypes.c_void_p)]


class SeedCfg(ctypes.Structure):
    _fields_ = [("top_frac", ctypes.c_float), ("k_new", ctypes.c_int32), ("r_nms", ctypes.c_float),
                ("eps", ctypes.c_float), ("min_abs_err", ctypes.c_float), ("w_rule", ctypes.c_int32)]


class SchedCfg(ctypes.Structure):
    _fields_ = [("k_l2", ctypes.c_int32), ("tau_l2", ctypes.c_float), ("k_l1", ctypes.c_int32),
                ("tau_l1", ctypes.c_float), ("tau_d", ctypes.c_float), ("T_e", ctypes.c_int32),
                ("M_e", ctypes.c_int32), ("lr0", ctypes.c_float), ("lr_final", ctypes.c_float),
                ("lr_min", ctypes.c_float), ("refine_epochs", ctypes.c_int32 * 4)]


class SchedState(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("epoch", "l1_active", "final_phase", "add_request", "refine_request", "b_f", "n_pruned", "lr",
                 "l2_ring", "bf_ring", "hold")]


STATS_BYTES = ctypes.sizeof(Stats)

# (name, restype, argtypes) of every exported symbol of include/erbf.h
class LaunchCfg(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("slot_chunk", ctypes.c_int32), ("samp_split", ctypes.c_int32),
                ("bucket_rank", ctypes.c_int32), ("fwd_chunk", ctypes.c_int32), ("bwd_waves", ctypes.c_int32),
                ("tile_order", ctypes.c_int32)]


_V = ctypes.c_void_p
_SIGS = [
    ("erbf_abi_version", ctypes.c_int32, []),
    ("erbf_last_error", ctypes.c_char_p, []),
    ("erbf_workspace_size", ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
    ("erbf_ctx_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Config), _V, ctypes.c_size_t,
                                       ctypes.POINTER(_V)]),
    ("erbf_ctx_destroy", None, [_V]),
    ("erbf_ctx_info", ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32)]),
    ("erbf_sdf_min", ctypes.c_int, [_V, ctypes.c_int64, _V, ctypes.c_int, _V]),
    ("erbf_targets_from_sdf", ctypes.c_int, [_V, ctypes.c_int64, ctypes.c_float, _V, _V]),
    ("erbf_band_bits", ctypes.c_int, [_V, ctypes.c_int64, ctypes.c_float, _V, _V]),
    ("erbf_octree_bits", ctypes.c_int, [_V, _V, ctypes.c_int32, _V, _V]),
    ("erbf_refine_level", ctypes.c_int, [_V, ctypes.c_int32, ctypes.POINTER(Level), _V]),
    ("erbf_eval", ctypes.c_int, [_V, ctypes.POINTER(Params), _V, _V, _V]),
    ("erbf_loss_grad", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(LossCfg), _V, _V, _V, _V, _V]),
    ("erbf_loss_grad_batched", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(LossCfg), _V, _V, _V, _V,
                                              _V]),
    ("erbf_loss_grad_minibatch", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(LossCfg), _V,
                                                ctypes.c_int32, _V, _V, _V, _V]),
    ("erbf_vjp", ctypes.c_int, [_V, ctypes.POINTER(Params), _V, _V, _V, _V]),
    ("erbf_adam_step", ctypes.c_int, [_V, ctypes.POINTER(Params), _V, _V, _V, _V, ctypes.POINTER(AdamCfg), _V]),
    ("erbf_train_step", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(LossCfg), ctypes.POINTER(AdamCfg),
                                       _V, _V, _V, _V, _V, _V, _V, _V]),
    ("erbf_timing_enable", ctypes.c_int, [_V, ctypes.c_int32]),
    ("erbf_timing_read", ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    ("erbf_set_variant", ctypes.c_int, [_V, ctypes.c_int32]),
    ("erbf_get_variant", ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_int32)]),
    ("erbf_set_launch", ctypes.c_int, [_V, ctypes.POINTER(LaunchCfg)]),
    ("erbf_get_launch", ctypes.c_int, [_V, ctypes.POINTER(LaunchCfg)]),
    ("erbf_autotune", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(LossCfg), _V, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), _V, _V]),
    ("erbf_seed_from_error", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.c_int32, _V, ctypes.c_float,
                                            ctypes.c_int64, ctypes.POINTER(SeedCfg), _V, _V,
                                            ctypes.POINTER(ctypes.c_int32), _V]),
    ("erbf_init_inscribed", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_float,
                                           ctypes.c_int32, _V, _V, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64), _V]),
    ("erbf_sdf_from_targets", ctypes.c_int, [_V, ctypes.c_int64, ctypes.c_float, _V, _V]),
    ("erbf_surface_scratch_size", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    ("erbf_surface_extract", ctypes.c_int, [_V, ctypes.c_int32, _V, ctypes.c_float, _V, ctypes.c_size_t, _V,
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _V]),
    ("erbf_surface_sample", ctypes.c_int, [_V, ctypes.c_int64, _V, ctypes.c_int64, _V, _V, _V, _V, _V]),
    ("erbf_surface_metrics", ctypes.c_int, [_V, _V, ctypes.c_int64, _V, _V, ctypes.c_int64, _V, _V, _V]),
    ("erbf_surface_metrics_noalloc", ctypes.c_int, [_V, _V, ctypes.c_int64, _V, _V, ctypes.c_int64, _V, _V]),
    ("erbf_sched_init", ctypes.c_int, [_V, ctypes.POINTER(SchedCfg), ctypes.POINTER(SchedState), _V]),
    ("erbf_sched_step", ctypes.c_int, [_V, ctypes.POINTER(Params), ctypes.POINTER(SchedCfg),
                                       ctypes.POINTER(SchedState), _V, _V, _V, _V]),
]

EXPORTED = [s[0] for s in _SIGS]

_lib = None


def load(path: str = None):
    """Load ``liberbf.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.erbf_abi_version() != ABI_VERSION:
        raise ImportError("liberbf.so ABI version mismatch")
    if path is None:
        _lib = lib
    return lib


def check(rc: int):
    if rc != ERBF_OK:
        msg = load().erbf_last_error()
        raise ErbfError(rc, msg.decode() if msg else "")
    return rc
