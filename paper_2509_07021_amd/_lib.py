"""ctypes binding of libmegs.so (include/megs.h): structures and function signatures only.

This module marshals arguments; every step of the renderer runs in the library's HIP
kernels. Loading fails loudly when the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmegs.so")

MEGS_OK, MEGS_ERR_ARG, MEGS_ERR_HIP, MEGS_ERR_CAPACITY, MEGS_ERR_UNSUPPORTED, MEGS_ERR_ALLOC = 0, -1, -2, -3, -4, -5
MEGS_F32, MEGS_F16, MEGS_BF16 = 0, 1, 2
MEGS_FLAG_ONE_STAGE_SORT = 1
MEGS_FLAG_PERSISTENT = 2
MEGS_FLAG_STATS = 4
MEGS_FLAG_DETERMINISTIC = 8
MEGS_FLAG_RECORD_PLANES = 16
STAGES = ("project", "depth_sort", "scan", "emit", "pair_sort", "ranges", "blend_fwd", "blend_bwd", "project_bwd")
MEGS_MAX_LOBES = 8
MEGS_MAX_VIEWS = 64
MEGS_NOALLOC_SCRATCH_BYTES = 64 << 20
AUTOTUNE_COMBOS = ((8, 1, 0), (16, 1, 0), (16, 2, 0), (16, 4, 0), (32, 1, 0), (32, 2, 0), (32, 4, 0), (16, 1, 8),
                   (32, 1, 8))   # (tile, waves, subtile)
AUTOTUNE_BATCHES = (32, 64, 128, 256)

EXPORTED = ("megs_render_forward", "megs_render_backward", "megs_state_status", "megs_graph_create",
            "megs_graph_launch", "megs_graph_status", "megs_graph_state", "megs_graph_destroy",
            "megs_autotune", "megs_profile_begin", "megs_profile_end", "megs_last_error", "megs_version",
            "megs_render_importance", "megs_lobe_range", "megs_select_topk", "megs_prox_apply", "megs_dual_update",
            "megs_penalty_grad", "megs_compact", "megs_photometric_loss", "megs_adam_step",
            "megs_render_forward_noalloc", "megs_state_counts", "megs_state_bytes", "megs_graph_capture")

PLANES = ("pos", "logscale", "quat", "op_logit", "pmask_logit",
          "base", "axis", "sharp", "amp", "lmask_logit")
ALL_PLANES = PLANES + ("sh",)   # "sh": spherical-harmonic coefficients (SH-colour scenes)

_vp = ctypes.c_void_p


class MegsScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("dt_geom", ctypes.c_int32),
                ("dt_color", ctypes.c_int32), ("dt_amp", ctypes.c_int32), ("reserved", ctypes.c_int32)] + \
               [(p, _vp) for p in PLANES] + [("lobe_off", _vp), ("n_lobes", ctypes.c_int64), ("sh", _vp),
                                             ("sh_degree", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class MegsCompacted(ctypes.Structure):
    _fields_ = [("scene", MegsScene), ("kept", _vp), ("lobe_src", _vp)]


class MegsSceneGrad(ctypes.Structure):
    _fields_ = [(p, _vp) for p in ALL_PLANES]


class MegsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("znear", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class MegsConfig(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("batch", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("waves", ctypes.c_int32), ("pair_capacity", ctypes.c_int64), ("subtile", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class MegsState(ctypes.Structure):
    _fields_ = [("n_records", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("pair_capacity", ctypes.c_int64),
                ("n_pixels", ctypes.c_int64), ("n_views", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("k", ctypes.c_int32),
                ("mean", _vp), ("conic_o", _vp), ("rgbd", _vp), ("radius", _vp), ("ntiles", _vp), ("cutoff", _vp),
                ("tile_keys", _vp), ("keys64", _vp), ("vals", _vp), ("ranges", _vp), ("T_final", _vp),
                ("last", _vp), ("device_status", _vp), ("internal", _vp), ("det_inv", _vp), ("det_order", _vp),
                ("det_offsets", _vp), ("det_count", _vp), ("packed", _vp), ("chol", _vp),
                ("work", _vp), ("work_bytes", ctypes.c_int64)]


class MegsCounts(ctypes.Structure):
    _fields_ = [("pairs_needed", ctypes.c_int64), ("culled", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("bad_lobes", ctypes.c_int32)]


class MegsMemory(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_size_t), ("pairs", ctypes.c_size_t), ("backward", ctypes.c_size_t),
                ("work", ctypes.c_size_t)]


class MegsProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)), ("count", ctypes.c_int64 * len(STAGES))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)

_lib = None


class MegsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libmegs status {status}: {message}")
        self.status = status


def load():
    """Load libmegs.so; raises when it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.megs_render_forward.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), ALLOC_FN, _vp,
                                      _vp, P(MegsState), _vp]
    L.megs_render_forward_noalloc.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), _vp,
                                              P(MegsState), _vp]
    L.megs_render_backward.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), P(MegsState),
                                       _vp, ALLOC_FN, _vp, P(MegsSceneGrad), _vp]
    L.megs_state_status.argtypes = [P(MegsState), P(ctypes.c_int64), _vp]
    L.megs_state_counts.argtypes = [P(MegsState), P(MegsCounts), _vp]
    L.megs_state_bytes.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), ctypes.c_int64,
                                   P(MegsMemory)]
    L.megs_graph_create.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), ALLOC_FN, _vp,
                                    _vp, _vp, P(MegsSceneGrad), ctypes.c_int32, _vp, P(_vp)]
    L.megs_graph_capture.argtypes = L.megs_graph_create.argtypes
    L.megs_graph_launch.argtypes = [_vp, _vp]
    L.megs_graph_status.argtypes = [_vp, P(ctypes.c_int64), _vp]
    L.megs_graph_state.argtypes = [_vp]
    L.megs_graph_state.restype = P(MegsState)
    L.megs_graph_destroy.argtypes = [_vp]
    L.megs_graph_destroy.restype = None
    L.megs_autotune.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), ALLOC_FN, _vp,
                                _vp, _vp, P(MegsSceneGrad), ctypes.c_int32, _vp, P(MegsConfig), P(ctypes.c_float)]
    L.megs_render_importance.argtypes = [P(MegsScene), P(MegsCamera), ctypes.c_int32, P(MegsConfig), ALLOC_FN,
                                         _vp, _vp, _vp, P(MegsState), _vp]
    L.megs_lobe_range.argtypes = [ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]
    L.megs_select_topk.argtypes = [_vp, ctypes.c_int64, ctypes.c_int64, ALLOC_FN, _vp, _vp, _vp]
    L.megs_prox_apply.argtypes = [ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
    L.megs_dual_update.argtypes = [ctypes.c_int64, _vp, _vp, _vp, _vp]
    L.megs_penalty_grad.argtypes = [ctypes.c_int64, ctypes.c_float, _vp, _vp, _vp, _vp, _vp]
    L.megs_compact.argtypes = [P(MegsScene), ctypes.c_double, ctypes.c_double, ALLOC_FN, _vp, _vp,
                               P(MegsCompacted)]
    L.megs_photometric_loss.argtypes = [_vp, _vp, ctypes.c_int32, P(ctypes.c_int32), ctypes.c_double, ALLOC_FN, _vp,
                                        _vp, _vp, _vp]
    L.megs_adam_step.argtypes = [ctypes.c_int64, _vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp]
    L.megs_profile_begin.argtypes = []
    L.megs_profile_end.argtypes = [P(MegsProfile)]
    for f in ("megs_render_forward", "megs_render_forward_noalloc", "megs_state_counts", "megs_state_bytes",
              "megs_render_backward",
              "megs_state_status", "megs_graph_create", "megs_graph_capture",
              "megs_graph_launch", "megs_graph_status", "megs_autotune", "megs_profile_begin", "megs_profile_end",
              "megs_render_importance", "megs_lobe_range", "megs_select_topk", "megs_prox_apply",
              "megs_dual_update", "megs_penalty_grad", "megs_compact", "megs_photometric_loss",
              "megs_adam_step"):
        getattr(L, f).restype = ctypes.c_int
    L.megs_last_error.restype = ctypes.c_char_p
    L.megs_last_error.argtypes = []
    L.megs_version.restype = ctypes.c_char_p
    L.megs_version.argtypes = []
    _lib = L
    return L


def check(status: int):
    if status != MEGS_OK:
        raise MegsError(status, load().megs_last_error().decode())
