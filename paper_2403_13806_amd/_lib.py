"""ctypes declarations of include/gs.h and the loader of libgs_hip.so.

Argument marshalling only: every computation happens in the HIP library. Loading fails
loudly when the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# GS_HIP_LIB names another build of the same library (the sanitizer run loads a host-only
# build with address and undefined-behaviour checks)
LIB_PATH = os.environ.get("GS_HIP_LIB") or os.path.join(_HERE, "libgs_hip.so")

c_void_p = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
u64 = ctypes.c_uint64
f32 = ctypes.c_float

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_CAPACITY = -2
GS_ERR_HIP = -3
GS_ERR_UNSUPPORTED = -4


class gs_camera(ctypes.Structure):
    _fields_ = [("R", f32 * 9), ("t", f32 * 3), ("fx", f32), ("fy", f32), ("cx", f32), ("cy", f32),
                ("width", i32), ("height", i32), ("znear", f32), ("reserved", i32)]


class gs_params(ctypes.Structure):
    _fields_ = [("lowpass", f32), ("kappa", f32), ("alpha_min", f32), ("alpha_max", f32), ("t_min", f32),
                ("guard", f32), ("bg", f32 * 3)]


class gs_gaussians(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("scale", c_void_p), ("quat", c_void_p), ("opacity", c_void_p),
                ("sh", c_void_p), ("n", i64), ("sh_degree", i32)]


class gs_gaussians_grad(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("scale", c_void_p), ("quat", c_void_p), ("opacity", c_void_p),
                ("sh", c_void_p), ("n", i64), ("sh_degree", i32), ("overwrite", i32)]


class gs_views(ctypes.Structure):
    _fields_ = [("cams", c_void_p), ("tile_offset", c_void_p), ("pixel_offset", c_void_p), ("n_views", i32),
                ("tile_w", i32), ("tile_h", i32), ("n_tiles", i32), ("n_pixels", i64), ("batch_depth", i32),
                ("lpt", i32), ("pixels_per_lane", i32), ("max_view_tiles", i32)]


class gs_projected(ctypes.Structure):
    _fields_ = [("splat", c_void_p), ("depth", c_void_p), ("rect", c_void_p), ("count", c_void_p), ("n", i64)]


class gs_bins(ctypes.Structure):
    _fields_ = [("keys", c_void_p), ("vals", c_void_p), ("ranges", c_void_p), ("capacity", u64),
                ("n_pairs", c_void_p), ("overflow", c_void_p), ("queue", c_void_p), ("entry_offset", c_void_p),
                ("overflow_sticky", c_void_p)]


class gs_adam_group(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p), ("count", i64),
                ("lr", f32), ("mode", i32)]


GS_ADAM_LINEAR, GS_ADAM_LOG, GS_ADAM_LOGIT = 0, 1, 2

assert ctypes.sizeof(gs_camera) == 80
SPLAT_BYTES = 64

EXPORTS = ["gs_view_layout", "gs_workspace_bytes", "gs_preprocess", "gs_bin_sort", "gs_bin_sort_noalloc",
           "gs_render_fwd", "gs_bin_sort_render_fwd", "gs_render_bwd",
           "gs_importance", "gs_cluster_visibility", "gs_bin_sort_importance", "gs_bin_sort_cluster_visibility",
           "gs_bits_to_list", "gs_kmeans", "gs_kmeans_seed",
           "gs_kmeans_workspace_bytes", "gs_kmeans_lloyd", "gs_nearest_centre",
           "gs_l1_loss_grad", "gs_ssim_workspace_bytes", "gs_ssim_loss_grad", "gs_prune_mask", "gs_prune",
           "gs_gather", "gs_nn_workspace_bytes", "gs_nn_distance", "gs_init_gaussians",
           "gs_adam_step", "gs_last_error"]

_lib = None


class GSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gs error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libgs_hip.so (built by __graft_entry__.build() / paper_2403_13806_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.gs_view_layout.argtypes = [P(gs_camera), i32, i32, i32, P(i32), P(i64)]
    L.gs_view_layout.restype = i32
    L.gs_workspace_bytes.argtypes = [i64, i32, u64, i32]
    L.gs_workspace_bytes.restype = ctypes.c_size_t
    L.gs_preprocess.argtypes = [P(gs_gaussians), P(gs_views), P(gs_params), c_void_p, i64, i32, P(gs_projected),
                                c_void_p]
    L.gs_preprocess.restype = i32
    L.gs_bin_sort.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_bin_sort.restype = i32
    L.gs_bin_sort_noalloc.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), c_void_p]
    L.gs_bin_sort_noalloc.restype = i32
    L.gs_render_fwd.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p]
    L.gs_bin_sort_render_fwd.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p,
                                         c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_bin_sort_render_fwd.restype = i32
    L.gs_bin_sort_importance.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p,
                                         c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_bin_sort_importance.restype = i32
    L.gs_bin_sort_cluster_visibility.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p,
                                                 i32, f32, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_bin_sort_cluster_visibility.restype = i32
    L.gs_l1_loss_grad.argtypes = [c_void_p, c_void_p, i64, f32, c_void_p, c_void_p, c_void_p]
    L.gs_l1_loss_grad.restype = i32
    L.gs_ssim_workspace_bytes.argtypes = [i32, i32, i32]
    L.gs_ssim_workspace_bytes.restype = ctypes.c_size_t
    L.gs_ssim_loss_grad.argtypes = [c_void_p, c_void_p, i32, i32, i32, i64, f32, c_void_p, c_void_p, c_void_p,
                                    ctypes.c_size_t, c_void_p]
    L.gs_ssim_loss_grad.restype = i32
    L.gs_render_fwd.restype = i32
    L.gs_render_bwd.argtypes = [P(gs_gaussians), P(gs_views), P(gs_projected), P(gs_bins), P(gs_params), c_void_p,
                                c_void_p, c_void_p, P(gs_gaussians_grad), c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_render_bwd.restype = i32
    L.gs_importance.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p, c_void_p]
    L.gs_importance.restype = i32
    L.gs_cluster_visibility.argtypes = [P(gs_projected), P(gs_views), P(gs_bins), P(gs_params), c_void_p, i32, f32,
                                        c_void_p, c_void_p]
    L.gs_cluster_visibility.restype = i32
    L.gs_bits_to_list.argtypes = [c_void_p, i64, c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_bits_to_list.restype = i32
    L.gs_prune_mask.argtypes = [c_void_p, i64, f32, c_void_p, c_void_p]
    L.gs_prune_mask.restype = i32
    L.gs_prune.argtypes = [c_void_p, i64, f32, P(c_void_p), P(c_void_p), i32, c_void_p, c_void_p, c_void_p,
                           ctypes.c_size_t, c_void_p]
    L.gs_prune.restype = i32
    L.gs_gather.argtypes = [c_void_p, i64, i64, P(c_void_p), P(c_void_p), i32, c_void_p]
    L.gs_gather.restype = i32
    L.gs_nn_workspace_bytes.argtypes = [i64]
    L.gs_nn_workspace_bytes.restype = ctypes.c_size_t
    L.gs_nn_distance.argtypes = [c_void_p, i64, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_nn_distance.restype = i32
    L.gs_init_gaussians.argtypes = [c_void_p, c_void_p, i64, i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, ctypes.c_size_t, c_void_p]
    L.gs_init_gaussians.restype = i32
    L.gs_adam_step.argtypes = [P(gs_adam_group), i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64, i32,
                               c_void_p]
    L.gs_adam_step.restype = i32
    L.gs_kmeans.argtypes = [c_void_p, i32, i32, u64, i32, c_void_p, c_void_p]
    L.gs_kmeans.restype = i32
    L.gs_kmeans_seed.argtypes = [c_void_p, i32, i32, u64, c_void_p]
    L.gs_kmeans_seed.restype = i32
    L.gs_kmeans_workspace_bytes.argtypes = [i64, i32, i32]
    L.gs_kmeans_workspace_bytes.restype = ctypes.c_size_t
    L.gs_kmeans_lloyd.argtypes = [c_void_p, i64, i32, i32, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_size_t,
                                  c_void_p]
    L.gs_kmeans_lloyd.restype = i32
    L.gs_nearest_centre.argtypes = [c_void_p, i32, c_void_p]
    L.gs_nearest_centre.restype = i32
    L.gs_last_error.argtypes = []
    L.gs_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(code: int):
    if code != GS_OK:
        raise GSError(code, load().gs_last_error().decode())
