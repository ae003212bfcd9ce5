"""ctypes loader for libveg.so and the C structs of include/veg.h."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, \
    c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libveg.so")

VEG_TILE = 16
VEG_MAX_FRAMES = 4096
VEG_L1_SLOTS = 64
VEG_REC_FLOATS = 12
VEG_G2D_COMPONENTS = 9

STATUS = {0: "VEG_OK", 1: "VEG_ERR_INVALID_ARG", 2: "VEG_ERR_CAPACITY", 3: "VEG_ERR_OUT_OF_BUDGET",
          4: "VEG_ERR_NOT_FOUND", 5: "VEG_ERR_BUSY", 6: "VEG_ERR_HIP", 7: "VEG_ERR_TIMEOUT", 8: "VEG_ERR_SHUTDOWN"}


class VegError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class veg_gaussians(Structure):
    _fields_ = [("n", c_int64), ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("scalars", c_void_p), ("weights", c_void_p), ("normals", c_void_p), ("k_ambient", c_void_p),
                ("k_diffuse", c_void_p), ("k_specular", c_void_p), ("shininess", c_void_p)]


class veg_camera(Structure):
    _fields_ = [("view", c_float * 12), ("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
                ("width", c_int32), ("height", c_int32)]


class veg_tf(Structure):
    _fields_ = [("rgba", c_void_p), ("k", c_int32)]


class veg_opts(Structure):
    _fields_ = [("alpha_clamp", c_float), ("alpha_min", c_float), ("t_min", c_float), ("lowpass", c_float),
                ("near_z", c_float), ("guard", c_float), ("bg", c_float * 3)]


class veg_proj(Structure):
    _fields_ = [("n", c_int64), ("n_frames", c_int32), ("width", c_int32), ("height", c_int32),
                ("tiles_x", c_int32), ("tiles_y", c_int32), ("total_tiles", c_int64), ("frames", c_void_p),
                ("rec", c_void_p), ("count", c_void_p), ("depth", c_void_p), ("tfs_per_view", c_int32)]


class veg_vq_field(Structure):
    _fields_ = [("dst", c_void_p), ("width", c_int32)]


class veg_densify_field(Structure):
    _fields_ = [("src", c_void_p), ("dst", c_void_p), ("width", c_int32), ("role", c_int32)]


class veg_bins(Structure):
    _fields_ = [("keys", c_void_p), ("vals", c_void_p), ("keys_alt", c_void_p), ("vals_alt", c_void_p),
                ("ranges", c_void_p), ("capacity", c_int64), ("hits", c_void_p), ("hit_words", c_int64)]


class veg_grads(Structure):
    _fields_ = [("d_means", c_void_p), ("d_log_scales", c_void_p), ("d_quats", c_void_p), ("d_scalars", c_void_p),
                ("d_weights", c_void_p), ("d_normals", c_void_p), ("d_k_ambient", c_void_p),
                ("d_k_diffuse", c_void_p), ("d_k_specular", c_void_p), ("d_shininess", c_void_p)]


class veg_serve_config(Structure):
    _fields_ = [("arena", c_void_p), ("arena_bytes", c_size_t), ("budget_bytes", c_size_t), ("max_batch", c_int32),
                ("n_streams", c_int32), ("use_graphs", c_int32), ("max_width", c_int32), ("max_height", c_int32),
                ("max_tf_k", c_int32), ("max_gaussians", c_int64), ("max_pairs", c_int64), ("max_entries", c_int64)]


class veg_request(Structure):
    _fields_ = [("model_id", c_int32), ("camera", veg_camera), ("tf_rgba", c_void_p), ("tf_k", c_int32),
                ("out_image", c_void_p), ("out_t_final", c_void_p), ("opts", veg_opts), ("t_arrival", c_double)]


class veg_serve_stats(Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("failed", c_int64), ("rejected", c_int64),
                ("batches", c_int64), ("retries", c_int64), ("mean_batch", c_double), ("p50_ms", c_double),
                ("p99_ms", c_double), ("max_ms", c_double), ("throughput_rps", c_double), ("mpix_per_s", c_double),
                ("gpu_busy_frac", c_double), ("peak_bytes", c_int64), ("graphs_captured", c_int64)]


P = POINTER
_SIGS = {
    "veg_status_str": (c_char_p, [c_int]),
    "veg_last_error": (c_char_p, []),
    "veg_version": (c_int, []),
    "veg_opts_default": (None, [P(veg_opts)]),
    "veg_frames_bytes": (c_size_t, [c_int32]),
    "veg_project": (c_int, [P(veg_gaussians), c_int32, P(veg_camera), P(veg_tf), P(veg_opts), P(veg_proj), c_void_p]),
    "veg_project_views": (c_int, [P(veg_gaussians), c_int32, c_int32, P(veg_camera), P(veg_tf), P(veg_opts),
                                  P(veg_proj), c_void_p]),
    "veg_bin_workspace_bytes": (c_size_t, [c_int64, c_int64]),
    "veg_bin_count": (c_int, [P(veg_proj), c_void_p, c_size_t, P(c_int64), c_void_p]),
    "veg_bin_sort": (c_int, [P(veg_proj), c_void_p, c_size_t, P(veg_bins), c_void_p]),
    "veg_bin_overflow": (c_int, [c_void_p, c_size_t, P(c_int64), P(c_int32), c_void_p]),
    "veg_bin_status": (c_int, [c_void_p, c_size_t, c_void_p, c_void_p]),
    "veg_bin_static": (c_int, [P(veg_proj), P(veg_bins), c_void_p, c_void_p]),
    "veg_bin_hit_words": (c_int64, [c_int64, c_int64]),
    "veg_render_fwd": (c_int, [P(veg_proj), P(veg_bins), P(veg_opts), c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p]),
    "veg_render_fwd_l1": (c_int, [P(veg_proj), P(veg_bins), P(veg_opts), c_void_p, c_float, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "veg_render_bwd": (c_int, [P(veg_proj), P(veg_bins), P(veg_opts), c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p]),
    "veg_project_bwd": (c_int, [P(veg_gaussians), P(veg_proj), P(veg_opts), c_void_p, P(veg_grads), c_void_p]),
    "veg_project_bwd_fused": (c_int, [P(veg_gaussians), P(veg_proj), P(veg_opts), c_void_p, P(veg_grads), c_void_p,
                                      c_void_p, c_int32, c_void_p]),
    "veg_l1_loss": (c_int, [c_void_p, c_void_p, c_int64, c_float, c_void_p, c_void_p, c_void_p]),
    "veg_fill_u32": (c_int, [c_void_p, c_int64, c_uint32, c_void_p]),
    "veg_ssim_workspace_bytes": (c_size_t, [c_int64, c_int32, c_int32]),
    "veg_ssim_loss": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_float, c_void_p, c_void_p, c_void_p,
                              c_size_t, c_void_p]),
    "veg_image_loss": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_float, c_float, c_void_p, c_void_p,
                               c_void_p, c_size_t, c_void_p]),
    "veg_adam_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_float, c_float, c_float,
                              c_int32, c_void_p]),
    "veg_densify_stats": (c_int, [P(veg_proj), c_void_p, c_void_p, c_void_p, c_void_p]),
    "veg_vq_decode": (c_int, [c_void_p, c_int64, c_void_p, c_int32, c_int32, P(veg_vq_field), c_int32, c_void_p]),
    "veg_densify_workspace_bytes": (c_size_t, [c_int64]),
    "veg_densify_plan": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float, c_void_p,
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
    "veg_densify_apply": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, P(veg_densify_field), c_int32,
                                  c_void_p, c_size_t, c_void_p]),
    "veg_debug_math": (c_int, [c_int32, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "veg_serve_arena_bytes": (c_size_t, [P(veg_serve_config)]),
    "veg_serve_create": (c_int, [P(veg_serve_config), P(c_void_p)]),
    "veg_serve_add_model": (c_int, [c_void_p, P(veg_gaussians), P(c_int32)]),
    "veg_serve_submit": (c_int, [c_void_p, P(veg_request), P(c_uint64)]),
    "veg_serve_poll": (c_int, [c_void_p, c_uint64, P(c_int32)]),
    "veg_serve_wait": (c_int, [c_void_p, c_uint64, c_int32]),
    "veg_serve_stats_get": (c_int, [c_void_p, P(veg_serve_stats)]),
    "veg_serve_stats_reset": (c_int, [c_void_p]),
    "veg_serve_destroy": (c_int, [c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Loads the in-tree libveg.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def declared_symbols():
    return sorted(_SIGS)


def check(status: int, where: str):
    if status != 0:
        lib = load()
        raise VegError(status, where, (lib.veg_last_error() or b"").decode(errors="replace"))
