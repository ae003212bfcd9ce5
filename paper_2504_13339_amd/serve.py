"""Python wrapper of the continuous-batching render server (veg_serve_* in libveg)."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, load
from . import veg as V

__all__ = ["Server", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "REQ_FAILED"]

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class Server:
    """Resident models + continuous batching.  The device arena is a torch tensor owned by
    this object; the library sub-allocates it and allocates nothing itself."""

    def __init__(self, max_gaussians: int, max_entries: int, max_batch: int = 8, n_streams: int = 2,
                 use_graphs: bool = True, max_width: int = 1920, max_height: int = 1080, max_tf_k: int = 256,
                 max_pairs: int = 0, budget_bytes: Optional[int] = None, device="cuda"):
        lib = load()
        cfg = _lib.veg_serve_config()
        cfg.max_batch, cfg.n_streams, cfg.use_graphs = int(max_batch), int(n_streams), int(bool(use_graphs))
        cfg.max_width, cfg.max_height, cfg.max_tf_k = int(max_width), int(max_height), int(max_tf_k)
        cfg.max_gaussians, cfg.max_pairs, cfg.max_entries = int(max_gaussians), int(max_pairs), int(max_entries)
        nbytes = lib.veg_serve_arena_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            check(1, "veg_serve_arena_bytes")
        self.arena = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        cfg.arena = ctypes.c_void_p(self.arena.data_ptr())
        cfg.arena_bytes = int(nbytes)
        cfg.budget_bytes = int(budget_bytes) if budget_bytes is not None else int(nbytes)
        self.cfg = cfg
        self._h = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(lib.veg_serve_create(ctypes.byref(cfg), ctypes.byref(self._h)), "veg_serve_create")
        self._models = []   # keeps the model tensors alive

    @property
    def arena_bytes(self) -> int:
        return int(self.cfg.arena_bytes)

    def add_model(self, g: V.Gaussians) -> int:
        mid = ctypes.c_int32(-1)
        gs = g.struct()
        check(load().veg_serve_add_model(self._h, ctypes.byref(gs), ctypes.byref(mid)), "veg_serve_add_model")
        self._models.append(g)
        return int(mid.value)

    def submit(self, model_id: int, camera, tf: np.ndarray, out_image: torch.Tensor,
               out_t_final: Optional[torch.Tensor] = None, opts=None, t_arrival: float = 0.0) -> int:
        """Queues a request.  ``t_arrival`` (time.perf_counter() seconds, 0 = now) is the
        time latency is measured from."""
        tf = np.ascontiguousarray(tf, dtype=np.float32)
        r = _lib.veg_request()
        r.model_id = int(model_id)
        r.camera = V.camera_struct(camera)
        r.tf_rgba = ctypes.c_void_p(tf.ctypes.data)
        r.tf_k = int(tf.shape[0])
        r.out_image = ctypes.c_void_p(out_image.data_ptr())
        r.out_t_final = ctypes.c_void_p(out_t_final.data_ptr()) if out_t_final is not None else None
        r.opts = opts if isinstance(opts, _lib.veg_opts) else V.make_opts(opts)
        r.t_arrival = float(t_arrival)
        rid = ctypes.c_uint64(0)
        check(load().veg_serve_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "veg_serve_submit")
        return int(rid.value)

    def poll(self, req_id: int) -> int:
        st = ctypes.c_int32(-1)
        check(load().veg_serve_poll(self._h, ctypes.c_uint64(req_id), ctypes.byref(st)), "veg_serve_poll")
        return int(st.value)

    def wait(self, req_id: int, timeout_ms: int = -1):
        check(load().veg_serve_wait(self._h, ctypes.c_uint64(req_id), int(timeout_ms)), "veg_serve_wait")

    def stats(self) -> dict:
        s = _lib.veg_serve_stats()
        check(load().veg_serve_stats_get(self._h, ctypes.byref(s)), "veg_serve_stats_get")
        return {name: getattr(s, name) for name, _ in s._fields_}

    def reset_stats(self):
        check(load().veg_serve_stats_reset(self._h), "veg_serve_stats_reset")

    def close(self):
        if self._h:
            check(load().veg_serve_destroy(self._h), "veg_serve_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
