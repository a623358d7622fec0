"""Python face of the serving ABI (``la_serve_*`` in ``include/la.h``)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._binding import (PolarInfo, ServeConfig, ServeStats, Status, check, context, lib,
                       make_opts)


class Server:
    """Continuous-batching polar server on one GPU.

    ``arena_bytes`` of device memory (a torch allocation owned by this object)
    holds every admitted request's state; requests wait in the queue until
    their footprint fits and a slot is free.  ``bands`` (0: the library's
    default of 2) is the number of size bands that tick independently."""

    def __init__(self, arena_bytes: int, device: int = 0, max_slots: int = 32,
                 max_queue: int = 4096, bands: int = 0):
        self._arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=f"cuda:{device}")
        base = self._arena.data_ptr()
        self._base = (base + 255) & ~255
        self._bytes = arena_bytes
        cfg = ServeConfig()
        cfg.max_slots = max_slots
        cfg.max_queue = max_queue
        cfg.bands = bands
        out = ctypes.c_void_p()
        check(lib().la_serve_create(context(device), ctypes.byref(cfg), self._base, arena_bytes,
                                    ctypes.byref(out)))
        self._srv = out
        self._shapes: dict[int, tuple[int, int]] = {}

    def submit(self, A: np.ndarray, **opts) -> int:
        A = np.ascontiguousarray(A, dtype=np.float32)
        m, n = A.shape
        o = make_opts(**opts)
        rid = ctypes.c_uint64()
        check(lib().la_serve_submit(self._srv, m, n, A.ctypes.data, n, ctypes.byref(o),
                                    ctypes.byref(rid)))
        self._shapes[rid.value] = (m, n)
        return rid.value

    def poll(self, rid: int, want_h: bool = True):
        """None while pending; else (status, U, H or None, info dict)."""
        if rid not in self._shapes:     # unknown here: let the library say so
            check(lib().la_serve_poll(self._srv, rid, None, None, None, None))
        m, n = self._shapes[rid]
        U = np.empty((m, n), np.float32)
        H = np.empty((n, n), np.float32) if want_h else None
        info = PolarInfo()
        rst = ctypes.c_int(0)
        st = lib().la_serve_poll(self._srv, rid, U.ctypes.data,
                                 H.ctypes.data if H is not None else None, ctypes.byref(info),
                                 ctypes.byref(rst))
        if st == Status.NOT_READY:
            return None
        check(st)
        del self._shapes[rid]
        return Status(rst.value), U, H, info.as_dict()

    def stats(self) -> dict:
        s = ServeStats()
        check(lib().la_serve_stats_get(self._srv, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_srv", None):
            lib().la_serve_destroy(self._srv)
            self._srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
