"""Batched form: many lattices of uneven size and parameters on one GPU.

Each phase of a step is one persistent launch over all instances' tiles;
runs of steps replay captured HIP graphs.  Marshalling only; the work runs in
the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np

from . import _lib
from ._lib import FIELDS, TelbmError, TelbmParams
from .solver import Params

_vp, _i, _i64, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
PROTOTYPES = {
    "telbm_batch_required_bytes": (_i, [ctypes.POINTER(TelbmParams), _i, ctypes.POINTER(_sz)]),
    "telbm_batch_create": (_i, [ctypes.POINTER(TelbmParams), _i, _vp, _sz, ctypes.POINTER(_vp)]),
    "telbm_batch_set_stream": (_i, [_vp, _vp]),
    "telbm_batch_tile_variants": (_i, [ctypes.POINTER(_i)]),
    "telbm_batch_tile_shape": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "telbm_batch_set_tiles": (_i, [_vp, _i, _i]),
    "telbm_batch_set_graph_steps": (_i, [_vp, _i]),
    "telbm_batch_set_mode": (_i, [_vp, _i]),
    "telbm_batch_init_fields": (_i, [_vp, _i, _vp, _vp, _vp, _i]),
    "telbm_batch_step": (_i, [_vp, _i64]),
    "telbm_batch_read": (_i, [_vp, _i, _i, _vp, _i]),
    "telbm_batch_sync": (_i, [_vp]),
    "telbm_batch_step_count": (_i, [_vp, ctypes.POINTER(_i64)]),
    "telbm_batch_destroy": (_i, [_vp]),
    "telbm_batch_last_error": (ctypes.c_char_p, [_vp]),
}


def _load():
    L = _lib.load()
    if not getattr(L, "_batch_protos", False):
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        L._batch_protos = True
    return L


def _arr(params: Sequence[Params]):
    A = TelbmParams * len(params)
    return A(*[p.c_struct() for p in params])


def tile_variants() -> List[tuple]:
    L = _load()
    n = ctypes.c_int()
    L.telbm_batch_tile_variants(ctypes.byref(n))
    out = []
    for v in range(n.value):
        bx, by = ctypes.c_int(), ctypes.c_int()
        L.telbm_batch_tile_shape(v, ctypes.byref(bx), ctypes.byref(by))
        out.append((bx.value, by.value))
    return out


def required_bytes(params: Sequence[Params]) -> int:
    L = _load()
    n = ctypes.c_size_t()
    rc = L.telbm_batch_required_bytes(_arr(params), len(params), ctypes.byref(n))
    if rc:
        raise TelbmError(rc, "invalid batch parameters")
    return n.value


class Batch:
    """A set of lattices advanced together on the current GPU."""

    def __init__(self, params: Sequence[Params], stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("telbm needs a GPU: no HIP device is visible")
        self.L = _load()
        self.params = list(params)
        self.mode = 0
        nbytes = required_bytes(self.params)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._cs = _arr(self.params)
        h = ctypes.c_void_p()
        rc = self.L.telbm_batch_create(self._cs, len(self.params), ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                       ctypes.byref(h))
        if rc:
            raise TelbmError(rc, "batch create failed")
        self.h = h
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._check(self.L.telbm_batch_set_stream(self.h, ctypes.c_void_p(self.stream.cuda_stream)))

    def _check(self, rc):
        if rc:
            m = self.L.telbm_batch_last_error(self.h)
            raise TelbmError(rc, m.decode() if m else "")

    def close(self):
        if getattr(self, "h", None):
            self.L.telbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_tiles(self, variant: int, wg_per_cu: int):
        self._check(self.L.telbm_batch_set_tiles(self.h, int(variant), int(wg_per_cu)))

    def set_graph_steps(self, n: int):
        self._check(self.L.telbm_batch_set_graph_steps(self.h, int(n)))

    def set_mode(self, mode: int):
        """0: persistent three-phase launches over (instance, tile) work lists;
        D2Q9 only: 1, the single solver's fused step per instance on parallel
        graph branches; 2, that fused step for all instances in one launch."""
        self._check(self.L.telbm_batch_set_mode(self.h, int(mode)))
        self.mode = int(mode)

    def init_fields(self, idx: int, rho, phi, u=None):
        p = self.params[idx]
        keep = [np.ascontiguousarray(rho, dtype=np.float64), np.ascontiguousarray(phi, dtype=np.float64)]
        assert keep[0].size == p.nodes and keep[1].size == p.nodes
        up = None
        if u is not None:
            uu = np.ascontiguousarray(np.asarray(u)[: p.dims], dtype=np.float64)
            keep.append(uu)
            up = uu.ctypes.data_as(ctypes.c_void_p)
        self._check(self.L.telbm_batch_init_fields(self.h, int(idx), keep[0].ctypes.data_as(ctypes.c_void_p),
                                                   keep[1].ctypes.data_as(ctypes.c_void_p), up, 0))

    def step(self, n: int = 1):
        self._check(self.L.telbm_batch_step(self.h, int(n)))

    def sync(self):
        self._check(self.L.telbm_batch_sync(self.h))

    def read(self, idx: int, field: str) -> np.ndarray:
        p = self.params[idx]
        out = np.empty(p.shape, dtype=np.float64)
        self._check(self.L.telbm_batch_read(self.h, int(idx), FIELDS[field], out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def read_device(self, idx: int, field: str, out):
        """One field of instance idx into a float64 CUDA tensor of its size."""
        p = self.params[idx]
        assert out.is_cuda and out.dtype.itemsize == 8 and out.numel() == p.nodes and out.is_contiguous()
        self._check(self.L.telbm_batch_read(self.h, int(idx), FIELDS[field], ctypes.c_void_p(out.data_ptr()), 1))
        return out

    @property
    def steps(self) -> int:
        n = ctypes.c_int64()
        self._check(self.L.telbm_batch_step_count(self.h, ctypes.byref(n)))
        return n.value
