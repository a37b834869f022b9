"""Python face of the three-liquid solver (``telbm_nl_*`` in include/telbm.h):
the extension of the ternary model to one more liquid, with a second phase
field psi (C3 = psi / chi).  Argument marshalling only; every step runs in
the library's HIP kernels and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np

from . import _lib
from ._lib import NL_FIELDS, TelbmError, TelbmNlParams
from .solver import Params


@dataclasses.dataclass
class NLParams:
    """The third liquid's double well and gradient coefficient."""
    lambda4: float = 0.140625
    kappa4: float = 0.045

    def c_struct(self) -> TelbmNlParams:
        return TelbmNlParams(self.lambda4, self.kappa4)


def _check(rc: int, handle=None):
    if rc != _lib.OK:
        msg = ""
        if handle:
            m = _lib.load().telbm_nl_last_error(handle)
            msg = m.decode() if m else ""
        raise TelbmError(rc, msg)


def mobility(p: Params, q: NLParams) -> np.ndarray:
    """The (phi, psi) mobility matrix divided by M."""
    out = (ctypes.c_double * 4)()
    cs, cq = p.c_struct(), q.c_struct()
    _check(_lib.load().telbm_nl_mobility(ctypes.byref(cs), ctypes.byref(cq), out))
    return np.array(out[:]).reshape(2, 2)


def required_bytes(p: Params, q: NLParams) -> int:
    n = ctypes.c_size_t()
    cs, cq = p.c_struct(), q.c_struct()
    _check(_lib.load().telbm_nl_required_bytes(ctypes.byref(cs), ctypes.byref(cq), ctypes.byref(n)))
    return n.value


class NLSolver:
    """Three liquids and the gas on the current GPU; state in a torch-owned arena."""

    def __init__(self, p: Params, q: NLParams, device: Optional[str] = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("telbm needs a GPU: no HIP device is visible")
        self.L = _lib.load()
        self.p, self.q = p, q
        self.device = torch.device(device or "cuda")
        nbytes = required_bytes(p, q)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert self.arena.data_ptr() % 256 == 0
        self._cs, self._cq = p.c_struct(), q.c_struct()
        h = ctypes.c_void_p()
        _check(self.L.telbm_nl_create(ctypes.byref(self._cs), ctypes.byref(self._cq),
                                      ctypes.c_void_p(self.arena.data_ptr()), nbytes, ctypes.byref(h)))
        self.h = h
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self.L.telbm_nl_set_stream(self.h, ctypes.c_void_p(self.stream.cuda_stream)), self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.telbm_nl_destroy(self.h)
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

    def init_fields(self, rho, phi, psi, u=None):
        """Host (numpy) fields, float64, of shape (nz, ny, nx); u has D leading components."""
        keep = []

        def ptr(a, comps=1):
            if a is None:
                return None
            arr = np.ascontiguousarray(a, dtype=np.float64)
            assert arr.size == comps * self.p.nodes, (arr.shape, comps, self.p.shape)
            keep.append(arr)
            return arr.ctypes.data_as(ctypes.c_void_p)

        uu = None if u is None else np.asarray(u)[: self.p.dims]
        _check(self.L.telbm_nl_init_fields(self.h, ptr(rho), ptr(phi), ptr(psi), ptr(uu, self.p.dims), 0), self.h)

    def step(self, n: int = 1):
        _check(self.L.telbm_nl_step(self.h, int(n)), self.h)

    def read(self, field: str) -> np.ndarray:
        out = np.empty(self.p.shape, dtype=np.float64)
        _check(self.L.telbm_nl_read(self.h, NL_FIELDS[field], out.ctypes.data_as(ctypes.c_void_p), 0), self.h)
        return out

    def fields(self) -> dict:
        f = {k: self.read(k) for k in ("rho", "phi", "psi")}
        f["c"] = np.stack([self.read(k) for k in ("c1", "c2", "c3")])
        f["mu"] = np.stack([self.read(k) for k in ("mu_rho", "mu_phi", "mu_psi")])
        f["u"] = np.stack([self.read(k) for k in ("ux", "uy", "uz")])
        f["force"] = np.stack([self.read(k) for k in ("fx", "fy", "fz")])
        return f

    @property
    def steps(self) -> int:
        n = ctypes.c_int64()
        _check(self.L.telbm_nl_step_count(self.h, ctypes.byref(n)), self.h)
        return n.value
