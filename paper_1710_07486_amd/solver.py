"""Python face of the C ABI: one solver instance on one GPU.

PyTorch supplies the device arena and the stream; every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: without the
built library or a GPU the constructor raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional

import numpy as np

from . import _lib
from ._lib import FIELDS, TelbmDiag, TelbmError, TelbmParams


@dataclasses.dataclass
class Params:
    """Parameters of the free energy (Eqs. 1-4), transport and lattice."""
    lattice: int = _lib.D2Q9
    precision: int = _lib.FP64
    nx: int = 64
    ny: int = 64
    nz: int = 1
    a: float = 0.037
    b: float = 0.2
    R: float = 1.0
    T: float = 0.0
    rho_g: float = 0.0
    rho_l: float = 0.0
    lambda1: float = 0.6
    lambda2: float = 0.140625
    lambda3: float = 0.140625
    kappa1: float = 1e-3
    kappa2: float = 0.045
    kappa3: float = 0.045
    chi: float = 5.0
    nu: float = 0.167
    mobility: float = 0.5
    tau_phi: float = 1.0
    rho_ref: float = 0.0
    diag_every: int = 0
    eos: int = 0          # 0 Carnahan-Starling (Eq. 4), 1 van der Waals, 2 Peng-Robinson
    omega: float = 0.344  # Peng-Robinson acentric factor
    walls: int = 0        # 1: solid walls at y = -1/2 and y = ny - 1/2 (bounce-back, geometric wetting)
    theta_rho_lo: float = math.pi / 2  # contact angles (radians) at the bottom (lo) and top (hi)
    theta_rho_hi: float = math.pi / 2  # wall, measured in the phase where rho / phi is large
    theta_phi_lo: float = math.pi / 2
    theta_phi_hi: float = math.pi / 2
    glattice: int = 0     # phase-field lattice: 0 as for f, 1 reduced (D2Q5 / D3Q7)

    def c_struct(self) -> TelbmParams:
        kw = {f: getattr(self, f) for f, _ in TelbmParams._fields_ if hasattr(self, f)}
        return TelbmParams(**kw)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self) -> int:
        return 2 if self.lattice == _lib.D2Q9 else 3


def _check(rc: int, handle=None):
    if rc != _lib.OK:
        msg = ""
        if handle:
            m = _lib.load().telbm_last_error(handle)
            msg = m.decode() if m else ""
        raise TelbmError(rc, msg)


EOS_CS, EOS_VDW, EOS_PR = 0, 1, 2


def critical_temperature(a=0.037, b=0.2, R=1.0, eos=EOS_CS, omega=0.344) -> float:
    out = ctypes.c_double()
    _check(_lib.load().telbm_eos_critical_temperature(eos, a, b, R, omega, ctypes.byref(out)))
    return out.value


def coexistence(T, a=0.037, b=0.2, R=1.0, eos=EOS_CS, omega=0.344):
    """(rho_g, rho_l, C, Psi0) from the library's Maxwell construction."""
    rg, rl, C, p0 = (ctypes.c_double() for _ in range(4))
    _check(_lib.load().telbm_eos_coexistence(eos, a, b, R, omega, T, ctypes.byref(rg), ctypes.byref(rl),
                                             ctypes.byref(C), ctypes.byref(p0)))
    return rg.value, rl.value, C.value, p0.value


def temperature_for_ratio(ratio, a=0.037, b=0.2, R=1.0, eos=EOS_CS, omega=0.344) -> float:
    T = ctypes.c_double()
    _check(_lib.load().telbm_eos_temperature_for_ratio(eos, a, b, R, omega, ratio, ctypes.byref(T)))
    return T.value


def required_bytes(p: Params) -> int:
    n = ctypes.c_size_t()
    cs = p.c_struct()
    _check(_lib.load().telbm_required_bytes(ctypes.byref(cs), ctypes.byref(n)))
    return n.value


class Solver:
    """One lattice on the current GPU; state lives in a torch-owned arena."""

    def __init__(self, p: Params, device: Optional[str] = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("telbm needs a GPU: no HIP device is visible")
        self.L = _lib.load()
        self.p = p
        self.device = torch.device(device or "cuda")
        nbytes = required_bytes(p)
        # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert self.arena.data_ptr() % 256 == 0
        self._cs = p.c_struct()
        h = ctypes.c_void_p()
        _check(self.L.telbm_create(ctypes.byref(self._cs), ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                   ctypes.byref(h)))
        self.h = h
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self.L.telbm_set_stream(self.h, ctypes.c_void_p(self.stream.cuda_stream)), self.h)

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.L.telbm_destroy(self.h)
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

    # -- the calls of the ABI ------------------------------------------------
    def init_fields(self, rho, phi, u=None):
        """Fields as numpy arrays (host) or torch CUDA tensors (device), float64."""
        import torch
        on_dev = isinstance(rho, torch.Tensor) and rho.is_cuda
        keep = []

        def ptr(a, comps=1):
            if a is None:
                return None
            if on_dev:
                t = a.to(torch.float64).contiguous()
                assert t.numel() == comps * self.p.nodes
                keep.append(t)
                return ctypes.c_void_p(t.data_ptr())
            arr = np.ascontiguousarray(a, dtype=np.float64)
            assert arr.size == comps * self.p.nodes, (arr.shape, comps, self.p.shape)
            keep.append(arr)
            return arr.ctypes.data_as(ctypes.c_void_p)

        uu = None
        if u is not None:
            uu = u[: self.p.dims]
        rc = self.L.telbm_init_fields(self.h, ptr(rho), ptr(phi), ptr(uu, self.p.dims), 1 if on_dev else 0)
        _check(rc, self.h)

    def step(self, n: int = 1):
        _check(self.L.telbm_step(self.h, int(n)), self.h)

    def sync(self):
        _check(self.L.telbm_sync(self.h), self.h)

    def read(self, field: str, device: bool = False, check: bool = True):
        """One field of the current state: numpy (host) or a torch CUDA tensor.
        With check=False a diagnosed instability does not raise (the field is
        still returned)."""
        import torch
        code = FIELDS[field]
        if device:
            out = torch.empty(self.p.shape, dtype=torch.float64, device=self.device)
            rc = self.L.telbm_read(self.h, code, ctypes.c_void_p(out.data_ptr()), 1)
        else:
            out = np.empty(self.p.shape, dtype=np.float64)
            rc = self.L.telbm_read(self.h, code, out.ctypes.data_as(ctypes.c_void_p), 0)
        if check or rc != _lib.ERR_UNSTABLE:
            _check(rc, self.h)
        return out

    def fields(self):
        f = {k: self.read(k) for k in ("rho", "phi", "c1", "c2", "mu_rho", "mu_phi")}
        f["u"] = np.stack([self.read(k) for k in ("ux", "uy", "uz")])
        f["force"] = np.stack([self.read(k) for k in ("fx", "fy", "fz")])
        return f

    def diagnostics(self, check: bool = True) -> dict:
        """Diagnostics of the current state (a diagnostic pass if none is taken)."""
        return self._diag(self.L.telbm_diagnostics, check)

    def last_diagnostics(self, check: bool = True) -> dict:
        """The diagnostics taken last (by a diagnosed step or a pass), no new pass."""
        return self._diag(self.L.telbm_last_diagnostics, check)

    def _diag(self, fn, check: bool) -> dict:
        d = TelbmDiag()
        rc = fn(self.h, ctypes.byref(d))
        if check or rc != _lib.ERR_UNSTABLE:
            _check(rc, self.h)
        return {"step": d.step, "mass": d.mass, "phi_total": d.phi_total, "mom": list(d.mom),
                "max_u": d.max_u, "min_rho": d.min_rho, "gamma_min": d.gamma_min,
                "gamma_max": d.gamma_max, "nonfinite": d.nonfinite, "unstable": rc == _lib.ERR_UNSTABLE}

    @property
    def steps(self) -> int:
        n = ctypes.c_int64()
        _check(self.L.telbm_step_count(self.h, ctypes.byref(n)), self.h)
        return n.value

    def time_kernels(self, n: int, span: bool = False):
        """Mean HIP-event duration (ms) of each kernel kind over n steps; with
        ``span`` also the mean time per step over the whole timed span (first
        launch start to last launch end), as (kinds dict, ms per step)."""
        ms = (ctypes.c_double * 8)()
        kinds = ctypes.c_int()
        _check(self.L.telbm_time_kernels(self.h, int(n), ms, ctypes.byref(kinds)), self.h)
        per = {self.L.telbm_kernel_name(self.h, k).decode(): ms[k] for k in range(kinds.value)}
        return (per, ms[kinds.value]) if span else per

    def algorithmic_bytes_per_update(self) -> float:
        return self.L.telbm_algorithmic_bytes_per_update(self.h)
