"""ctypes wrapper of the FP64 CPU oracle (``telbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here imports the
GPU library, and the GPU library never imports this module.

Arrays are numpy float64.  Population arrays have shape ``(Q, nz, ny, nx)``
(x fastest), fields ``(nz, ny, nx)``, vector fields ``(3, nz, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import math
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "telbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

D2Q9, D3Q27 = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("T", ctypes.c_double), ("rho_g", ctypes.c_double), ("rho_l", ctypes.c_double),
        ("C", ctypes.c_double),
        ("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double), ("lambda3", ctypes.c_double),
        ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
        ("chi", ctypes.c_double), ("nu", ctypes.c_double), ("mobility", ctypes.c_double),
        ("tau_phi", ctypes.c_double),
        ("eos", ctypes.c_int32), ("pad", ctypes.c_int32), ("omega", ctypes.c_double),
        ("walls", ctypes.c_int32), ("pad2", ctypes.c_int32),
        ("theta_rho_lo", ctypes.c_double), ("theta_rho_hi", ctypes.c_double),
        ("theta_phi_lo", ctypes.c_double), ("theta_phi_hi", ctypes.c_double),
        ("glattice", ctypes.c_int32), ("pad3", ctypes.c_int32),
    ]


@dataclasses.dataclass
class Params:
    """Physical and lattice parameters, with the paper's symbols."""
    lattice: int = D2Q9
    nx: int = 32
    ny: int = 32
    nz: int = 1
    a: float = 0.037
    b: float = 0.2
    R: float = 1.0
    T: float = 0.0
    rho_g: float = 0.0
    rho_l: float = 0.0
    C: float = 0.0
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
    eos: int = 0          # 0 Carnahan-Starling (Eq. 4), 1 van der Waals, 2 Peng-Robinson
    pad: int = 0
    omega: float = 0.344  # Peng-Robinson acentric factor
    walls: int = 0        # 1: solid walls at y = -1/2 and y = ny - 1/2 (bounce-back, geometric wetting)
    pad2: int = 0
    theta_rho_lo: float = math.pi / 2  # contact angles in radians, measured in the phase
    theta_rho_hi: float = math.pi / 2  # where the field is large; lo = bottom wall, hi = top
    theta_phi_lo: float = math.pi / 2
    theta_phi_hi: float = math.pi / 2
    glattice: int = 0     # phase-field lattice: 0 as for f, 1 reduced (D2Q5 / D3Q7)
    pad3: int = 0

    def c_struct(self) -> OrcParams:
        return OrcParams(**{f: getattr(self, f) for f, _ in OrcParams._fields_})

    @property
    def Q(self) -> int:
        return 9 if self.lattice == D2Q9 else 27

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


class OrcNL(ctypes.Structure):
    _fields_ = [("lambda4", ctypes.c_double), ("kappa4", ctypes.c_double),
                ("mobility_form", ctypes.c_int32), ("pad", ctypes.c_int32)]


@dataclasses.dataclass
class NLParams:
    """The third liquid of the extension to more liquid components: its double
    well and gradient coefficients, and the mobility form (0 consistent
    matrix, 1 one mobility per order parameter)."""
    lambda4: float = 0.140625
    kappa4: float = 0.045
    mobility_form: int = 0

    def c_struct(self) -> OrcNL:
        return OrcNL(self.lambda4, self.kappa4, self.mobility_form, 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i32, vp, P = ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(OrcParams)
        L.orc_lattice_info.argtypes = [ctypes.c_int, vp, vp]
        L.orc_lattice_info.restype = ctypes.c_int
        for name in ("orc_psi_eos", "orc_psi_prime"):
            getattr(L, name).argtypes = [d, d, d, d, d, d]
            getattr(L, name).restype = d
        for name in ("orc_pressure", "orc_dpdrho"):
            getattr(L, name).argtypes = [d, d, d, d, d]
            getattr(L, name).restype = d
        I = ctypes.c_int
        for name in ("orc_eos_psi", "orc_eos_psi_prime"):
            getattr(L, name).argtypes = [I, d, d, d, d, d, d, d]
            getattr(L, name).restype = d
        L.orc_eos_pressure.argtypes = [I, d, d, d, d, d, d]
        L.orc_eos_pressure.restype = d
        L.orc_eos_attraction.argtypes = [I, d, d, d, d, d]
        L.orc_eos_attraction.restype = d
        L.orc_eos_critical_temperature.argtypes = [I, d, d, d, d, vp]
        L.orc_eos_critical_temperature.restype = d
        L.orc_eos_maxwell.argtypes = [I, d, d, d, d, d, vp]
        L.orc_eos_maxwell.restype = ctypes.c_int
        L.orc_eos_temperature_for_ratio.argtypes = [I, d, d, d, d, d, vp]
        L.orc_eos_temperature_for_ratio.restype = ctypes.c_int
        L.orc_critical_temperature.argtypes = [d, d, d, vp]
        L.orc_critical_temperature.restype = d
        L.orc_maxwell.argtypes = [d, d, d, d, vp]
        L.orc_maxwell.restype = ctypes.c_int
        L.orc_temperature_for_ratio.argtypes = [d, d, d, d, vp]
        L.orc_temperature_for_ratio.restype = ctypes.c_int
        L.orc_concentrations.argtypes = [P, d, d, vp, vp]
        L.orc_gradient_coefficients.argtypes = [P, vp]
        L.orc_mu_bulk.argtypes = [P, d, d, vp]
        for name in ("orc_f_bulk", "orc_bulk_pressure"):
            getattr(L, name).argtypes = [P, d, d]
            getattr(L, name).restype = d
        L.orc_laplacian.argtypes = [P, vp, vp]
        L.orc_gradient.argtypes = [P, vp, vp]
        L.orc_feq.argtypes = [ctypes.c_int, d, vp, vp]
        L.orc_geq.argtypes = [ctypes.c_int, d, d, d, vp, vp]
        L.orc_geq_reduced.argtypes = [ctypes.c_int, d, d, d, vp, vp]
        L.orc_kbc_split.argtypes = [ctypes.c_int, vp, vp, vp]
        L.orc_kbc_gamma.argtypes = [ctypes.c_int, d, vp, vp, vp]
        L.orc_kbc_gamma.restype = d
        L.orc_collide_node.argtypes = [ctypes.c_int, d, vp, vp, vp, vp]
        L.orc_init.argtypes = [P, vp, vp, vp, vp, vp]
        L.orc_init.restype = ctypes.c_int
        L.orc_run.argtypes = [P, vp, vp, ctypes.c_int64, vp]
        L.orc_run.restype = ctypes.c_int
        L.orc_fields.argtypes = [P, vp, vp] + [vp] * 8
        L.orc_fields.restype = ctypes.c_int
        NP = ctypes.POINTER(OrcNL)
        L.orc_nl_concentrations.argtypes = [P, d, d, d, vp]
        L.orc_nl_mobility.argtypes = [P, NP, vp]
        L.orc_nl_mobility.restype = ctypes.c_int
        L.orc_nl_mu_bulk.argtypes = [P, NP, d, d, d, vp]
        L.orc_nl_f_bulk.argtypes = [P, NP, d, d, d]
        L.orc_nl_f_bulk.restype = d
        L.orc_nl_init.argtypes = [P, NP] + [vp] * 7
        L.orc_nl_init.restype = ctypes.c_int
        L.orc_nl_run.argtypes = [P, NP, vp, vp, vp, ctypes.c_int64]
        L.orc_nl_run.restype = ctypes.c_int
        L.orc_nl_fields.argtypes = [P, NP] + [vp] * 10
        L.orc_nl_fields.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
        del i32
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Lattice and thermodynamics
# ---------------------------------------------------------------------------

def lattice_info(lattice: int):
    Q = 9 if lattice == D2Q9 else 27
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    lib().orc_lattice_info(lattice, c.ctypes.data_as(ctypes.c_void_p), _ptr(w))
    return c, w


def psi_eos(a, b, R, T, C, rho):
    return lib().orc_psi_eos(a, b, R, T, C, rho)


def psi_prime(a, b, R, T, C, rho):
    return lib().orc_psi_prime(a, b, R, T, C, rho)


def pressure(a, b, R, T, rho):
    return lib().orc_pressure(a, b, R, T, rho)


def dpdrho(a, b, R, T, rho):
    return lib().orc_dpdrho(a, b, R, T, rho)


def critical_temperature(a=0.037, b=0.2, R=1.0):
    rc = ctypes.c_double()
    Tc = lib().orc_critical_temperature(a, b, R, ctypes.byref(rc))
    return Tc, rc.value


def maxwell(T, a=0.037, b=0.2, R=1.0):
    """Returns (rho_g, rho_l, C, Psi0) or raises ValueError for T >= T_c."""
    out = np.zeros(4)
    if lib().orc_maxwell(a, b, R, T, _ptr(out)) != 0:
        raise ValueError("T outside (0, T_c)")
    return tuple(out)


def temperature_for_ratio(ratio, a=0.037, b=0.2, R=1.0):
    """Returns (T, rho_g, rho_l, C, Psi0) with rho_l / rho_g == ratio."""
    out = np.zeros(5)
    if lib().orc_temperature_for_ratio(a, b, R, ratio, _ptr(out)) != 0:
        raise ValueError("ratio must exceed 1")
    return tuple(out)


# Equations of state by kind: 0 Carnahan-Starling (Eq. 4), 1 van der Waals,
# 2 Peng-Robinson (acentric factor omega).
CS, VDW, PR = 0, 1, 2


def eos_psi(kind, a, b, R, omega, T, C, rho):
    return lib().orc_eos_psi(kind, a, b, R, omega, T, C, rho)


def eos_psi_prime(kind, a, b, R, omega, T, C, rho):
    return lib().orc_eos_psi_prime(kind, a, b, R, omega, T, C, rho)


def eos_pressure(kind, a, b, R, omega, T, rho):
    return lib().orc_eos_pressure(kind, a, b, R, omega, T, rho)


def eos_attraction(kind, a, b, R, omega, T):
    """a for CS and vdW; a alpha(T) for Peng-Robinson."""
    return lib().orc_eos_attraction(kind, a, b, R, omega, T)


def eos_critical_temperature(kind, a, b, R, omega=0.344):
    rc = ctypes.c_double()
    Tc = lib().orc_eos_critical_temperature(kind, a, b, R, omega, ctypes.byref(rc))
    return Tc, rc.value


def eos_maxwell(kind, T, a, b, R, omega=0.344):
    out = np.zeros(4)
    if lib().orc_eos_maxwell(kind, a, b, R, omega, T, _ptr(out)) != 0:
        raise ValueError("T outside (0, T_c)")
    return tuple(out)


def eos_temperature_for_ratio(kind, ratio, a, b, R, omega=0.344):
    out = np.zeros(5)
    if lib().orc_eos_temperature_for_ratio(kind, a, b, R, omega, ratio, _ptr(out)) != 0:
        raise ValueError("ratio must exceed 1")
    return tuple(out)


def coexisting_params(ratio: float, T: Optional[float] = None, **kw) -> Params:
    """Params at the temperature whose Maxwell density ratio is ``ratio``, or,
    if ``T`` is given, at that temperature (rho_g, rho_l and C are always the
    Maxwell construction's at the temperature used)."""
    p = Params(**kw)
    if T:
        rg, rl, C, _ = eos_maxwell(p.eos, T, p.a, p.b, p.R, p.omega)
    else:
        T, rg, rl, C, _ = eos_temperature_for_ratio(p.eos, ratio, p.a, p.b, p.R, p.omega)
    p.T, p.rho_g, p.rho_l, p.C = T, rg, rl, C
    return p


def workload_params(wl) -> Params:
    """Params of a synthetic workload: its temperature if it fixes one (a
    temperature chosen for the lattice model's own density ratio), else the
    temperature of its Maxwell density ratio."""
    return coexisting_params(wl.ratio, T=getattr(wl, "T", 0.0) or None, **wl.physics())


# ---------------------------------------------------------------------------
# Free energy pieces
# ---------------------------------------------------------------------------

def concentrations(p: Params, rho, phi):
    c1, c2 = ctypes.c_double(), ctypes.c_double()
    lib().orc_concentrations(ctypes.byref(p.c_struct()), rho, phi, ctypes.byref(c1), ctypes.byref(c2))
    return c1.value, c2.value


def gradient_coefficients(p: Params):
    out = np.zeros(3)
    lib().orc_gradient_coefficients(ctypes.byref(p.c_struct()), _ptr(out))
    return tuple(out)


def mu_bulk(p: Params, rho, phi):
    out = np.zeros(2)
    lib().orc_mu_bulk(ctypes.byref(p.c_struct()), rho, phi, _ptr(out))
    return tuple(out)


def f_bulk(p: Params, rho, phi):
    """Bulk free-energy density of Eq. (2) (Psi0 = Psi(rho_g))."""
    return lib().orc_f_bulk(ctypes.byref(p.c_struct()), float(rho), float(phi))


def bulk_pressure(p: Params, rho, phi):
    """rho mu_rho + phi mu_phi - f_B of a uniform state."""
    return lib().orc_bulk_pressure(ctypes.byref(p.c_struct()), float(rho), float(phi))


def laplacian(p: Params, psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(p.shape)
    out = np.zeros_like(psi)
    lib().orc_laplacian(ctypes.byref(p.c_struct()), _ptr(psi), _ptr(out))
    return out


def gradient(p: Params, psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(p.shape)
    out = np.zeros((3,) + p.shape)
    lib().orc_gradient(ctypes.byref(p.c_struct()), _ptr(psi), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Node-level collision pieces
# ---------------------------------------------------------------------------

def feq(lattice, rho, u):
    Q = 9 if lattice == D2Q9 else 27
    u = np.ascontiguousarray(np.resize(np.asarray(u, dtype=np.float64), 3))
    out = np.zeros(Q)
    lib().orc_feq(lattice, rho, _ptr(u), _ptr(out))
    return out


def geq(lattice, phi, mu_phi, Gamma, u, reduced=False):
    """Phase-field equilibrium on the full lattice, or (reduced) on its rest
    and axis directions (D2Q5 / D3Q7; zero elsewhere)."""
    Q = 9 if lattice == D2Q9 else 27
    u = np.ascontiguousarray(np.resize(np.asarray(u, dtype=np.float64), 3))
    out = np.zeros(Q)
    fn = lib().orc_geq_reduced if reduced else lib().orc_geq
    fn(lattice, phi, mu_phi, Gamma, _ptr(u), _ptr(out))
    return out


def kbc_split(lattice, df):
    df = np.ascontiguousarray(df, dtype=np.float64)
    ds, dh = np.zeros_like(df), np.zeros_like(df)
    lib().orc_kbc_split(lattice, _ptr(df), _ptr(ds), _ptr(dh))
    return ds, dh


def kbc_gamma(lattice, beta, feq_, ds, dh):
    return lib().orc_kbc_gamma(lattice, beta, _ptr(np.ascontiguousarray(feq_)),
                               _ptr(np.ascontiguousarray(ds)), _ptr(np.ascontiguousarray(dh)))


def collide_node(lattice, beta, f, force=(0.0, 0.0, 0.0)):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(np.resize(np.asarray(force, dtype=np.float64), 3))
    out = np.zeros_like(f)
    g = ctypes.c_double()
    lib().orc_collide_node(lattice, beta, _ptr(f), _ptr(F), _ptr(out), ctypes.byref(g))
    return out, g.value


# ---------------------------------------------------------------------------
# Whole lattice
# ---------------------------------------------------------------------------

class State:
    """Post-streaming populations f, g of shape (Q, nz, ny, nx)."""

    def __init__(self, p: Params, rho0, phi0, u0=None):
        self.p = p
        self.f = np.zeros((p.Q,) + p.shape)
        self.g = np.zeros((p.Q,) + p.shape)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(p.shape)
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.shape)
        u = None
        if u0 is not None:
            u = np.zeros((3,) + p.shape)
            u0 = np.asarray(u0, dtype=np.float64)
            u[: u0.shape[0]] = u0.reshape((u0.shape[0],) + p.shape)
        rc = lib().orc_init(ctypes.byref(p.c_struct()), _ptr(rho0), _ptr(phi0), _ptr(u),
                            _ptr(self.f), _ptr(self.g))
        if rc != 0:
            raise MemoryError("oracle init failed")
        self.steps = 0

    def run(self, nsteps: int, diag: bool = False):
        d = np.zeros((max(nsteps, 1), 10)) if diag else None
        rc = lib().orc_run(ctypes.byref(self.p.c_struct()), _ptr(self.f), _ptr(self.g),
                           int(nsteps), _ptr(d))
        if rc != 0:
            raise MemoryError("oracle run failed")
        self.steps += nsteps
        return d

    def fields(self):
        p = self.p
        sh = p.shape
        out = {k: np.zeros(sh) for k in ("rho", "phi", "c1", "c2", "mu_rho", "mu_phi")}
        out["u"] = np.zeros((3,) + sh)
        out["force"] = np.zeros((3,) + sh)
        rc = lib().orc_fields(ctypes.byref(p.c_struct()), _ptr(self.f), _ptr(self.g),
                              _ptr(out["rho"]), _ptr(out["phi"]), _ptr(out["u"]), _ptr(out["c1"]),
                              _ptr(out["c2"]), _ptr(out["mu_rho"]), _ptr(out["mu_phi"]),
                              _ptr(out["force"]))
        if rc != 0:
            raise MemoryError("oracle fields failed")
        return out


# ---------------------------------------------------------------------------
# Three liquids and the gas (the extension to more liquid components)
# ---------------------------------------------------------------------------

def nl_concentrations(p: Params, rho, phi, psi):
    out = np.zeros(3)
    lib().orc_nl_concentrations(ctypes.byref(p.c_struct()), float(rho), float(phi), float(psi), _ptr(out))
    return tuple(out)


def nl_mobility(p: Params, nl: NLParams) -> np.ndarray:
    """The (phi, psi) mobility matrix divided by M."""
    out = np.zeros(4)
    if lib().orc_nl_mobility(ctypes.byref(p.c_struct()), ctypes.byref(nl.c_struct()), _ptr(out)) != 0:
        raise ValueError("the consistent mobility needs positive kappas")
    return out.reshape(2, 2)


def nl_mu_bulk(p: Params, nl: NLParams, rho, phi, psi):
    out = np.zeros(3)
    lib().orc_nl_mu_bulk(ctypes.byref(p.c_struct()), ctypes.byref(nl.c_struct()), float(rho), float(phi),
                         float(psi), _ptr(out))
    return tuple(out)


def nl_f_bulk(p: Params, nl: NLParams, rho, phi, psi):
    return lib().orc_nl_f_bulk(ctypes.byref(p.c_struct()), ctypes.byref(nl.c_struct()), float(rho), float(phi),
                               float(psi))


class NLState:
    """Post-streaming populations f, g, h of shape (Q, nz, ny, nx) of the
    three-liquid model."""

    def __init__(self, p: Params, nl: NLParams, rho0, phi0, psi0, u0=None):
        self.p, self.nl = p, nl
        self.f = np.zeros((p.Q,) + p.shape)
        self.g = np.zeros((p.Q,) + p.shape)
        self.h = np.zeros((p.Q,) + p.shape)
        arr = [np.ascontiguousarray(v, dtype=np.float64).reshape(p.shape) for v in (rho0, phi0, psi0)]
        u = None
        if u0 is not None:
            u = np.zeros((3,) + p.shape)
            u0 = np.asarray(u0, dtype=np.float64)
            u[: u0.shape[0]] = u0.reshape((u0.shape[0],) + p.shape)
        rc = lib().orc_nl_init(ctypes.byref(p.c_struct()), ctypes.byref(nl.c_struct()), *(_ptr(v) for v in arr),
                               _ptr(u), _ptr(self.f), _ptr(self.g), _ptr(self.h))
        if rc != 0:
            raise ValueError("three-liquid oracle init failed (walls, reduced lattice or kappa <= 0?)")
        self.steps = 0

    def run(self, nsteps: int):
        rc = lib().orc_nl_run(ctypes.byref(self.p.c_struct()), ctypes.byref(self.nl.c_struct()), _ptr(self.f),
                              _ptr(self.g), _ptr(self.h), int(nsteps))
        if rc != 0:
            raise MemoryError("three-liquid oracle run failed")
        self.steps += nsteps

    def fields(self):
        sh = self.p.shape
        out = {k: np.zeros(sh) for k in ("rho", "phi", "psi")}
        for k in ("u", "c", "mu", "force"):
            out[k] = np.zeros((3,) + sh)
        rc = lib().orc_nl_fields(ctypes.byref(self.p.c_struct()), ctypes.byref(self.nl.c_struct()), _ptr(self.f),
                                 _ptr(self.g), _ptr(self.h), _ptr(out["rho"]), _ptr(out["phi"]), _ptr(out["psi"]),
                                 _ptr(out["u"]), _ptr(out["c"]), _ptr(out["mu"]), _ptr(out["force"]))
        if rc != 0:
            raise MemoryError("three-liquid oracle fields failed")
        return out


def discrete_coexistence(p: Params, steps: int = 20000, n: int = 256, width: float = 2.0):
    """(rho_g, rho_l) of a relaxed flat slab of liquid 1 in gas with p's free
    energy on p's lattice: the discretised model's own coexistence densities."""
    import dataclasses
    q = dataclasses.replace(p, nx=n, ny=1, nz=1)
    x = np.arange(n, dtype=np.float64)
    c1 = 0.5 * (np.tanh((x - n / 4) / width) - np.tanh((x - 3 * n / 4) / width))
    st = State(q, (p.rho_g + (p.rho_l - p.rho_g) * c1).reshape(1, 1, n), (q.chi * c1).reshape(1, 1, n))
    st.run(steps)
    r = st.fields()["rho"]
    return float(r[0, 0, 0]), float(r[0, 0, n // 2])


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
