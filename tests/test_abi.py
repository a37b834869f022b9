"""CPU checks of the C ABI library: it loads, exports every symbol that
include/telbm.h declares, validates parameters before touching a device, and
its host thermodynamics (an implementation independent of the oracle's)
agree with the oracle.  No compute call is made here: no GPU is needed."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(telbm_\w+)\s*\(", text, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1710_07486_amd import _lib
    return _lib.load()


def test_header_declares_the_problem_calls():
    names = declared_symbols()
    for must in ("telbm_create", "telbm_init_fields", "telbm_step", "telbm_read", "telbm_diagnostics",
                 "telbm_destroy", "telbm_coexistence", "telbm_required_bytes", "telbm_set_stream"):
        assert must in names, must


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_prototypes_cover_header():
    import importlib
    from paper_1710_07486_amd import _lib
    covered = set(_lib.PROTOTYPES)
    for mod in ("batch", "surrogate"):
        try:
            covered |= set(importlib.import_module("paper_1710_07486_amd." + mod).PROTOTYPES)
        except ImportError:
            pass
    assert set(declared_symbols()) <= covered, set(declared_symbols()) - covered


def test_library_thermodynamics_match_oracle(orc):
    import paper_1710_07486_amd as T
    Tc_l = T.critical_temperature()
    Tc_o, _ = orc.critical_temperature()
    assert abs(Tc_l / Tc_o - 1) < 1e-12
    for tr in (0.45, 0.485, 0.6, 0.8, 0.95):
        rg, rl, C, p0 = T.coexistence(tr * Tc_o)
        og, ol, oC, op0 = orc.maxwell(tr * Tc_o)
        assert abs(rg / og - 1) < 1e-9 and abs(rl / ol - 1) < 1e-11
        assert abs(C - oC) < 1e-11 and abs(p0 - op0) < 1e-12
    for ratio in (10.0, 150.0, 1000.0):
        assert abs(T.temperature_for_ratio(ratio) / orc.temperature_for_ratio(ratio)[0] - 1) < 1e-11


@pytest.mark.parametrize("kind,a,b", [(1, 9.0 / 49.0, 2.0 / 21.0), (2, 2.0 / 49.0, 2.0 / 21.0)], ids=["vdw", "pr"])
def test_library_thermodynamics_match_oracle_other_eos(orc, kind, a, b):
    """The library's van der Waals and Peng-Robinson critical point, Maxwell
    construction and temperature for a ratio against the oracle's (written
    apart: spinodal curve and chemical-potential shooting in the library,
    golden-section critical point and pressure bisection in the oracle)."""
    import paper_1710_07486_amd as T
    Tc_l = T.critical_temperature(a, b, 1.0, kind)
    Tc_o, _ = orc.eos_critical_temperature(kind, a, b, 1.0)
    assert abs(Tc_l / Tc_o - 1) < 1e-12
    for tr in (0.95, 0.8, 0.6, 0.5):
        rg, rl, C, p0 = T.coexistence(tr * Tc_o, a, b, 1.0, kind)
        og, ol, oC, op0 = orc.eos_maxwell(kind, tr * Tc_o, a, b, 1.0)
        assert abs(rg / og - 1) < 1e-11 and abs(rl / ol - 1) < 1e-11
        assert abs(C - oC) < 1e-11 and abs(p0 - op0) < 1e-11
    for ratio in (10.0, 1000.0):
        assert abs(T.temperature_for_ratio(ratio, a, b, 1.0, kind) /
                   orc.eos_temperature_for_ratio(kind, ratio, a, b, 1.0)[0] - 1) < 1e-11


def test_unknown_eos_is_rejected(orc):
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib
    p = T.Params(T=T.temperature_for_ratio(10.0), eos=3)
    with pytest.raises(_lib.TelbmError):
        T.required_bytes(p)
    with pytest.raises(_lib.TelbmError):
        T.critical_temperature(0.037, 0.2, 1.0, 3)


def test_parameter_validation_without_device(orc):
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib
    T0 = orc.temperature_for_ratio(10.0)[0]
    good = T.Params(nx=16, ny=16, T=T0)
    assert T.required_bytes(good) >= 2 * 18 * 256 * 8
    bad = [dict(T=0.5), dict(T=-1.0), dict(nz=2), dict(nx=0), dict(nu=0.0), dict(tau_phi=0.5),
           dict(chi=0.0), dict(lattice=7), dict(precision=3), dict(rho_g=2.0, rho_l=1.0),
           dict(mobility=-1.0)]
    for kw in bad:
        p = T.Params(nx=16, ny=16, T=T0)
        for k, v in kw.items():
            setattr(p, k, v)
        with pytest.raises(T.TelbmError) as e:
            T.required_bytes(p)
        assert e.value.code == _lib.ERR_INVAL, kw
    # the arena of the mixed-precision form is about half
    big = T.Params(nx=256, ny=256, T=T0)
    mixed = T.Params(nx=256, ny=256, T=T0, precision=T.FP32_MIXED)
    assert T.required_bytes(mixed) < 0.7 * T.required_bytes(big)
    p3 = T.Params(lattice=T.D3Q27, nx=8, ny=8, nz=8, T=T0)
    assert T.required_bytes(p3) >= 2 * 54 * 512 * 8


def test_lattices_beyond_32_bit_offsets_are_rejected(orc):
    """The kernels address each FP64 slice of N values with 32-bit byte
    offsets: N = 2^29 is refused (single solver and batch member), N just
    below is accepted, in 2D and 3D."""
    import ctypes
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib
    T0 = orc.temperature_for_ratio(10.0)[0]
    for kw in (dict(nx=1 << 15, ny=1 << 14), dict(lattice=T.D3Q27, nx=1 << 10, ny=1 << 10, nz=1 << 9)):
        p = T.Params(T=T0, **kw)
        with pytest.raises(T.TelbmError) as e:
            T.required_bytes(p)
        assert e.value.code == _lib.ERR_INVAL
        arr = (_lib.TelbmParams * 1)(p.c_struct())
        n = ctypes.c_size_t()
        assert _lib.load().telbm_batch_required_bytes(arr, 1, ctypes.byref(n)) == _lib.ERR_INVAL
    ok = T.Params(T=T0, nx=(1 << 15) - 1, ny=1 << 14)
    assert T.required_bytes(ok) > 0


def test_null_arguments_are_rejected(lib):
    from paper_1710_07486_amd import _lib
    assert lib.telbm_step(None, 1) == _lib.ERR_INVAL
    assert lib.telbm_read(None, 0, None, 0) == _lib.ERR_INVAL
    assert lib.telbm_destroy(None) == _lib.ERR_INVAL
    assert lib.telbm_required_bytes(None, None) == _lib.ERR_INVAL
    assert lib.telbm_coexistence(0.037, 0.2, 1.0, 1.0, None, None, None, None) == _lib.ERR_INVAL


def test_wall_parameters_are_validated(orc):
    """Walls: accepted on D2Q9 and D3Q27 in both precisions and in the
    batched form (members with and without walls); rejected with ny < 2, with
    contact angles outside (0, pi) and with walls other than 0/1."""
    import math
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib
    from paper_1710_07486_amd.batch import required_bytes as batch_bytes
    T0 = orc.temperature_for_ratio(10.0)[0]
    for kw in (dict(), dict(precision=T.FP32_MIXED), dict(lattice=T.D3Q27, nz=8),
               dict(lattice=T.D3Q27, nz=8, precision=T.FP32_MIXED)):
        assert T.required_bytes(T.Params(nx=16, ny=16, T=T0, walls=1, **kw)) > 0
    bad = [dict(ny=1), dict(theta_rho_lo=0.0),
           dict(theta_phi_hi=math.pi), dict(theta_rho_hi=float("nan")), dict(walls=2)]
    for kw in bad:
        p = T.Params(nx=16, ny=16, T=T0, walls=1)
        for k, v in kw.items():
            setattr(p, k, v)
        with pytest.raises(T.TelbmError) as e:
            T.required_bytes(p)
        assert e.value.code == _lib.ERR_INVAL, kw
    assert batch_bytes([T.Params(nx=16, ny=16, T=T0, walls=1), T.Params(nx=24, ny=16, T=T0)]) > 0
    with pytest.raises(T.TelbmError):
        batch_bytes([T.Params(nx=16, ny=16, T=T0, walls=1, theta_rho_lo=0.0)])


def test_reduced_phase_field_lattice_parameters(orc):
    """glattice 1: accepted on D2Q9 (both precisions) and D3Q27 FP64, with a
    smaller arena and algorithmic byte count; rejected on D3Q27 FP32-mixed,
    with other values, and in the batched form."""
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib
    from paper_1710_07486_amd.batch import required_bytes as batch_bytes
    T0 = orc.temperature_for_ratio(10.0)[0]
    full = T.required_bytes(T.Params(nx=256, ny=256, T=T0))
    red = T.required_bytes(T.Params(nx=256, ny=256, T=T0, glattice=1))
    assert red < full
    assert T.required_bytes(T.Params(lattice=T.D3Q27, nx=8, ny=8, nz=8, T=T0, glattice=1)) > 0
    for kw in (dict(lattice=T.D3Q27, nz=8, precision=T.FP32_MIXED, glattice=1), dict(glattice=2)):
        p = T.Params(nx=16, ny=16, T=T0)
        for k, v in kw.items():
            setattr(p, k, v)
        with pytest.raises(T.TelbmError) as e:
            T.required_bytes(p)
        assert e.value.code == _lib.ERR_INVAL, kw
    with pytest.raises(T.TelbmError):
        batch_bytes([T.Params(nx=16, ny=16, T=T0, glattice=1)])


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library every entry (solver, batch, surrogate
    kernels) raises: there is no CPU fallback."""
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd import _lib as L
    from paper_1710_07486_amd import batch as B
    from paper_1710_07486_amd import surrogate as S
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libtelbm.so")
    for call in (L.load, B._load, S._load, lambda: T.temperature_for_ratio(100.0)):
        with pytest.raises(ImportError, match="is missing"):
            call()
    # the solver refuses first for want of a GPU where there is none
    with pytest.raises((ImportError, RuntimeError)):
        T.Solver(T.Params(nx=8, ny=8, T=0.03, rho_g=0.1, rho_l=1.0))


def test_three_liquid_mobility_matches_oracle(orc):
    """The library's closed-form mobility matrix (host) against the oracle's
    product of the concentration mobility with the pseudo-inverse maps."""
    import numpy as np
    from paper_1710_07486_amd import nliquid as NL
    import paper_1710_07486_amd as T
    rng = np.random.default_rng(11)
    T0 = orc.temperature_for_ratio(10.0)[0]
    for _ in range(8):
        k2, k3, k4 = rng.uniform(0.01, 0.2, 3)
        p = T.Params(nx=16, ny=16, T=T0, kappa2=k2, kappa3=k3)
        m_lib = NL.mobility(p, NL.NLParams(kappa4=k4))
        m_orc = orc.nl_mobility(orc.coexisting_params(10.0, kappa2=k2, kappa3=k3), orc.NLParams(kappa4=k4))
        assert np.allclose(m_lib, m_orc, rtol=1e-13, atol=1e-15), (m_lib, m_orc)


def test_three_liquid_parameters_are_validated(orc):
    """Accepted on D2Q9 and D3Q27 FP64; rejected in the FP32-mixed form, with
    walls, with the reduced phase-field lattice and with a kappa <= 0."""
    from paper_1710_07486_amd import _lib
    from paper_1710_07486_amd import nliquid as NL
    import paper_1710_07486_amd as T
    T0 = orc.temperature_for_ratio(10.0)[0]
    q = NL.NLParams()
    assert NL.required_bytes(T.Params(nx=16, ny=16, T=T0), q) >= 2 * 3 * 9 * 256 * 8 + 6 * 256 * 8
    assert NL.required_bytes(T.Params(lattice=T.D3Q27, nx=8, ny=8, nz=8, T=T0), q) >= 2 * 3 * 27 * 512 * 8
    bad = [(dict(precision=T.FP32_MIXED), q), (dict(walls=1), q), (dict(glattice=1), q), (dict(kappa3=0.0), q),
           (dict(), NL.NLParams(kappa4=-0.1)), (dict(), NL.NLParams(lambda4=float("nan")))]
    for kw, qq in bad:
        p = T.Params(nx=16, ny=16, T=T0)
        for k, v in kw.items():
            setattr(p, k, v)
        with pytest.raises(T.TelbmError) as e:
            NL.required_bytes(p, qq)
        assert e.value.code == _lib.ERR_INVAL, kw
