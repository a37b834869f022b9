"""The allocation-free decode (telbm_surrogate_decode_noalloc) against the
workspace decode (telbm_surrogate_decode), both called through the C ABI:
bit-identical outputs on two calls in a row, the second with a smaller input
(the static workspace keeps the first call's contents), and a size beyond the
static workspace rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(rng, n, h, w):
    import torch
    rho_g, rho_l, chi = 0.7, 7.0, 5.0
    s = rng.uniform(0, 1, size=(n, h, w))
    q = rng.uniform(-1, 1, size=(n, h, w)) * s
    rho = rho_g + (rho_l - rho_g) * s
    phi = chi * q
    ux, uy = rng.normal(size=(2, n, h, w)) * 0.01
    y = (rng.normal(size=(n, h, w, 32)) * 0.2).astype(np.float32)
    dev = [torch.from_numpy(a).cuda() for a in (rho, phi, ux, uy)]
    return torch.from_numpy(y).cuda(), dev, (rho_g, rho_l, chi)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def test_noalloc_decode_matches_workspace_decode():
    import torch
    from paper_1710_07486_amd import surrogate as S
    L = S._load()
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    rng = np.random.default_rng(11)
    assert L.telbm_surrogate_decode_noalloc_max_bytes() == 16 << 20
    for n, h, w in ((3, 96, 130), (2, 40, 33)):
        print("[case] noalloc decode", n, h, w, flush=True)
        y, (rho, phi, ux, uy), (rho_g, rho_l, chi) = _inputs(rng, n, h, w)
        ref = [torch.empty_like(rho) for _ in range(4)]
        got = [torch.full_like(rho, np.nan) for _ in range(4)]
        b = ctypes.c_size_t()
        assert L.telbm_surrogate_decode_workspace_bytes(n, h, w, ctypes.byref(b)) == 0
        ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
        assert L.telbm_surrogate_decode(_p(y), _p(rho), _p(phi), _p(ux), _p(uy), n, h, w, rho_g, rho_l, chi, S.U_SCALE,
                                        *[_p(t) for t in ref], _p(ws), ws.numel(), sp) == 0
        assert L.telbm_surrogate_decode_noalloc(_p(y), _p(rho), _p(phi), _p(ux), _p(uy), n, h, w, rho_g, rho_l, chi,
                                                S.U_SCALE, *[_p(t) for t in got], sp) == 0
        torch.cuda.synchronize()
        for a, b_ in zip(ref, got):
            assert torch.equal(a, b_)
        # the decode restores each image's total density (what it conserves)
        for k in range(n):
            assert abs(float(got[0][k].sum() / rho[k].sum()) - 1) < 1e-12


def test_noalloc_decode_rejects_sizes_beyond_the_static_workspace():
    from paper_1710_07486_amd import surrogate as S
    from paper_1710_07486_amd import _lib
    L = S._load()
    b = ctypes.c_size_t()
    n, h, w = 40, 256, 256
    assert L.telbm_surrogate_decode_workspace_bytes(n, h, w, ctypes.byref(b)) == 0
    assert b.value > L.telbm_surrogate_decode_noalloc_max_bytes()
    dummy = ctypes.c_void_p(256)
    rc = L.telbm_surrogate_decode_noalloc(dummy, dummy, dummy, None, None, n, h, w, 0.7, 7.0, 5.0, S.U_SCALE,
                                          dummy, dummy, dummy, dummy, None)
    assert rc == _lib.ERR_NOMEM
