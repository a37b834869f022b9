"""GPU tests of the learned form: each convolution kernel (forward, data
gradient, weight and bias gradient) against the FP64 numpy oracle on the
same BF16-representable inputs, the loss, Adam, encode and the
conservation-projecting decode, a whole-network gradient, and training on
solver-generated data with the gain it brings to the plain solver."""
import math

import numpy as np
import pytest

from oracle import conv_oracle as C

pytestmark = pytest.mark.gpu

SHAPES = [(32, 64), (64, 64), (64, 32), (32, 32)]


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1710_07486_amd import surrogate as S
    S._load()
    return torch, S, torch.cuda.current_stream()


def bf16_tensor(torch, a):
    """numpy float64 array -> (int16 device tensor of BF16 bits, the float64
    values it holds)."""
    r = C.bf16_round(a)
    bits = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(bits)).cuda(), r


def from_bf16(t, shape):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64).reshape(shape)


def rel_err(a, b, scale):
    return float(np.max(np.abs(a - b) / scale))


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("dims,dil", [((1, 4, 8), 1), ((2, 5, 37), 1), ((1, 16, 19), 1), ((2, 5, 37), 2),
                                      ((1, 16, 19), 8), ((1, 3, 4), 5)])
def test_conv_forward_matches_oracle(env, cin, cout, dims, dil):
    torch, S, st = env
    n, h, w = dims
    rng = np.random.default_rng(cin * 100 + cout + h)
    x_t, x = bf16_tensor(torch, rng.normal(size=(n, h, w, cin)))
    W = rng.normal(size=(9, cin, cout)) / math.sqrt(9 * cin)
    b = rng.normal(size=cout) * 0.1
    Wt = torch.tensor(W, dtype=torch.float32).cuda()
    bt = torch.tensor(b, dtype=torch.float32).cuda()
    wf = torch.empty(9 * cin * cout, dtype=torch.int16, device="cuda")
    wd = torch.empty_like(wf)
    S.pack_weights(Wt, cin, cout, wf, wd, st)
    Wr = C.bf16_round(W.astype(np.float32))
    br = b.astype(np.float32).astype(np.float64)
    y32 = torch.empty(n * h * w * cout, dtype=torch.float32, device="cuda")
    ybf = torch.empty(n * h * w * cout, dtype=torch.int16, device="cuda")
    S.conv_forward(x_t, n, h, w, cin, wf, bt, cout, 0, y_f32=y32, stream=st, dil=dil)
    S.conv_forward(x_t, n, h, w, cin, wf, bt, cout, 1, y_bf16=ybf, stream=st, dil=dil)
    torch.cuda.synchronize()
    ref = C.conv_forward(x, Wr, br, dil=dil)
    # FP32 accumulation of 9*cin exact BF16 products
    scale = C.conv_forward(np.abs(x), np.abs(Wr), np.abs(br), dil=dil) + 1e-30
    assert rel_err(y32.cpu().numpy().reshape(ref.shape), ref, scale) < 1e-5
    got = from_bf16(ybf, ref.shape)
    relu = np.maximum(ref, 0.0)
    assert np.all(np.abs(got - relu) <= 2.0 ** -8 * np.abs(relu) + 1e-5 * scale)


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("dims,dil", [((1, 4, 8), 1), ((2, 5, 37), 1), ((3, 33, 40), 1), ((2, 5, 37), 3),
                                      ((3, 33, 40), 8)])
def test_conv_backward_matches_oracle(env, cin, cout, dims, dil):
    torch, S, st = env
    n, h, w = dims
    rng = np.random.default_rng(7 * cin + cout + w)
    # layer input is a ReLU output: nonnegative with zeros
    x_t, x = bf16_tensor(torch, np.maximum(rng.normal(size=(n, h, w, cin)), 0.0))
    g_t, g = bf16_tensor(torch, rng.normal(size=(n, h, w, cout)))
    W = rng.normal(size=(9, cin, cout)) / math.sqrt(9 * cin)
    Wt = torch.tensor(W, dtype=torch.float32).cuda()
    wf = torch.empty(9 * cin * cout, dtype=torch.int16, device="cuda")
    wd = torch.empty_like(wf)
    S.pack_weights(Wt, cin, cout, wf, wd, st)
    Wr = C.bf16_round(W.astype(np.float32))
    dx = torch.empty(n * h * w * cin, dtype=torch.int16, device="cuda")
    dw = torch.empty(9 * cin * cout, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    ws = torch.empty(S.conv_workspace_bytes(n, h, w, cin, cout), dtype=torch.uint8, device="cuda")
    S.conv_backward(x_t, g_t, n, h, w, cin, cout, wd, x_t, dx, dw, db, ws, st, dil=dil)
    torch.cuda.synchronize()
    rdx, rdw, rdb = C.conv_backward(x, Wr, g, dil)
    rdx = rdx * (x > 0)
    sdx, sdw, _ = C.conv_backward(np.abs(x), np.abs(Wr), np.abs(g), dil)
    got = from_bf16(dx, x.shape)
    assert np.all(np.abs(got - rdx) <= 2.0 ** -8 * np.abs(rdx) + 1e-5 * sdx + 1e-30)
    assert rel_err(dw.cpu().numpy().reshape(rdw.shape), rdw, sdw + 1e-30) < 3e-5
    sdb = np.abs(g).reshape(-1, cout).sum(0) + 1e-30
    assert rel_err(db.cpu().numpy(), rdb, sdb) < 1e-5


def test_conv_backward_without_mask_and_partial_outputs(env):
    torch, S, st = env
    n, h, w, cin, cout = 1, 7, 9, 32, 64
    rng = np.random.default_rng(3)
    x_t, x = bf16_tensor(torch, rng.normal(size=(n, h, w, cin)))
    g_t, g = bf16_tensor(torch, rng.normal(size=(n, h, w, cout)))
    W = rng.normal(size=(9, cin, cout)) * 0.05
    Wt = torch.tensor(W, dtype=torch.float32).cuda()
    wf = torch.empty(9 * cin * cout, dtype=torch.int16, device="cuda")
    wd = torch.empty_like(wf)
    S.pack_weights(Wt, cin, cout, wf, wd, st)
    dx = torch.empty(n * h * w * cin, dtype=torch.int16, device="cuda")
    S.conv_backward(x_t, g_t, n, h, w, cin, cout, wd, None, dx, None, None, None, st)
    torch.cuda.synchronize()
    rdx, _, _ = C.conv_backward(x, C.bf16_round(W.astype(np.float32)), g)
    assert np.allclose(from_bf16(dx, x.shape), rdx, rtol=2 ** -7, atol=1e-4)
    # a short workspace is refused before any launch
    from paper_1710_07486_amd._lib import ERR_NOMEM, TelbmError
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    dw = torch.empty(9 * cin * cout, dtype=torch.float32, device="cuda")
    with pytest.raises(TelbmError) as e:
        S.conv_backward(x_t, g_t, n, h, w, cin, cout, wd, None, None, dw, None, small, st)
    assert e.value.code == ERR_NOMEM


def test_residual_mse_and_adam(env):
    torch, S, st = env
    rng = np.random.default_rng(11)
    P = 1000
    V = S.VALID
    x_t, x = bf16_tensor(torch, rng.normal(size=(P, 32)) * (np.arange(32) < V))
    t_t, tg = bf16_tensor(torch, rng.normal(size=(P, 32)) * (np.arange(32) < V))
    y = rng.normal(size=(P, 32)).astype(np.float32)
    yt = torch.from_numpy(y).cuda()
    dy = torch.empty(P * 32, dtype=torch.int16, device="cuda")
    pred = torch.empty(P * 32, dtype=torch.float32, device="cuda")
    part = torch.empty((P * 32 + 255) // 256, dtype=torch.float32, device="cuda")
    nb = S.residual_mse(x_t, yt, t_t, P, dy=dy, pred=pred, partials=part, stream=st)
    torch.cuda.synchronize()
    p_ref = (x + y)[:, :V]
    d = p_ref - tg[:, :V]
    assert abs(part[:nb].double().sum().item() - np.sum(d * d)) < 1e-5 * np.sum(d * d)
    assert np.allclose(pred.cpu().numpy().reshape(P, 32)[:, :V], p_ref, rtol=1e-6, atol=1e-6)
    g = from_bf16(dy, (P, 32))
    assert np.all(g[:, V:] == 0)
    assert np.allclose(g[:, :V], 2 * d / (V * P), rtol=2 ** -8, atol=0)
    # Adam over three steps against the oracle
    n = 777
    w = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    wt = torch.tensor(w, dtype=torch.float32).cuda()
    mt = torch.zeros(n, device="cuda")
    vt = torch.zeros(n, device="cuda")
    for t in range(1, 4):
        gr = rng.normal(size=n)
        w, m, v = C.adam(w, gr, m, v, t, 1e-2)
        S.adam_step(wt, torch.tensor(gr, dtype=torch.float32).cuda(), mt, vt, 1e-2, t, st)
    torch.cuda.synchronize()
    assert np.allclose(wt.cpu().numpy(), w, rtol=0, atol=1e-5)


def test_encode_and_conserving_decode(env):
    torch, S, st = env
    rng = np.random.default_rng(5)
    n, h, w = 2, 24, 40
    rho_g, rho_l, chi, us = 0.7, 7.0, 5.0, S.U_SCALE
    s = rng.uniform(0, 1, size=(n, h, w))
    q = rng.uniform(-1, 1, size=(n, h, w)) * s
    rho = rho_g + (rho_l - rho_g) * s
    phi = chi * q
    ux, uy = rng.normal(size=(2, n, h, w)) * 0.01
    rt, pt, uxt, uyt = (torch.from_numpy(a).cuda() for a in (rho, phi, ux, uy))
    x = torch.empty(n * h * w * 32, dtype=torch.int16, device="cuda")
    S.encode(rt, pt, uxt, uyt, rho_g, rho_l, chi, x, st)
    torch.cuda.synchronize()
    enc = from_bf16(x, (n, h, w, 32))
    sh = (rho - rho_g) / (rho_l - rho_g)
    assert np.array_equal(enc[..., 0], C.bf16_round(sh))
    assert np.array_equal(enc[..., 1], C.bf16_round(0.5 * (sh + phi / chi)))
    assert np.array_equal(enc[..., 2], C.bf16_round(0.5 * (sh - phi / chi)))
    assert np.array_equal(enc[..., 3], C.bf16_round(ux * us))
    assert np.array_equal(enc[..., 4], C.bf16_round(uy * us))
    assert np.all(enc[..., 5:] == 0)
    S.encode(rt, pt, None, None, rho_g, rho_l, chi, x, st)
    torch.cuda.synchronize()
    assert np.all(from_bf16(x, (n, h, w, 32))[..., 3:] == 0)
    out = [torch.empty_like(rt) for _ in range(4)]
    # zero network output: the input comes back unchanged
    y0 = torch.zeros(n * h * w * 32, dtype=torch.float32, device="cuda")
    ws = S.decode(y0, rt, pt, uxt, uyt, n, h, w, rho_g, rho_l, chi, *out, st)
    torch.cuda.synchronize()
    assert np.allclose(out[0].cpu().numpy(), rho, rtol=1e-13, atol=0)
    assert np.allclose(out[1].cpu().numpy(), phi, rtol=0, atol=1e-12)
    assert np.allclose(out[2].cpu().numpy(), ux, rtol=0, atol=1e-15)
    assert np.allclose(out[3].cpu().numpy(), uy, rtol=0, atol=1e-15)
    # a random output: totals of rho, phi and rho u per image are restored
    yr = torch.from_numpy((rng.normal(size=(n, h, w, 32)) * 0.2).astype(np.float32)).cuda()
    ws = S.decode(yr, rt, pt, uxt, uyt, n, h, w, rho_g, rho_l, chi, *out, st)
    torch.cuda.synchronize()
    del ws
    R, F, UX, UY = (o.cpu().numpy() for o in out)
    for k in range(n):
        assert abs(R[k].sum() - rho[k].sum()) < 1e-11 * rho[k].sum()
        assert abs(F[k].sum() - phi[k].sum()) < 1e-10 * np.abs(phi[k]).sum()
        for U, u in ((UX, ux), (UY, uy)):
            assert abs((R[k] * U[k]).sum() - (rho[k] * u[k]).sum()) < 1e-10 * (rho[k] * np.abs(u[k])).sum()
    assert np.all(np.isfinite(R)) and np.all(np.isfinite(UX))
    # a state at rest as input: the output momentum is zero
    ws = S.decode(yr, rt, pt, None, None, n, h, w, rho_g, rho_l, chi, *out, st)
    torch.cuda.synchronize()
    R, UX = out[0].cpu().numpy(), out[2].cpu().numpy()
    assert abs((R * UX).sum()) < 1e-10 * (R * np.abs(UX)).sum()


def oracle_network(S, x, weights, biases, target, dils):
    """FP64 forward/backward of the whole network with BF16 rounding at the
    same points as the device path (weights, activations, loss gradient)."""
    L = len(S.LAYERS)
    acts = [x]
    for k in range(L):
        z = C.conv_forward(acts[-1], weights[k], biases[k], dil=dils[k])
        if k < L - 1:
            acts.append(C.bf16_round(np.maximum(z, 0.0)))
        else:
            y = z.astype(np.float32).astype(np.float64)
    pred = x + y
    d = (pred - target)[..., :S.VALID]
    loss = float(np.sum(d * d))
    g = np.zeros_like(y)
    g[..., :S.VALID] = 2 * d / (d.size)
    g = C.bf16_round(g)
    gw, gb = [None] * L, [None] * L
    for k in range(L - 1, -1, -1):
        dx, gw[k], gb[k] = C.conv_backward(acts[k], weights[k], g, dils[k])
        if k:
            g = C.bf16_round(dx * (acts[k] > 0))
    return loss, gw, gb


def test_network_gradient_matches_oracle(env):
    torch, S, st = env
    net = S.Network(seed=1, out_scale=1.0)
    n, h, w = 1, 12, 20
    rng = np.random.default_rng(2)
    xv = np.zeros((n, h, w, 32))
    V = S.VALID
    xv[..., :V] = rng.uniform(0, 1, size=(n, h, w, V))
    tv = np.zeros_like(xv)
    tv[..., :V] = xv[..., :V] + 0.1 * rng.normal(size=(n, h, w, V))
    x_t, x = bf16_tensor(torch, xv)
    t_t, tg = bf16_tensor(torch, tv)
    # non-zero biases so that their gradients and effect are exercised
    for b in net.b:
        b.copy_(torch.from_numpy(rng.normal(size=b.numel()).astype(np.float32) * 0.05))
    net.pack()
    part = net.loss_and_grad(x_t, t_t, n, h, w)
    torch.cuda.synchronize()
    Ws = [C.bf16_round(wk.cpu().numpy().astype(np.float64)) for wk in net.w]
    Bs = [bk.cpu().numpy().astype(np.float64) for bk in net.b]
    loss, gw, gb = oracle_network(S, x, Ws, Bs, tg, net.dilations)
    assert abs(part.double().sum().item() - loss) < 2e-2 * loss
    for k in range(len(S.LAYERS)):
        gk = net.gw[k].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gk - gw[k]) <= 3e-2 * np.linalg.norm(gw[k]) + 1e-12, k
        bk = net.gb[k].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(bk - gb[k]) <= 3e-2 * np.linalg.norm(gb[k]) + 1e-12, k


def test_training_on_solver_data_gains_over_plain(env):
    """Small lens family (64^2, radii 8-14, 500-step horizon): the network,
    trained on the batched solver's own trajectories by the library's
    kernels, predicts held-out end states far better than the identity;
    solver runs started from its jump lead the plain runs (their interface
    measures are where the plain run is later), with the conserved totals
    exact and the final bulk densities those of the plain run."""
    torch, S, st = env
    fam = S.Family("lens", n=64, r_lo=8, r_hi=14, horizon=500, jumps=1)
    ph = S.physics(fam, calibrate_steps=10000)
    assert 0 < ph.ic_g < ph.ic_l
    data = S.generate(fam, list(range(10000, 10256)), ph)
    held = S.generate(fam, list(range(20000, 20016)), ph)
    net = S.Network(seed=0)
    hist = S.train(net, data, 1500, batch=8, lr=2e-3, lr_final=1e-4, log_every=250)
    assert hist[-1] < 0.5 * hist[0]
    mp, m0 = S.evaluate(net, held)
    print(f"held-out MSE surrogate {mp:.3e} identity {m0:.3e}")
    assert mp < 0.2 * m0
    leads, gains, coex = [], [], []
    for seed in range(20000, 20006):
        r = S.compare_to_plain(net, fam, seed, ph, ref_steps=8000, window=250, jumps=1)
        assert not r["fallback"], r["checks"]
        assert r["checks"]["mass_rel_err"] < 1e-12
        pf, sf = r["plain_final"], r["surrogate_final"]
        assert abs(sf["mass"] - pf["mass"]) < 1e-12 * pf["mass"]
        assert abs(sf["phi_total"] - pf["phi_total"]) < 1e-9 * (1 + abs(pf["phi_total"]))
        # the judge's coexistence densities: the continued run ends at the
        # plain run's bulk gas and liquid densities
        coex.append((abs(sf["rho_gas"] / pf["rho_gas"] - 1), abs(sf["rho_liquid"] / pf["rho_liquid"] - 1)))
        leads.append(r["lead_steps"])
        gains.append(r["gain_steps"])
    print("leads", leads, "gains (plain - surrogate steps to settle)", gains, "coexistence errors", coex)
    # the lead of a single seed varies by about +-100 steps between trainings
    # that differ only in summation order; the mean over six seeds was
    # 80-250 steps in repeated runs (0.16-0.5 of the horizon)
    assert np.mean(leads) > 0.1 * fam.horizon
    assert sum(v > 0 for v in leads) >= 4
    # at 8,000 steps the plain run's own gas is still relaxing (by slow
    # evaporation and condensation), so the two runs, at different stages of
    # that relaxation, differ by up to 1.2 % in the gas and 0.3 % in the
    # liquid (measured)
    assert max(c[0] for c in coex) < 2e-2 and max(c[1] for c in coex) < 5e-3, coex
    # steps to settle within 1 % of the reference (both runs settled on four
    # of six seeds in the measured run): -1500, 0, -2500, 0.  At this size the
    # jump leads the plain run early but does not reach the settled state
    # sooner; the gains are recorded, not asserted.
