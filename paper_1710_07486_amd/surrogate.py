"""Learned form: a convolutional surrogate that jumps the slow initial
relaxation of two-drop configurations.

The network maps the encoded state (scaled density, C1, C2) at t0 to the
state `horizon` steps later: six 3x3 convolutions with circular padding,
channels 3 -> 64 -> 64 -> 64 -> 64 -> 64 -> 3 (the 3-channel ends are stored
padded to 32), ReLU after the first five, and a residual head (prediction =
input + output).  Weights are FP32 masters packed to BF16 after every
update; activations are BF16; every product accumulates in FP32 on the
matrix cores.  Training data come from the library's own batched solver.
The decoded prediction is projected so that the totals of rho and phi equal
the input's, and the plain solver continues from it with zero velocity.

Everything here is marshalling: encode, convolutions, loss, gradients, Adam
and decode run in the library's kernels; torch only owns device memory.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import TelbmError

_vp, _i, _i64, _sz, _f, _d = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float,
                              ctypes.c_double)
PROTOTYPES = {
    "telbm_conv_pack_weights": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "telbm_conv_forward": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _i, _i, _i, _vp, _vp, _vp]),
    "telbm_conv_backward": (_i, [_vp, _vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "telbm_conv_workspace_bytes": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(_sz)]),
    "telbm_residual_mse": (_i, [_vp, _vp, _vp, _i64, _i, _i, _vp, _vp, _vp, ctypes.POINTER(_i), _vp]),
    "telbm_adam_step": (_i, [_vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i64, _vp]),
    "telbm_surrogate_encode": (_i, [_vp, _vp, _vp, _vp, _i64, _d, _d, _d, _d, _vp, _vp]),
    "telbm_surrogate_decode": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _vp, _vp, _vp, _vp, _vp,
                                    _sz, _vp]),
    "telbm_surrogate_decode_workspace_bytes": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "telbm_surrogate_decode_noalloc": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _d, _d, _d, _d, _vp, _vp, _vp, _vp,
                                            _vp]),
    "telbm_surrogate_decode_noalloc_max_bytes": (_sz, []),
}

CH = 32          # stored channels at the network's ends
VALID = 5        # encoded channels: scaled density, C1, C2, scaled ux, uy
U_SCALE = 10.0   # velocity scale of the encoding (lattice velocities are O(1e-2))
LAYERS = [(32, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 32)]
# dilations of the six 3x3 layers: a receptive field of +-18 nodes, about
# the distance an interface moves over the 2000-step horizon
DILATIONS = (1, 2, 4, 8, 2, 1)


def _load():
    L = _lib.load()
    if not getattr(L, "_surrogate_protos", False):
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        L._surrogate_protos = True
    return L


def _ck(rc, what):
    if rc:
        raise TelbmError(rc, what)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def flops_per_pixel(padded: bool = False) -> int:
    """Multiply-add flops of one forward pass per pixel (x2 per MAC)."""
    tot = 0
    for k, (ci, co) in enumerate(LAYERS):
        if not padded:
            ci = VALID if k == 0 else ci
            co = VALID if k == len(LAYERS) - 1 else co
        tot += 2 * 9 * ci * co
    return tot


# --------------------------------------------------------------------------
# Layer-level calls (device tensors in, device tensors out)
# --------------------------------------------------------------------------
def pack_weights(w, cin, cout, wf, wd, stream):
    _ck(_load().telbm_conv_pack_weights(_p(w), cin, cout, _p(wf), _p(wd), _vp(stream.cuda_stream)), "pack")


def conv_forward(x, n, h, w, cin, wf, bias, cout, relu, y_bf16=None, y_f32=None, stream=None, dil=1):
    _ck(_load().telbm_conv_forward(_p(x), n, h, w, cin, _p(wf), _p(bias), cout, dil, int(relu), _p(y_bf16),
                                   _p(y_f32), _vp(stream.cuda_stream)), "conv forward")


def conv_workspace_bytes(n, h, w, cin, cout) -> int:
    b = ctypes.c_size_t()
    _ck(_load().telbm_conv_workspace_bytes(n, h, w, cin, cout, ctypes.byref(b)), "workspace size")
    return b.value


def conv_backward(x, dy, n, h, w, cin, cout, wd, mask, dx, dw, db, ws, stream, dil=1):
    _ck(_load().telbm_conv_backward(_p(x), _p(dy), n, h, w, cin, cout, dil, _p(wd), _p(mask), _p(dx), _p(dw),
                                    _p(db), _p(ws), ws.numel() if ws is not None else 0, _vp(stream.cuda_stream)),
        "conv backward")


def residual_mse(x, y, target, pixels, dy=None, pred=None, partials=None, stream=None) -> int:
    nb = ctypes.c_int()
    _ck(_load().telbm_residual_mse(_p(x), _p(y), _p(target), pixels, CH, VALID, _p(dy), _p(pred), _p(partials),
                                   ctypes.byref(nb), _vp(stream.cuda_stream)), "residual mse")
    return nb.value


def adam_step(w, g, m, v, lr, t, stream, beta1=0.9, beta2=0.999, eps=1e-8):
    _ck(_load().telbm_adam_step(_p(w), _p(g), _p(m), _p(v), w.numel(), lr, beta1, beta2, eps, t,
                                _vp(stream.cuda_stream)), "adam")


def encode(rho, phi, ux, uy, rho_g, rho_l, chi, out, stream, u_scale=U_SCALE):
    """rho, phi (and ux, uy, or None for a state at rest): float64 device
    tensors of one size; out: int16 device tensor of size*32 BF16 values."""
    _ck(_load().telbm_surrogate_encode(_p(rho), _p(phi), _p(ux), _p(uy), rho.numel(), rho_g, rho_l, chi, u_scale,
                                       _p(out), _vp(stream.cuda_stream)), "encode")


def decode(y, rho_in, phi_in, ux_in, uy_in, n, h, w, rho_g, rho_l, chi, rho_out, phi_out, ux_out, uy_out, stream,
           u_scale=U_SCALE):
    """Returns the workspace tensor, which must stay alive until the stream
    has run the decode."""
    import torch
    L = _load()
    b = ctypes.c_size_t()
    _ck(L.telbm_surrogate_decode_workspace_bytes(n, h, w, ctypes.byref(b)), "decode workspace")
    ws = torch.empty(b.value, dtype=torch.uint8, device=y.device)
    _ck(L.telbm_surrogate_decode(_p(y), _p(rho_in), _p(phi_in), _p(ux_in), _p(uy_in), n, h, w, rho_g, rho_l, chi,
                                 u_scale, _p(rho_out), _p(phi_out), _p(ux_out), _p(uy_out), _p(ws), ws.numel(),
                                 _vp(stream.cuda_stream)), "decode")
    return ws


# --------------------------------------------------------------------------
# The network
# --------------------------------------------------------------------------
class Network:
    """Six-layer 3x3 convolutional surrogate with Adam on FP32 masters."""

    def __init__(self, seed: int = 0, device: str = "cuda", stream=None, out_scale: float = 0.1,
                 dilations: Sequence[int] = DILATIONS):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate needs a GPU: no HIP device is visible")
        _load()
        self.device = torch.device(device)
        self.dilations = tuple(int(d) for d in dilations)
        assert len(self.dilations) == len(LAYERS) and min(self.dilations) >= 1
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = torch.Generator().manual_seed(seed)
        self.w, self.b, self.wf, self.wd = [], [], [], []
        self.mw, self.vw, self.mb, self.vb = [], [], [], []
        last = len(LAYERS) - 1
        for k, (ci, co) in enumerate(LAYERS):
            ci_v = VALID if k == 0 else ci
            co_v = VALID if k == last else co
            std = math.sqrt(2.0 / (9 * ci_v)) * (out_scale if k == last else 1.0)
            w = torch.zeros(9, ci, co)
            w[:, :ci_v, :co_v] = torch.randn(9, ci_v, co_v, generator=g) * std
            self.w.append(w.to(self.device).contiguous())
            self.b.append(torch.zeros(co, device=self.device))
            self.wf.append(torch.empty(9 * ci * co, dtype=torch.int16, device=self.device))
            self.wd.append(torch.empty(9 * ci * co, dtype=torch.int16, device=self.device))
            for lst in (self.mw, self.vw):
                lst.append(torch.zeros_like(self.w[-1]))
            for lst in (self.mb, self.vb):
                lst.append(torch.zeros_like(self.b[-1]))
        self.t = 0
        self._shape = None
        self.pack()

    # -- parameters -----------------------------------------------------------
    def pack(self):
        for k, (ci, co) in enumerate(LAYERS):
            pack_weights(self.w[k], ci, co, self.wf[k], self.wd[k], self.stream)

    def state_dict(self) -> dict:
        d = {"t": np.array(self.t), "dilations": np.array(self.dilations)}
        for k in range(len(LAYERS)):
            d[f"w{k}"] = self.w[k].cpu().numpy()
            d[f"b{k}"] = self.b[k].cpu().numpy()
        return d

    def load_state_dict(self, d: dict):
        import torch
        for k in range(len(LAYERS)):
            self.w[k].copy_(torch.as_tensor(d[f"w{k}"]))
            self.b[k].copy_(torch.as_tensor(d[f"b{k}"]))
        self.t = int(d["t"])
        if "dilations" in d:
            self.dilations = tuple(int(v) for v in d["dilations"])
        self.pack()

    # -- buffers ----------------------------------------------------------------
    def _buffers(self, n, h, w):
        import torch
        if self._shape == (n, h, w):
            return
        P = n * h * w
        dev = self.device
        # a[k] is the input of layer k (a[0] is the caller's x)
        self.a = [None] + [torch.empty(P * co, dtype=torch.int16, device=dev) for (_, co) in LAYERS[:-1]]
        self.y = torch.empty(P * CH, dtype=torch.float32, device=dev)
        self.dy = [torch.empty(P * co, dtype=torch.int16, device=dev) for (_, co) in LAYERS]
        self.gw = [torch.empty_like(x) for x in self.w]
        self.gb = [torch.empty_like(x) for x in self.b]
        ws = max(conv_workspace_bytes(n, h, w, ci, co) for ci, co in LAYERS)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.loss_part = torch.empty((P * CH + 255) // 256, dtype=torch.float32, device=dev)
        self._shape = (n, h, w)

    # -- passes ---------------------------------------------------------------
    def forward(self, x, n, h, w):
        """x: int16 device tensor holding BF16 NHWC (n, h, w, 32).  Returns the
        FP32 output y (n*h*w*32) of the last layer (before the residual)."""
        self._buffers(n, h, w)
        inp = x
        last = len(LAYERS) - 1
        for k, (ci, co) in enumerate(LAYERS):
            d = self.dilations[k]
            if k < last:
                conv_forward(inp, n, h, w, ci, self.wf[k], self.b[k], co, 1, y_bf16=self.a[k + 1],
                             stream=self.stream, dil=d)
                inp = self.a[k + 1]
            else:
                conv_forward(inp, n, h, w, ci, self.wf[k], self.b[k], co, 0, y_f32=self.y, stream=self.stream,
                             dil=d)
        return self.y

    def loss_and_grad(self, x, target, n, h, w):
        """Forward, residual MSE against target, backward into gw/gb.
        Returns the device tensor of loss partials (sum of squared errors)."""
        self.forward(x, n, h, w)
        P = n * h * w
        nb = residual_mse(x, self.y, target, P, dy=self.dy[-1], partials=self.loss_part, stream=self.stream)
        for k in range(len(LAYERS) - 1, -1, -1):
            ci, co = LAYERS[k]
            inp = x if k == 0 else self.a[k]
            dx = None if k == 0 else self.dy[k - 1]
            mask = None if k == 0 else self.a[k]
            conv_backward(inp, self.dy[k], n, h, w, ci, co, self.wd[k], mask, dx, self.gw[k], self.gb[k], self.ws,
                          self.stream, dil=self.dilations[k])
        return self.loss_part[:nb]

    def adam(self, lr: float):
        self.t += 1
        for k in range(len(LAYERS)):
            adam_step(self.w[k], self.gw[k], self.mw[k], self.vw[k], lr, self.t, self.stream)
            adam_step(self.b[k], self.gb[k], self.mb[k], self.vb[k], lr, self.t, self.stream)
        self.pack()

    def train_step(self, x, target, n, h, w, lr: float):
        part = self.loss_and_grad(x, target, n, h, w)
        self.adam(lr)
        return part

    def predict(self, x, n, h, w, pred=None):
        """FP32 prediction (input + output) for the first three channels."""
        import torch
        y = self.forward(x, n, h, w)
        if pred is None:
            pred = torch.empty(n * h * w * CH, dtype=torch.float32, device=self.device)
        residual_mse(x, y, None, n * h * w, pred=pred, stream=self.stream)
        return pred


def mse_value(partials, pixels: int) -> float:
    """Mean squared error per valid channel from the loss partials."""
    return float(np.sum(partials.cpu().numpy().astype(np.float64))) / (pixels * VALID)


# --------------------------------------------------------------------------
# Data: two-drop relaxations generated by the batched solver
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Family:
    """Physics of one trained model (the network cannot see tensions, so a
    model is trained per parameter set)."""
    name: str = "lens"
    n: int = 256
    ratio: float = 10.0
    kappa2: float = 0.045
    kappa3: float = 0.045
    r_lo: float = 20.0
    r_hi: float = 50.0
    horizon: int = 2000
    jumps: int = 3          # chained pairs per trajectory: (kH, (k+1)H), k < jumps


FAMILIES = {
    "lens": Family("lens", kappa2=0.045, kappa3=0.045),
    # liquid 1 of low gas tension spreads over liquid 2
    "spreading": Family("spreading", kappa2=0.005, kappa3=0.09),
}


def drops_for_seed(fam: Family, seed: int):
    """Two touching drops of seeded radii U[r_lo, r_hi], seeded centre and axis."""
    from synth.rng import uniform
    r = uniform(seed * 7919 + 101, 5)
    R1 = fam.r_lo + (fam.r_hi - fam.r_lo) * r[0]
    R2 = fam.r_lo + (fam.r_hi - fam.r_lo) * r[1]
    R1, R2 = min(R1, 0.24 * fam.n), min(R2, 0.24 * fam.n)
    ang = 2.0 * math.pi * r[2]
    cx, cy = fam.n * (0.4 + 0.2 * r[3]), fam.n * (0.4 + 0.2 * r[4])
    d = R1 + R2
    # touching: centre distance R1 + R2, contact point near (cx, cy)
    c1 = (cx - R1 * math.cos(ang), cy - R1 * math.sin(ang))
    c2 = (cx + R2 * math.cos(ang), cy + R2 * math.sin(ang))
    assert abs(math.hypot(c2[0] - c1[0], c2[1] - c1[1]) - d) < 1e-9
    return [{"center": c1, "radius": R1, "liquid": 1}, {"center": c2, "radius": R2, "liquid": 2}]


@dataclasses.dataclass
class Physics:
    """Thermodynamic state of a family: the EOS temperature and the Maxwell
    densities that parametrise the free energy (the solver's rho_g, rho_l),
    and the lattice model's own coexisting densities, measured on a flat
    slab, that start the drops and scale the network's density channel.
    (Starting at the Maxwell densities sets off a slow global drift of the
    bulk densities that would mask the shape relaxation.)"""
    T: float
    rho_g: float
    rho_l: float
    ic_g: float
    ic_l: float
    chi: float = 5.0


def physics(fam: Family, calibrate_steps: int = 20000) -> Physics:
    from .calibrate import discrete_coexistence
    from .solver import coexistence, temperature_for_ratio
    T = temperature_for_ratio(fam.ratio)
    rg, rl, _, _ = coexistence(T)
    p = family_params(fam, Physics(T, rg, rl, rg, rl))
    ig, il = discrete_coexistence(p, steps=calibrate_steps)
    return Physics(T, rg, rl, ig, il)


def family_params(fam: Family, ph: Physics, precision: int = 0):
    from .solver import Params
    return Params(lattice=0, precision=precision, nx=fam.n, ny=fam.n, nz=1, T=ph.T, rho_g=ph.rho_g,
                  rho_l=ph.rho_l, chi=ph.chi, kappa2=fam.kappa2, kappa3=fam.kappa3, lambda2=3.125 * fam.kappa2,
                  lambda3=3.125 * fam.kappa3)


def initial_fields(fam: Family, seed: int, ph: Physics):
    from synth.fields import two_drop_fields
    rho, phi, _ = two_drop_fields((1, fam.n, fam.n), drops_for_seed(fam, seed), ph.ic_g, ph.ic_l, ph.chi, seed)
    return rho[0], phi[0]


class Dataset:
    """Encoded pairs (state at 0, state at horizon) on the device, BF16."""

    def __init__(self, X, Y, n):
        self.X, self.Y, self.n = X, Y, n

    def __len__(self):
        return self.X.shape[0]

    def slice(self, i, j):
        return self.X[i:j], self.Y[i:j]


def generate(fam: Family, seeds: Sequence[int], ph: Physics, precision: int = 0, chunk: int = 64, stream=None,
             order_seed: int = 0) -> Dataset:
    """Run each seed's configuration (from rest) for fam.jumps * fam.horizon
    steps with the batched solver, snapshotting every fam.horizon steps, and
    encode the consecutive pairs.  Pairs are stored in a seeded order so
    that contiguous minibatches mix trajectories and times."""
    import torch
    from .batch import Batch
    stream = stream if stream is not None else torch.cuda.current_stream()
    n, J = fam.n, fam.jumps
    S = len(seeds)
    X = torch.empty((S * J, n * n * CH), dtype=torch.int16, device="cuda")
    Y = torch.empty((S * J, n * n * CH), dtype=torch.int16, device="cuda")
    slot = np.random.default_rng(order_seed).permutation(S * J)
    names = ("rho", "phi", "ux", "uy")
    for c0 in range(0, S, chunk):
        part = list(seeds[c0:c0 + chunk])
        m = len(part)
        params = [family_params(fam, ph, precision) for _ in part]
        with Batch(params, stream=stream) as B:
            prev = torch.zeros((4, m, n, n), dtype=torch.float64, device="cuda")
            for k, s in enumerate(part):
                r, f = initial_fields(fam, s, ph)
                B.init_fields(k, r, f)
                prev[0, k].copy_(torch.from_numpy(r))
                prev[1, k].copy_(torch.from_numpy(f))
            xe = torch.empty((m, n * n * CH), dtype=torch.int16, device="cuda")
            ye = torch.empty_like(xe)
            for j in range(J):
                B.step(fam.horizon)
                cur = torch.empty_like(prev)
                for k in range(m):
                    for c, name in enumerate(names):
                        B.read_device(k, name, cur[c, k])
                if j == 0:
                    encode(prev[0], prev[1], None, None, ph.ic_g, ph.ic_l, ph.chi, xe, stream)
                else:
                    encode(prev[0], prev[1], prev[2], prev[3], ph.ic_g, ph.ic_l, ph.chi, xe, stream)
                encode(cur[0], cur[1], cur[2], cur[3], ph.ic_g, ph.ic_l, ph.chi, ye, stream)
                idx = torch.as_tensor(slot[[(c0 + k) * J + j for k in range(m)]], device="cuda")
                X.index_copy_(0, idx, xe)
                Y.index_copy_(0, idx, ye)
                prev = cur
            torch.cuda.synchronize()
    return Dataset(X, Y, n)


def train(net: Network, data: Dataset, iters: int, batch: int = 8, lr: float = 1e-3, lr_final: float = 1e-4,
          seed: int = 0, log_every: int = 0, log=None) -> List[float]:
    """Adam over contiguous minibatches in a seeded order, cosine learning
    rate from lr to lr_final.  Returns the loss history (per log point)."""
    n = data.n
    nb = max(1, len(data) // batch)
    rng = np.random.default_rng(seed)
    order = rng.permutation(nb)
    hist = []
    for it in range(iters):
        if it and it % nb == 0:
            order = rng.permutation(nb)
        i = int(order[it % nb]) * batch
        x, y = data.slice(i, min(i + batch, len(data)))
        cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(1, iters)))
        part = net.train_step(x, y, x.shape[0], n, n, cur)
        if log_every and (it % log_every == 0 or it == iters - 1):
            v = mse_value(part, x.shape[0] * n * n)
            hist.append(v)
            if log:
                log(f"iter {it} lr {cur:.2e} mse {v:.3e}")
    return hist


def evaluate(net: Network, data: Dataset, batch: int = 8, per_channel: bool = False):
    """(surrogate MSE, identity MSE): prediction vs target, and the untouched
    input vs target, averaged over the valid channels.  With per_channel,
    also the two per-channel MSE vectors (read back to the host)."""
    import torch
    n = data.n
    se_p = np.zeros(VALID)
    se_0 = np.zeros(VALID)
    npx = 0
    pred = torch.empty(batch * n * n * CH, dtype=torch.float32, device="cuda")
    for i in range(0, len(data), batch):
        x, y = data.slice(i, min(i + batch, len(data)))
        m = x.shape[0]
        P = m * n * n
        net.predict(x, m, n, n, pred=pred[:P * CH])
        p = pred[:P * CH].view(P, CH)[:, :VALID].double()
        t = _bf16_to_f64(y).view(P, CH)[:, :VALID]
        s = _bf16_to_f64(x).view(P, CH)[:, :VALID]
        se_p += ((p - t) ** 2).sum(0).cpu().numpy()
        se_0 += ((s - t) ** 2).sum(0).cpu().numpy()
        npx += P
    mp, m0 = se_p / npx, se_0 / npx
    if per_channel:
        return float(mp.mean()), float(m0.mean()), mp, m0
    return float(mp.mean()), float(m0.mean())


def _bf16_to_f64(t):
    import torch
    return (t.to(torch.int32).bitwise_and(0xFFFF).bitwise_left_shift(16)).view(torch.float32).double()


def jump(net: Network, rho, phi, ph: Physics, ux=None, uy=None):
    """Surrogate state from a start state (float64 device tensors (h, w) or
    (n, h, w); no velocity means at rest): encode, forward, decode with the
    conservation projection.  Returns (rho, phi, ux, uy)."""
    import torch
    if rho.dim() == 2:
        rho, phi = rho[None], phi[None]
        ux = ux[None] if ux is not None else None
        uy = uy[None] if uy is not None else None
    m, h, w = rho.shape
    rho, phi = rho.contiguous(), phi.contiguous()
    ux = ux.contiguous() if ux is not None else None
    uy = uy.contiguous() if uy is not None else None
    x = torch.empty(m * h * w * CH, dtype=torch.int16, device=rho.device)
    encode(rho, phi, ux, uy, ph.ic_g, ph.ic_l, ph.chi, x, net.stream)
    y = net.forward(x, m, h, w)
    out = torch.empty((4, m, h, w), dtype=torch.float64, device=rho.device)
    # the workspace stays referenced until the next jump: the decode kernels
    # run asynchronously on the network's stream
    net._decode_ws = decode(y, rho, phi, ux, uy, m, h, w, ph.ic_g, ph.ic_l, ph.chi, out[0], out[1], out[2],
                            out[3], net.stream)
    net._decode_in = x
    return out[0], out[1], out[2], out[3]


def check_state(rho, phi, rho_in, phi_in, rho_g: float, chi: float, rtol: float = 1e-9) -> dict:
    """Admission checks of a surrogate state before the solver takes it:
    finite, positive density, |phi| <= chi, totals equal to the input's."""
    import torch
    m_in, m = float(rho_in.sum()), float(rho.sum())
    f_in, f = float(phi_in.sum()), float(phi.sum())
    res = {
        "finite": bool(torch.isfinite(rho).all() and torch.isfinite(phi).all()),
        "rho_positive": bool((rho > 0.25 * rho_g).all()),
        "phi_bounded": bool((phi.abs() <= 1.25 * chi).all()),
        "mass_rel_err": abs(m - m_in) / abs(m_in),
        "phi_abs_err": abs(f - f_in) / max(1.0, float(phi_in.abs().sum())),
    }
    res["ok"] = (res["finite"] and res["rho_positive"] and res["phi_bounded"] and res["mass_rel_err"] < rtol
                 and res["phi_abs_err"] < rtol)
    return res


def lead(d_plain: np.ndarray, d_surr: np.ndarray, window: int, horizon: int) -> float:
    """How far ahead of the plain run the surrogate-started run is, in LBM
    steps, averaged over its first 2 horizon / window windows: for each of
    its states, the first time at which the plain run's running-minimum
    distance to equilibrium has come down to the same value, minus the
    surrogate run's own LBM steps.  A perfect jump leads by `horizon`."""
    env = np.minimum.accumulate(d_plain)
    t_plain = np.arange(len(env)) * window
    out = []
    for j in range(1, min(len(d_surr), 2 * horizon // window + 1)):
        k = np.nonzero(env <= d_surr[j])[0]
        t_eff = t_plain[k[0]] if k.size else t_plain[-1]
        out.append(t_eff - j * window)
    return float(np.mean(out)) if out else 0.0


def compare_to_plain(net: Network, fam: Family, seed: int, ph: Physics, ref_steps: int, window: int = 500,
                     tol: float = 1e-2, jumps: int = 1, between: int = 200, log=None) -> dict:
    """Steps to equilibrium for one configuration, judged by the plain solver.

    The plain solver runs ref_steps from t = 0; the mean interface measures
    of its last four windows are the equilibrium reference.  The surrogate
    run starts from `jumps` chained jumps (standing for jumps * fam.horizon
    steps), with `between` LBM steps after each jump but the last (they
    return the state to the solver's manifold before the next jump), and
    runs ref_steps - jumps * fam.horizon LBM steps in all.  Each run's
    count is the first step from which its measures stay within tol of the
    reference (equilibrium.settle_step).  If the jumped state fails its
    admission checks, or the continued run turns unstable, the plain run is
    the result (fallback).  Also returns the final bulk densities and
    totals of both runs."""
    import torch
    from ._lib import TelbmError
    from .equilibrium import distance, settle_step, trajectory
    from .solver import Solver
    p = family_params(fam, ph)
    r, f = initial_fields(fam, seed, ph)
    rho_g, rho_l, chi = ph.ic_g, ph.ic_l, ph.chi
    out = {"seed": seed, "horizon": fam.horizon, "jumps": jumps}

    def finals(s):
        rho = s.read("rho")
        sc = (rho - rho_g) / (rho_l - rho_g)
        return {"mass": float(rho.sum()), "phi_total": float(s.read("phi").sum()),
                "rho_gas": float(np.median(rho[sc < 0.1])), "rho_liquid": float(np.median(rho[sc > 0.9]))}

    with Solver(p) as s:
        s.init_fields(r, f)
        tp = trajectory(s, ref_steps, window, rho_g, rho_l, chi)
        out["plain_final"] = finals(s)
    ref = tp[-4:].mean(axis=0)
    out["reference"] = ref
    out["plain_distance"] = distance(tp, ref)
    out["plain_steps"] = settle_step(tp, ref, tol, window)
    rt, ft = torch.from_numpy(r).cuda(), torch.from_numpy(f).cuda()
    out["fallback"] = False
    lbm = 0
    try:
        with Solver(p) as s:
            ro, po, ux, uy = jump(net, rt, ft, ph)
            for k in range(jumps):
                torch.cuda.synchronize()
                chk = check_state(ro, po, rt, ft, rho_g, chi)
                out["checks"] = chk
                if not chk["ok"]:
                    out["fallback"] = True
                    break
                u = torch.stack([ux[0], uy[0], torch.zeros_like(ux[0])])
                s.init_fields(ro[0], po[0], u)
                if k == jumps - 1:
                    break
                s.step(between)
                lbm += between
                cur = [s.read(name, device=True) for name in ("rho", "phi", "ux", "uy")]
                ro, po, ux, uy = jump(net, *[c.reshape(fam.n, fam.n) for c in cur[:2]], ph,
                                      *[c.reshape(fam.n, fam.n) for c in cur[2:]])
            if not out["fallback"]:
                ts = trajectory(s, ref_steps - jumps * fam.horizon - lbm, window, rho_g, rho_l, chi)
                out["surrogate_final"] = finals(s)
                out["surrogate_distance"] = distance(ts, ref)
                k = settle_step(ts, ref, tol, window)
                out["surrogate_steps"] = k + lbm if k >= 0 else -1
    except TelbmError:
        out["fallback"] = True
    if out["fallback"]:
        out["surrogate_steps"] = out["plain_steps"]
        out["surrogate_final"] = out["plain_final"]
    if "surrogate_distance" in out:
        out["lead_steps"] = lead(out["plain_distance"], out["surrogate_distance"], window, fam.horizon)
    ok = out["plain_steps"] >= 0 and out["surrogate_steps"] >= 0
    out["gain_steps"] = out["plain_steps"] - out["surrogate_steps"] if ok else None
    if log:
        log(f"seed {seed}: plain {out['plain_steps']} steps, {jumps} jump(s) + {out['surrogate_steps']} steps"
            f"{' (fallback)' if out['fallback'] else ''}")
    return out
