"""Learned surrogate of the coupled LB freezing step: a 3-level U-Net that maps
the fields of a 2D grid at two time levels, 64 LB steps apart, to the fields
64 steps ahead (the change of phi, f_l, T, C; the new value of u and p),
built from the BF16 MFMA kernels of ``liblbfz.so`` (``include/lbfz_nn.h``).
The binding marshals arguments only; PyTorch holds the device memory.

Network (NHWC, bf16 activations, FP32 master weights; 3x3 convolutions with
zero padding, ReLU after every convolution but the head):

    X0 (16 ch: phi, f_l, T, C, u_x, u_y, u_z = 0, p 64 steps ago, then now)
    L1a 16->32, L1b 32->32 = S1 ........................ CAT1[:, 32:64]
    maxpool -> L2a 32->64, L2b 64->64 = S2 .............. CAT2[:, 64:128]
    maxpool -> L3a 64->128, L3b 128->128
    upsample -> U2 128->64 ............................. CAT2[:, 0:64]
    L4a 128->64, L4b 64->64
    upsample -> U1 64->32 .............................. CAT1[:, 0:32]
    L5a 64->32, L5b 32->32, head 1x1 32->8 (the eight fields), FP32 output

The skip concatenations are channel slices of CAT1 / CAT2 written in place by
the layers that produce them.  The pressure and the earlier time level are
what make the velocity predictable: in the weakly compressible flow, u and p
together fix the acoustic part of the flow, and the two levels its phase.
Screening: the prediction of a grid is accepted when its phase-field mass
residual -- how far the change of sum phi over the stride is from the
scheme's own budget, sum phi div u per step (Sec. 3.1), integrated by the
trapezoid rule between the two ends -- is at most 1e-3 of the grid's liquid
volume and its solute sum is within 1e-3 of the one before the stride (the
solute budget of Sec. 3.4 is exact), else the grid is advanced by the LB
step instead.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import lbfz

NEXP = 8         # fields of one time level: phi, f_l, T, C, u_x, u_y, u_z (0 in 2D), p
NF = NEXP        # predicted fields: the same eight, 64 steps ahead
NLEV = 2         # input time levels: 64 steps ago and now
NIN = NLEV * NEXP  # input planes
CIN0 = 16        # input channels
HEAD = 8         # head channels
FIELD_NAMES = ("phi", "fl", "T", "C", "ux", "uy", "uz", "p")
# the fields the screening restarts an accepted grid from (RESTART_FIELDS of
# the batch: phi, f_l, T, C, u_x, u_y, p), as indices into FIELD_NAMES
RESTART_IDX = (0, 1, 2, 3, 4, 5, 7)
LBFZ_NN_EINVAL = -1  # codes of the lbfz_nn_* calls (include/lbfz_nn.h)
LBFZ_NN_EHIP = -3


class lbfz_conv_args(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("in_cs", ctypes.c_int32), ("in_co", ctypes.c_int32),
                ("Cin", ctypes.c_int32), ("w", ctypes.c_void_p), ("dz_cs", ctypes.c_int32),
                ("N", ctypes.c_int32), ("bias", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("out_cs", ctypes.c_int32), ("out_co", ctypes.c_int32),
                ("out_f32", ctypes.c_int32), ("relu", ctypes.c_int32), ("sign", ctypes.c_int32),
                ("B", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("taps", ctypes.c_int32), ("up", ctypes.c_int32), ("pool", ctypes.c_void_p),
                ("pool_cs", ctypes.c_int32), ("pool_co", ctypes.c_int32)]


class lbfz_tail_args(ctypes.Structure):
    _fields_ = [("head_w", ctypes.c_void_p), ("head_b", ctypes.c_void_p), ("nh", ctypes.c_int32),
                ("nf", ctypes.c_int32), ("before", ctypes.c_void_p),
                ("before_stride", ctypes.c_int64), ("shift", ctypes.c_void_p),
                ("scale", ctypes.c_void_p), ("resid", ctypes.c_void_p), ("pred", ctypes.c_void_p),
                ("pred_stride", ctypes.c_int64)]


_nn = None


def nnlib():
    global _nn
    if _nn is None:
        L = lbfz.lib()
        vp, i32, lg = ctypes.c_void_p, ctypes.c_int32, ctypes.c_long
        f32, u32 = ctypes.c_float, ctypes.c_uint32
        cp = ctypes.POINTER(lbfz_conv_args)
        sig = {
            "lbfz_nn_conv": [cp, vp],
            "lbfz_nn_conv_tail": [cp, ctypes.POINTER(lbfz_tail_args), vp],
            "lbfz_nn_conv_wgrad": [cp, vp, i32, vp, vp],
            "lbfz_nn_bias_grad": [vp, lg, i32, i32, vp, i32, vp, vp],
            "lbfz_nn_relu_bwd": [vp, i32, i32, vp, i32, i32, vp, i32, lg, i32, vp],
            "lbfz_nn_maxpool2": [vp, i32, i32, vp, i32, i32, i32, i32, i32, vp],
            "lbfz_nn_maxpool2_bwd": [vp, i32, i32, vp, i32, vp, i32, i32, i32, i32, i32, i32, i32,
                                     vp],
            "lbfz_nn_upsample2": [vp, i32, i32, i32, i32, vp, vp],
            "lbfz_nn_upsample2_bwd": [vp, i32, i32, i32, i32, vp, vp],
            "lbfz_nn_fill_u32": [vp, lg, u32, vp],
            "lbfz_nn_mse": [vp, i32, vp, lg, i32, vp, vp, vp, i32, vp, vp],
            "lbfz_nn_plane_sums": [vp, i32, lg, lg, vp, vp],
            "lbfz_nn_phi_div_sums": [vp, i32, lg, i32, i32, i32, i32, i32, i32, vp, i32, vp,
                                     vp],
            "lbfz_nn_scale_planes": [vp, i32, lg, i32, lg, vp, i32, vp],
            "lbfz_nn_pack_images": [vp, i32, lg, i32, i32, vp, vp, vp, i32, vp],
            "lbfz_nn_apply_images": [vp, i32, vp, i32, lg, i32, i32, vp, vp, vp, vp, lg, vp],
            "lbfz_nn_adam": [vp, vp, vp, vp, vp, lg, f32, f32, f32, f32, i32, vp],
            "lbfz_nn_to_bf16": [vp, vp, lg, vp],
            "lbfz_nn_transpose_w": [vp, i32, i32, i32, vp, vp],
            "lbfz_nn_pack_fields": [vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, i32, i32, vp],
            "lbfz_nn_pack_delta": [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, i32,
                                   vp],
            "lbfz_nn_apply_delta": [vp, i32, vp, i32, i32, i32, vp, vp, vp, vp, i32, vp],
        }
        for nm, args in sig.items():
            fn = getattr(L, nm)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _nn = L
    return _nn


def _ck(rc, where):
    if rc != 0:
        raise RuntimeError(f"{where} failed (code {rc})")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def conv_args(x, x_cs, x_co, cin, w, n, out, out_cs, out_co, B, H, W, taps, bias=None,
              relu=False, sign=1, out_f32=False, dz_cs=0, up=False, pool=None, pool_cs=0):
    a = lbfz_conv_args()
    a.in_ = x.data_ptr()
    a.in_cs, a.in_co, a.Cin = x_cs, x_co, cin
    a.w = w.data_ptr()
    a.dz_cs = dz_cs
    a.N = n
    a.bias = bias.data_ptr() if bias is not None else None
    a.out = out.data_ptr() if out is not None else None
    a.out_cs, a.out_co, a.out_f32 = out_cs, out_co, int(out_f32)
    a.relu, a.sign = int(relu), sign
    a.B, a.H, a.W, a.taps = B, H, W, taps
    a.up = int(up)
    if pool is not None:
        a.pool, a.pool_cs, a.pool_co = pool.data_ptr(), pool_cs, 0
    return a


@dataclass
class Layer:
    name: str
    cin: int
    cout: int
    taps: int
    relu: bool
    level: int        # 0: full size, 1: /2, 2: /4


LAYERS = (
    Layer("L1a", CIN0, 32, 9, True, 0), Layer("L1b", 32, 32, 9, True, 0),
    Layer("L2a", 32, 64, 9, True, 1), Layer("L2b", 64, 64, 9, True, 1),
    Layer("L3a", 64, 128, 9, True, 2), Layer("L3b", 128, 128, 9, True, 2),
    Layer("U2", 128, 64, 9, True, 1), Layer("L4a", 128, 64, 9, True, 1),
    Layer("L4b", 64, 64, 9, True, 1), Layer("U1", 64, 32, 9, True, 0),
    Layer("L5a", 64, 32, 9, True, 0), Layer("L5b", 32, 32, 9, True, 0),
    Layer("head", 32, HEAD, 1, False, 0),
)


def init_weights(seed: int = 0) -> dict:
    """He-normal weights [cout][taps][cin] (zero for the padded input channels
    and head outputs), zero biases; FP32 numpy."""
    rng = np.random.default_rng(seed)
    out = {}
    for L in LAYERS:
        fan_in = L.taps * (NIN if L.name == "L1a" else L.cin)
        w = rng.standard_normal((L.cout, L.taps, L.cin)) * np.sqrt(2.0 / fan_in)
        if L.name == "L1a":
            w[:, :, NIN:] = 0.0
        if L.name == "head":
            w *= 0.1
            w[NF:] = 0.0
        out[L.name] = (w.astype(np.float32), np.zeros(L.cout, np.float32))
    return out


class UNet:
    """The network on one GPU for batches of B images of S x S pixels."""

    def __init__(self, weights: dict, B: int, S: int, device: int = 0, stream=None):
        import torch
        if S % 4:
            raise ValueError("image side must be a multiple of 4")
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.B, self.S = B, S
        self.L = {L.name: L for L in LAYERS}
        # parameters: one flat FP32 buffer (master), bf16 copy, grads, Adam moments
        self.offsets = {}
        n = 0
        for L in LAYERS:
            nw = L.cout * L.taps * L.cin
            self.offsets[L.name] = (n, nw, n + nw, L.cout)
            n += nw + L.cout
        self.nparam = n
        f = dict(dtype=torch.float32, device=self.dev)
        self.wf = torch.zeros(n, **f)
        host = np.zeros(n, np.float32)
        for L in LAYERS:
            o, nw, ob, nb = self.offsets[L.name]
            w, b = weights[L.name]
            host[o:o + nw] = w.reshape(-1)
            host[ob:ob + nb] = b
        self.wf.copy_(torch.from_numpy(host))
        self.gf = torch.zeros(n, **f)
        self.m = torch.zeros(n, **f)
        self.v = torch.zeros(n, **f)
        self.wb = torch.zeros(n, dtype=torch.bfloat16, device=self.dev)
        self.wt = {L.name: torch.zeros(L.cout * L.taps * L.cin, dtype=torch.bfloat16,
                                       device=self.dev) for L in LAYERS}
        self.adam_step = 0
        self._sync_bf16()
        # activations and gradients
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        s0, s1, s2 = S * S, (S // 2) ** 2, (S // 4) ** 2
        t = {}
        t["X0"] = torch.zeros(B * s0 * CIN0, **bf)
        t["A1"] = torch.zeros(B * s0 * 32, **bf)
        t["CAT1"] = torch.zeros(B * s0 * 64, **bf)
        t["P1"] = torch.zeros(B * s1 * 32, **bf)
        t["A2"] = torch.zeros(B * s1 * 64, **bf)
        t["CAT2"] = torch.zeros(B * s1 * 128, **bf)
        t["P2"] = torch.zeros(B * s2 * 64, **bf)
        t["A3"] = torch.zeros(B * s2 * 128, **bf)
        t["A3b"] = torch.zeros(B * s2 * 128, **bf)
        t["A4"] = torch.zeros(B * s1 * 64, **bf)
        t["A4b"] = torch.zeros(B * s1 * 64, **bf)
        t["A5"] = torch.zeros(B * s0 * 32, **bf)
        t["A5b"] = torch.zeros(B * s0 * 32, **bf)
        t["OUT"] = torch.zeros(B * s0 * HEAD, **f)
        # gradients (dX of each tensor) and pre-activation gradients (dz)
        for k in ("A1", "CAT1", "P1", "A2", "CAT2", "P2", "A3", "A3b", "A4", "A4b", "A5", "A5b"):
            t["d" + k] = torch.zeros_like(t[k])
        # gradients at the up-convolutions' (full) resolution
        t["dU2"] = torch.zeros(B * s1 * 128, **bf)
        t["dU1"] = torch.zeros(B * s0 * 64, **bf)
        t["dOUT"] = torch.zeros(B * s0 * HEAD, **bf)
        t["dz"] = torch.zeros(B * s0 * 128, **bf)   # largest dz (reused per layer)
        self.t = t
        self.nsplit = 64
        maxw = max(L.cout * L.taps * L.cin for L in LAYERS)
        self.part = torch.zeros(self.nsplit * maxw, **f)
        self.bpart = torch.zeros(256 * 256, **f)
        self.lpart = torch.zeros(1024, dtype=torch.float64, device=self.dev)
        self.loss_t = torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.target = torch.zeros(B * s0 * NF, **f)

    # ------------------------------------------------------------------ utils
    @property
    def st(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _sync_bf16(self):
        L = nnlib()
        _ck(L.lbfz_nn_to_bf16(_p(self.wf), _p(self.wb), self.nparam, self.st), "to_bf16")
        for Ly in LAYERS:
            o, nw, _, _ = self.offsets[Ly.name]
            _ck(L.lbfz_nn_transpose_w(ctypes.c_void_p(self.wb.data_ptr() + 2 * o), Ly.cout,
                                      Ly.taps, Ly.cin, _p(self.wt[Ly.name]), self.st),
                "transpose_w")

    def _w(self, name):
        o, nw, ob, nb = self.offsets[name]
        return (ctypes.c_void_p(self.wb.data_ptr() + 2 * o),
                ctypes.c_void_p(self.wf.data_ptr() + 4 * ob))

    def _dims(self, level):
        s = self.S >> level
        return self.B, s, s

    # ---------------------------------------------------------------- forward
    def _conv(self, name, x, x_cs, x_co, out, out_cs, out_co, out_f32=False, up=False,
              pool=None, pool_cs=0):
        Ly = self.L[name]
        B, H, W = self._dims(Ly.level)
        wb, bias = self._w(name)
        a = lbfz_conv_args()
        a.in_, a.in_cs, a.in_co, a.Cin = x.data_ptr(), x_cs, x_co, Ly.cin
        a.w, a.dz_cs, a.N = wb.value, 0, Ly.cout
        a.bias, a.out = bias.value, out.data_ptr()
        a.out_cs, a.out_co, a.out_f32 = out_cs, out_co, int(out_f32)
        a.relu, a.sign = int(Ly.relu), 1
        a.B, a.H, a.W, a.taps, a.up = B, H, W, Ly.taps, int(up)
        if pool is not None:
            a.pool, a.pool_cs, a.pool_co = pool.data_ptr(), pool_cs, 0
        _ck(nnlib().lbfz_nn_conv(ctypes.byref(a), self.st), "conv " + name)

    def forward(self):
        """X0 -> OUT (FP32, HEAD channels)."""
        t = self.t
        self._forward_body()
        self._conv("L5b", t["A5"], 32, 0, t["A5b"], 32, 0)
        self._conv("head", t["A5b"], 32, 0, t["OUT"], HEAD, 0, out_f32=True)

    def predict_fields(self, nimg, before, before_stride, pred, pred_stride, nf, shift, scale,
                       resid):
        """Inference: the prediction of the grids of images 0 .. nimg - 1 (as
        lbfz_nn_apply_images of forward()'s output), with the last convolution,
        the head and the prediction fused into one launch (lbfz_nn_conv_tail:
        neither A5b nor OUT is written)."""
        if not 0 < nimg <= self.B:
            raise ValueError("nimg out of range")
        t = self.t
        self._forward_body()
        Ly = self.L["L5b"]
        B, H, W = self._dims(Ly.level)
        wb, bias = self._w("L5b")
        a = lbfz_conv_args()
        a.in_, a.in_cs, a.in_co, a.Cin = t["A5"].data_ptr(), 32, 0, Ly.cin
        a.w, a.dz_cs, a.N = wb.value, 0, Ly.cout
        a.bias, a.out = bias.value, None
        a.out_cs, a.out_co, a.out_f32 = 32, 0, 0
        a.relu, a.sign = int(Ly.relu), 1
        a.B, a.H, a.W, a.taps, a.up = nimg, H, W, 9, 0
        hw, hb = self._w("head")
        ta = lbfz_tail_args()
        ta.head_w, ta.head_b, ta.nh, ta.nf = hw.value, hb.value, HEAD, nf
        ta.before, ta.before_stride = before.data_ptr(), before_stride
        ta.shift, ta.scale, ta.resid = shift.data_ptr(), scale.data_ptr(), resid.data_ptr()
        ta.pred, ta.pred_stride = pred.data_ptr(), pred_stride
        _ck(nnlib().lbfz_nn_conv_tail(ctypes.byref(a), ctypes.byref(ta), self.st), "conv_tail")

    def _forward_body(self):
        """X0 -> A5 (every layer before the last convolution)."""
        L, t = nnlib(), self.t
        B, S = self.B, self.S
        self._conv("L1a", t["X0"], CIN0, 0, t["A1"], 32, 0)
        # the encoder's second convolutions also write the pooled tensors
        self._conv("L1b", t["A1"], 32, 0, t["CAT1"], 64, 32, pool=t["P1"], pool_cs=32)
        self._conv("L2a", t["P1"], 32, 0, t["A2"], 64, 0)
        self._conv("L2b", t["A2"], 64, 0, t["CAT2"], 128, 64, pool=t["P2"], pool_cs=64)
        self._conv("L3a", t["P2"], 64, 0, t["A3"], 128, 0)
        self._conv("L3b", t["A3"], 128, 0, t["A3b"], 128, 0)
        # the up-convolutions read the half-resolution tensor through nearest 2x
        # upsampling inside the convolution's loads
        self._conv("U2", t["A3b"], 128, 0, t["CAT2"], 128, 0, up=True)
        self._conv("L4a", t["CAT2"], 128, 0, t["A4"], 64, 0)
        self._conv("L4b", t["A4"], 64, 0, t["A4b"], 64, 0)
        self._conv("U1", t["A4b"], 64, 0, t["CAT1"], 64, 0, up=True)
        self._conv("L5a", t["CAT1"], 64, 0, t["A5"], 32, 0)

    # --------------------------------------------------------------- backward
    def _layer_bwd(self, name, x, x_cs, x_co, dy, dy_cs, dy_co, y, y_cs, y_co, dx, dx_cs,
                   dx_co, need_dx=True, up=False):
        """Gradients of one convolution: dz = relu'(y) dy, dW, db into gf, and
        dx (overwritten, at the layer's resolution) when need_dx; up: x is the
        half-resolution tensor the layer reads through 2x upsampling."""
        L, t = nnlib(), self.t
        Ly = self.L[name]
        B, H, W = self._dims(Ly.level)
        P = B * H * W
        N = Ly.cout
        st = self.st
        if Ly.relu:
            dz = t["dz"]
            _ck(L.lbfz_nn_relu_bwd(_p(dy), dy_cs, dy_co, _p(y), y_cs, y_co, _p(dz), N, P, N, st),
                "relu_bwd " + name)
            dz_p, dz_cs = dz, N
        else:
            if dy_co != 0:
                raise ValueError("a head without activation reads its gradient at offset 0")
            dz_p, dz_cs = dy, dy_cs
        o, nw, ob, nb = self.offsets[name]
        a = lbfz_conv_args()
        a.in_, a.in_cs, a.in_co, a.Cin = x.data_ptr(), x_cs, x_co, Ly.cin
        a.w, a.dz_cs, a.N = dz_p.data_ptr(), dz_cs, N
        a.B, a.H, a.W, a.taps, a.sign, a.up = B, H, W, Ly.taps, 1, int(up)
        # partial rows: the 3 x 3 kernel takes what the buffer holds for this
        # layer (it uses about 512 blocks), the 1 x 1 one up to 1024 pixel splits
        rows = self.part.numel() // nw if Ly.taps == 9 else min(self.part.numel() // nw, 1024)
        _ck(L.lbfz_nn_conv_wgrad(ctypes.byref(a), _p(self.part), rows,
                                 ctypes.c_void_p(self.gf.data_ptr() + 4 * o), st),
            "wgrad " + name)
        _ck(L.lbfz_nn_bias_grad(_p(dz_p), P, dz_cs, N, _p(self.bpart), 256,
                                ctypes.c_void_p(self.gf.data_ptr() + 4 * ob), st),
            "bias_grad " + name)
        if need_dx:
            d = lbfz_conv_args()
            d.in_, d.in_cs, d.in_co, d.Cin = dz_p.data_ptr(), dz_cs, 0, N
            d.w, d.N = self.wt[name].data_ptr(), Ly.cin
            d.out, d.out_cs, d.out_co, d.out_f32 = dx.data_ptr(), dx_cs, dx_co, 0
            d.relu, d.sign = 0, -1
            d.B, d.H, d.W, d.taps = B, H, W, Ly.taps
            _ck(L.lbfz_nn_conv(ctypes.byref(d), st), "dgrad " + name)

    def backward(self):
        """Gradients of the loss (dOUT set by loss()) into gf."""
        L, t = nnlib(), self.t
        B, S = self.B, self.S
        st = self.st
        self._layer_bwd("head", t["A5b"], 32, 0, t["dOUT"], HEAD, 0, None, 0, 0, t["dA5b"], 32, 0)
        self._layer_bwd("L5b", t["A5"], 32, 0, t["dA5b"], 32, 0, t["A5b"], 32, 0, t["dA5"], 32, 0)
        self._layer_bwd("L5a", t["CAT1"], 64, 0, t["dA5"], 32, 0, t["A5"], 32, 0, t["dCAT1"], 64, 0)
        self._layer_bwd("U1", t["A4b"], 64, 0, t["dCAT1"], 64, 0, t["CAT1"], 64, 0, t["dU1"], 64, 0,
                        up=True)
        _ck(L.lbfz_nn_upsample2_bwd(_p(t["dU1"]), B, S // 2, S // 2, 64, _p(t["dA4b"]), st),
            "up1_bwd")
        self._layer_bwd("L4b", t["A4"], 64, 0, t["dA4b"], 64, 0, t["A4b"], 64, 0, t["dA4"], 64, 0)
        self._layer_bwd("L4a", t["CAT2"], 128, 0, t["dA4"], 64, 0, t["A4"], 64, 0, t["dCAT2"], 128,
                        0)
        self._layer_bwd("U2", t["A3b"], 128, 0, t["dCAT2"], 128, 0, t["CAT2"], 128, 0, t["dU2"],
                        128, 0, up=True)
        _ck(L.lbfz_nn_upsample2_bwd(_p(t["dU2"]), B, S // 4, S // 4, 128, _p(t["dA3b"]), st),
            "up2_bwd")
        self._layer_bwd("L3b", t["A3"], 128, 0, t["dA3b"], 128, 0, t["A3b"], 128, 0, t["dA3"],
                        128, 0)
        self._layer_bwd("L3a", t["P2"], 64, 0, t["dA3"], 128, 0, t["A3"], 128, 0, t["dP2"], 64, 0)
        _ck(L.lbfz_nn_maxpool2_bwd(_p(t["CAT2"]), 128, 64, _p(t["dP2"]), 64, _p(t["dCAT2"]), 128,
                                   64, 1, B, S // 2, S // 2, 64, st), "pool2_bwd")
        self._layer_bwd("L2b", t["A2"], 64, 0, t["dCAT2"], 128, 64, t["CAT2"], 128, 64, t["dA2"],
                        64, 0)
        self._layer_bwd("L2a", t["P1"], 32, 0, t["dA2"], 64, 0, t["A2"], 64, 0, t["dP1"], 32, 0)
        _ck(L.lbfz_nn_maxpool2_bwd(_p(t["CAT1"]), 64, 32, _p(t["dP1"]), 32, _p(t["dCAT1"]), 64,
                                   32, 1, B, S, S, 32, st), "pool1_bwd")
        self._layer_bwd("L1b", t["A1"], 32, 0, t["dCAT1"], 64, 32, t["CAT1"], 64, 32, t["dA1"], 32,
                        0)
        self._layer_bwd("L1a", t["X0"], CIN0, 0, t["dA1"], 32, 0, t["A1"], 32, 0, None, 0, 0,
                        need_dx=False)

    def loss(self, with_grad: bool = True, channel_weights=None) -> None:
        """MSE of OUT's first NF channels against target (FP32 [P][NF]), each
        channel weighted (device FP32 [NF], or None for 1); the value lands in
        loss_t (device), dOUT is set when with_grad."""
        P = self.B * self.S * self.S
        _ck(nnlib().lbfz_nn_mse(_p(self.t["OUT"]), HEAD, _p(self.target), P, NF,
                                _p(channel_weights), _p(self.t["dOUT"]) if with_grad else None,
                                _p(self.lpart), 1024, _p(self.loss_t), self.st), "mse")

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.adam_step += 1
        _ck(nnlib().lbfz_nn_adam(_p(self.wf), _p(self.gf), _p(self.m), _p(self.v), _p(self.wb),
                                 self.nparam, lr, b1, b2, eps, self.adam_step, self.st), "adam")
        for Ly in LAYERS:
            o, nw, _, _ = self.offsets[Ly.name]
            _ck(nnlib().lbfz_nn_transpose_w(ctypes.c_void_p(self.wb.data_ptr() + 2 * o), Ly.cout,
                                            Ly.taps, Ly.cin, _p(self.wt[Ly.name]), self.st),
                "transpose_w")

    def weights(self) -> dict:
        """Current FP32 weights as numpy, layout of init_weights."""
        host = self.wf.cpu().numpy()
        out = {}
        for Ly in LAYERS:
            o, nw, ob, nb = self.offsets[Ly.name]
            out[Ly.name] = (host[o:o + nw].reshape(Ly.cout, Ly.taps, Ly.cin).copy(),
                            host[ob:ob + nb].copy())
        return out

    def grads(self) -> dict:
        host = self.gf.cpu().numpy()
        out = {}
        for Ly in LAYERS:
            o, nw, ob, nb = self.offsets[Ly.name]
            out[Ly.name] = (host[o:o + nw].reshape(Ly.cout, Ly.taps, Ly.cin).copy(),
                            host[ob:ob + nb].copy())
        return out


# ---------------------------------------------------------------------------
# data, training and screening

STRIDE = 64      # LB steps spanned by one prediction
SOLUTE_PLANE = 3  # C: the network sees a grid's solute over its mean
PHI_DIV_PARTS = 16  # row sets per grid of the check's sum phi div u (blocks per grid)
MASS_TOL = 1e-3  # screening: largest accepted phase-field mass residual


def generate_snapshots(case_ids, side: int, nsnap: int, device: int = 0, storage: str = "f32"):
    """Run the LB step (batched, on the GPU) for the sweep grids case_ids with
    their side replaced by `side`, and keep the NEXP fields every STRIDE
    steps: a device tensor [ncases][nsnap][NEXP][side][side] FP32 (snapshot 0
    = the initial state), with the solute of every snapshot over its own mean
    (SOLUTE_PLANE: the network's scale for C; the LB conserves the solute, so
    the mean is the grid's constant).  Snapshots s - 1 and s of a grid are
    adjacent in memory: together they are the network input of time level s.
    Returns (snapshots, params of each grid)."""
    import torch
    from .workloads import sweep_case
    cases = [sweep_case(k, side=side) for k in case_ids]
    b = lbfz.Batch(cases, device=device, storage=storage)
    snaps = torch.zeros((len(cases), nsnap, NEXP, side, side), dtype=torch.float32,
                        device=b.device)
    for s in range(nsnap):
        if s:
            b.step(STRIDE)
        b.fields_all_to_device(NEXP, snaps[:, s], nsnap * NEXP * side * side)
    bad = sum(b.totals(i)["nonfinite"] for i in range(len(cases)))
    b.close()
    if bad:
        raise RuntimeError("non-finite LB state while generating snapshots")
    L, SS, nimg = nnlib(), side * side, len(cases) * nsnap
    sums = torch.zeros(nimg, dtype=torch.float64, device=snaps.device)
    st = ctypes.c_void_p(torch.cuda.current_stream(snaps.device).cuda_stream)
    _ck(L.lbfz_nn_plane_sums(_p(snaps[0, 0, SOLUTE_PLANE]), nimg, SS, NEXP * SS, _p(sums), st),
        "plane_sums")
    _ck(L.lbfz_nn_scale_planes(_p(snaps), nimg, NEXP * SS, SOLUTE_PLANE, SS, _p(sums), 0, st),
        "scale_planes")
    torch.cuda.synchronize()
    return snaps, [c[0] for c in cases]


# 1: the network learns the change of the field over STRIDE steps (phi, f_l,
# T, C evolve slowly); 0: its new value (u and p oscillate acoustically, and
# their change over a stride is as large as they are)
RESIDUAL = (1.0, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0)
# loss weight per field (u_z is identically zero in 2D)
LOSS_WEIGHT = (1.0, 1.0, 2.0, 1.0, 1.0, 1.0, 0.0, 1.0)


class Normaliser:
    """Per-field shift / scale of the network input (the fields, the same for
    both time levels) and of its target (the change over STRIDE steps, or the
    new value -- RESIDUAL), from a snapshot tensor [grids][snapshots][NEXP][S][S]."""

    def __init__(self, snaps):
        import torch
        x = snaps[:, :-1].transpose(0, 2).reshape(NEXP, -1)
        r = torch.tensor(RESIDUAL, dtype=snaps.dtype, device=snaps.device)
        d = (snaps[:, 1:, :NF] - r[None, None, :, None, None] * snaps[:, :-1, :NF])
        d = d.transpose(0, 2).reshape(NF, -1)
        self.in_shift = x.mean(dim=1).repeat(NLEV)
        self.in_scale = (1.0 / x.std(dim=1).clamp_min(1e-12)).repeat(NLEV)
        self.d_shift = d.mean(dim=1)
        self.d_scale = 1.0 / d.std(dim=1).clamp_min(1e-12)
        self.resid = r
        for k in ("in_shift", "in_scale", "d_shift", "d_scale", "resid"):
            setattr(self, k, getattr(self, k).to(torch.float32).contiguous())


def load_pairs(net: UNet, snaps, norm: Normaliser, pairs) -> None:
    """Images b = 0..len(pairs)-1 of the network input and target from the
    (grid, snapshot) pairs, s >= NLEV - 1: input = snapshots s - 1 and s (the
    two time levels, adjacent in memory), target = snapshot s + 1 against s."""
    L = nnlib()
    S = net.S
    for b, (i, s) in enumerate(pairs):
        before, after = snaps[i, s], snaps[i, s + 1]
        _ck(L.lbfz_nn_pack_fields(_p(snaps[i, s - NLEV + 1]), NIN, S, S, 0, 0, S, _p(norm.in_shift),
                                  _p(norm.in_scale), _p(net.t["X0"]), CIN0, b, net.st),
            "pack_fields")
        _ck(L.lbfz_nn_pack_delta(_p(after), _p(before), NF, S, S, 0, 0, S, _p(norm.d_shift),
                                 _p(norm.d_scale), _p(norm.resid), _p(net.target), b, net.st),
            "pack_delta")


def train(net: UNet, snaps, norm: Normaliser, iters: int, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0):
    """Adam on the MSE of the normalised change, random (grid, snapshot)
    pairs, cosine-decayed learning rate.  Returns the loss history."""
    import math
    import torch
    rng = np.random.default_rng(seed)
    ng, ns = snaps.shape[0], snaps.shape[1] - 1
    wch = torch.tensor(LOSS_WEIGHT, dtype=torch.float32, device=net.dev)
    hist = []
    for it in range(iters):
        pairs = [(int(rng.integers(ng)), int(rng.integers(NLEV - 1, ns)))
                 for _ in range(net.B)]
        load_pairs(net, snaps, norm, pairs)
        net.forward()
        net.loss(channel_weights=wch)
        net.backward()
        net.adam(lr * 0.5 * (1.0 + math.cos(math.pi * it / max(iters, 1))))
        if log_every and (it % log_every == 0 or it == iters - 1):
            hist.append((it, float(net.loss_t.cpu().numpy()[0])))
    return hist


def predict(net: UNet, snaps, norm: Normaliser, pairs, out):
    """Predicted fields after STRIDE steps for the (grid, snapshot) pairs
    (s >= NLEV - 1) into out [len(pairs)][NF][S][S] (device, FP32)."""
    L = nnlib()
    S = net.S
    for b, (i, s) in enumerate(pairs):
        _ck(L.lbfz_nn_pack_fields(_p(snaps[i, s - NLEV + 1]), NIN, S, S, 0, 0, S, _p(norm.in_shift),
                                  _p(norm.in_scale), _p(net.t["X0"]), CIN0, b, net.st),
            "pack_fields")
    net.forward()
    for b, (i, s) in enumerate(pairs):
        _ck(L.lbfz_nn_apply_delta(_p(net.t["OUT"]), HEAD, _p(snaps[i, s]), NF, S, S,
                                  _p(norm.d_shift), _p(norm.d_scale), _p(norm.resid), _p(out[b]),
                                  b, net.st), "apply_delta")


# ---------------------------------------------------------------- screening
# screening: largest accepted relative drift of sum C (None: not checked).  The
# LB conserves the solute to FP32 rounding (relative drift about 1e-8 over a
# stride), so the check rejects no LB state
SOLUTE_TOL = 1e-3


def mass_residual(sum_phi_b, sum_phi_a, q_b, q_a, n: int) -> float:
    """Phase-field mass residual of a prediction from per-grid sums: each LB
    step adds sum phi div u to sum phi (the phase-field source, Sec. 3.1;
    freezing enters through div u = mdot, Eq. NS1, and so does the flow's
    compression), so over a stride
        |sum phi_after - sum phi_before - (STRIDE / 2) (q_b + q_a)|
    over the liquid volume sum (1 + phi_before) / 2 of the n nodes, where q is
    sum phi div u of the state at either end (the trapezoid rule)."""
    dphi = sum_phi_a - sum_phi_b
    denom = 0.5 * (n + sum_phi_b)
    return abs(dphi - 0.5 * STRIDE * (q_b + q_a)) / max(denom, 1e-30)


def solute_drift(sum_c_b, sum_c_a) -> float:
    """|sum C_after - sum C_before| / |sum C_before|: the LB step conserves
    the solute (Sec. 3.4) to FP32 rounding, so the drift of a prediction
    measures its error in the one field with an exact budget."""
    return abs(sum_c_a - sum_c_b) / max(abs(sum_c_b), 1e-30)


def check(sums_before, sums_after, n: int, q_b: float, q_a: float, mass_tol: float = MASS_TOL,
          solute_tol: float = SOLUTE_TOL):
    """Accept a prediction (True) or send its grid to the LB (False): the
    phase-field mass residual within mass_tol and, when solute_tol is given,
    the solute drift within it; a non-finite prediction is never accepted.
    sums_*: per-field sums (phi, f_l, T, C, ...) of the grid before the
    stride and of the prediction; q_b, q_a: sum phi div u of the two.
    Returns (accept, mass residual, drift)."""
    r = mass_residual(sums_before[0], sums_after[0], q_b, q_a, n)
    d = solute_drift(sums_before[3], sums_after[3])
    ok = bool(np.all(np.isfinite(sums_after)) and np.isfinite(q_a) and r <= mass_tol and
              (solute_tol is None or d <= solute_tol))
    return ok, r, d


def check_all(sums_before, sums_after, n: int, q_b, q_a, mass_tol: float = MASS_TOL,
              solute_tol: float = SOLUTE_TOL):
    """check() for many grids at once (row i / entry i: grid i), in array
    arithmetic: the same values, without a Python loop over the grids.
    Returns the list of (accept, residual, drift)."""
    sb = np.asarray(sums_before, dtype=np.float64)
    sa = np.asarray(sums_after, dtype=np.float64)
    q_b = np.asarray(q_b, dtype=np.float64)
    q_a = np.asarray(q_a, dtype=np.float64)
    dphi = sa[:, 0] - sb[:, 0]
    denom = np.maximum(0.5 * (n + sb[:, 0]), 1e-30)
    r = np.abs(dphi - 0.5 * STRIDE * (q_b + q_a)) / denom
    d = np.abs(sa[:, 3] - sb[:, 3]) / np.maximum(np.abs(sb[:, 3]), 1e-30)
    ok = np.all(np.isfinite(sa), axis=1) & np.isfinite(q_a) & (r <= mass_tol)
    if solute_tol is not None:
        ok &= d <= solute_tol
    return [(bool(ok[i]), float(r[i]), float(d[i])) for i in range(sb.shape[0])]


class Screener:
    """Screens a batched sweep (an lbfz.Batch of equal S x S grids with walls
    on y) STRIDE steps at a time: one surrogate forward over every grid;
    grids whose prediction passes the check are restarted from it
    (equilibrium populations of the predicted phi, f_l, T, C, u and p), the
    rest are advanced by the LB (subset step).  The network reads two time
    levels: observe() records the grids' state, and a prediction needs the
    state of STRIDE steps earlier recorded first (observe(), then STRIDE
    steps of the batch, then predict() or stride()).  net: a UNet of batch >=
    the number of grids and side S.  The recorded levels hold each grid's
    solute over its mean (solute_before: the current level's sums of C);
    predictions are on the grids' own scale."""

    def __init__(self, net: UNet, norm: Normaliser, batch, mass_tol: float = MASS_TOL,
                 solute_tol: float = SOLUTE_TOL):
        import torch
        self.net, self.norm, self.batch = net, norm, batch
        self.n = len(batch.cfgs)
        S = net.S
        if any(sh != (S, S) for sh in batch.shapes) or self.n > net.B:
            raise ValueError("screening needs grids of the network's side, at most its batch")
        self.S = S
        self.walls = [int(c.get("walls", 1)) for c in batch.cfgs]
        if len(set(self.walls)) != 1:
            raise ValueError("screening needs grids with the same boundaries")
        self.mass_tol, self.solute_tol = mass_tol, solute_tol
        f = dict(dtype=torch.float32, device=net.dev)
        # the two time levels of every grid, as the network reads them:
        # hist[i, :NEXP] STRIDE steps ago, hist[i, NEXP:] now
        self.hist = torch.zeros((self.n, NIN, S, S), **f)
        self.before = self.hist[:, NEXP:]          # the current level (a view)
        self.pred = torch.zeros((self.n, NF, S, S), **f)
        # per-grid sums in one buffer, so that the check needs one
        # device-to-host copy: sum phi of the current level, every field of
        # the prediction, sum phi div u now and predicted, and the current
        # level's solute sum (the scale of its C plane)
        self.nsb, self.nsa = self.n, self.n * NF
        self.sums = torch.zeros(self.nsb + self.nsa + 3 * self.n, dtype=torch.float64,
                                device=net.dev)
        self.csum = self.sums[self.nsb + self.nsa + 2 * self.n:]
        self.parts = torch.zeros(self.n * PHI_DIV_PARTS, dtype=torch.float64, device=net.dev)
        self.levels = 0  # time levels recorded so far
        self.time = 0  # LB steps screened so far (the batch's own counter only
        # moves when some grid falls back to the LB)
        self.fused = True  # network tail, head and prediction in one launch

    def observe(self):
        """Record the grids' current state as the newer time level (the
        previous newer one becomes the older), its solute over its mean."""
        SS = self.S * self.S
        L, st = nnlib(), self.net.st
        if self.levels:
            self.hist[:, :NEXP].copy_(self.hist[:, NEXP:])
        self.batch.fields_all_to_device(NEXP, self.before, NIN * SS)
        cur = self.hist[0, NEXP]
        _ck(L.lbfz_nn_plane_sums(_p(self.hist[0, NEXP + SOLUTE_PLANE]), self.n, SS, NIN * SS,
                                 _p(self.csum), st), "plane_sums")
        _ck(L.lbfz_nn_scale_planes(_p(cur), self.n, NIN * SS, SOLUTE_PLANE, SS, _p(self.csum), 0,
                                   st), "scale_planes")
        self.levels += 1

    def predict(self):
        """Record the current state (observe()), run the network on the two
        levels, apply its output: self.pred holds the fields STRIDE steps
        ahead.  Returns the per-grid (accept, mass residual, solute drift) of
        the check."""
        if self.levels < 1:
            raise RuntimeError("observe() the grids STRIDE steps before the first prediction")
        self.observe()
        L, net, S, st = nnlib(), self.net, self.S, self.net.st
        SS = S * S
        _ck(L.lbfz_nn_pack_images(_p(self.hist), self.n, NIN * SS, NIN, S,
                                  _p(self.norm.in_shift), _p(self.norm.in_scale),
                                  _p(net.t["X0"]), CIN0, st), "pack_images")
        cur = self.hist[0, NEXP]                   # plane 0 of grid 0's current level
        if self.fused:
            net.predict_fields(self.n, cur, NIN * SS, self.pred, NF * SS, NF,
                               self.norm.d_shift, self.norm.d_scale, self.norm.resid)
        else:
            net.forward()
            _ck(L.lbfz_nn_apply_images(_p(net.t["OUT"]), HEAD, _p(cur), self.n, NIN * SS, NF,
                                       S, _p(self.norm.d_shift), _p(self.norm.d_scale),
                                       _p(self.norm.resid), _p(self.pred), NF * SS, st),
                "apply_images")
        # the prediction's solute back on its grid's scale
        _ck(L.lbfz_nn_scale_planes(_p(self.pred), self.n, NF * SS, SOLUTE_PLANE, SS,
                                   _p(self.csum), 1, st), "scale_planes")
        sums = self.sums
        sb = sums[:self.nsb]
        sa = sums[self.nsb:self.nsb + self.nsa]
        qb = sums[self.nsb + self.nsa:self.nsb + self.nsa + self.n]
        qa = sums[self.nsb + self.nsa + self.n:self.nsb + self.nsa + 2 * self.n]
        _ck(L.lbfz_nn_plane_sums(_p(cur), self.n, SS, NIN * SS, _p(sb), st), "plane_sums")
        _ck(L.lbfz_nn_plane_sums(_p(self.pred), self.n * NF, SS, SS, _p(sa), st), "plane_sums")
        walls = self.walls[0]
        _ck(L.lbfz_nn_phi_div_sums(_p(cur), self.n, NIN * SS, S, S, walls, 0, 4, 5,
                                   _p(self.parts), PHI_DIV_PARTS, _p(qb), st), "phi_div_sums")
        _ck(L.lbfz_nn_phi_div_sums(_p(self.pred), self.n, NF * SS, S, S, walls, 0, 4, 5,
                                   _p(self.parts), PHI_DIV_PARTS, _p(qa), st), "phi_div_sums")
        host = sums.cpu().numpy()
        # the check reads sum phi and sum C of the state before the stride
        hb = np.zeros((self.n, NF))
        hb[:, 0] = host[:self.nsb]
        hb[:, SOLUTE_PLANE] = host[self.nsb + self.nsa + 2 * self.n:]
        ha = host[self.nsb:self.nsb + self.nsa].reshape(self.n, NF)
        q = host[self.nsb + self.nsa:self.nsb + self.nsa + 2 * self.n]
        self.solute_before = hb[:, SOLUTE_PLANE].copy()
        return check_all(hb, ha, SS, q[:self.n], q[self.n:], self.mass_tol, self.solute_tol)

    def stride(self):
        """One screened stride; returns the accept mask (list of bool) and the
        check values."""
        res = self.predict()
        acc = [r[0] for r in res]
        rej = [i for i in range(self.n) if not acc[i]]
        if rej:
            # the LB fallback advances only the rejected grids; the others are
            # restarted from their predictions at the new time level
            self.batch.select(rej)
            self.batch.step(STRIDE)
        self.time += STRIDE
        SS = self.S * self.S
        self.batch.restart_many([i for i in range(self.n) if acc[i]],
                                [self.pred[0, f] for f in RESTART_IDX], [NF * SS] * 7)
        self.batch.select([])
        return acc, res


def rel_l2(a, b) -> list:
    """Per-field ||a - b|| / ||b|| over [NF][...] tensors."""
    return [float((a[f] - b[f]).double().norm() / (b[f].double().norm() + 1e-30))
            for f in range(NF)]
