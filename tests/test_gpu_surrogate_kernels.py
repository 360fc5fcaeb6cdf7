"""BF16 MFMA kernels of the surrogate network against plain PyTorch CPU float64
on the same bf16-rounded operands.

Bars (relative to the largest reference value): forward and data-gradient
outputs stored in bf16 within 6e-3 (bf16 rounding is 2^-9 of a value; the
FP32 accumulation adds < 1e-5); FP32 outputs (weight gradients, head output)
within 1e-4 (bf16 products are exact in FP32, the sums carry FP32 rounding of
up to ~1e5 terms).  The whole network against the CPU reference with the same
weights: loss within 1e-2, output within 3e-2, and every parameter gradient
within 0.1 relative L2 with cosine similarity >= 0.995 -- the activations and
the gradients flowing back are rounded to bf16 (2^-9) at every one of up to
13 layers, so the first layers' gradients carry several percent of rounding
(7.6e-2 measured for the first layer, the deepest in the backward chain)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _bf16(a):
    import torch
    return torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a, np.float32)).to(dtype).cuda()


def _rel(got, ref):
    return float(np.abs(np.asarray(got, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-30))


# 3 x 3 layers run the direct kernel (4 x 64 pixel tiles, 32 or 64 output
# channels per block, 32- or 16-channel input chunks), 1 x 1 the implicit
# GEMM: the cases cover both widths, ragged tiles in x and y (widths below
# and above 64), partial and multiple input chunks (Cin 16, 48, 96, 192) and
# several column blocks (N 72, 128, 256)
@pytest.mark.parametrize("B,H,W,Cin,N,taps", [(2, 16, 16, 16, 32, 9), (1, 12, 20, 32, 40, 9),
                                              (2, 8, 8, 64, 72, 9), (2, 16, 16, 32, 8, 1),
                                              (1, 20, 24, 32, 64, 9), (1, 10, 30, 64, 128, 9),
                                              (1, 9, 14, 96, 32, 9), (2, 6, 11, 192, 64, 9),
                                              (1, 16, 24, 128, 256, 9), (1, 9, 20, 16, 64, 9),
                                              (1, 7, 12, 48, 32, 9)])
def test_conv_forward_and_gradients(B, H, W, Cin, N, taps):
    import torch
    import torch.nn.functional as F
    from paper_2511_09422_amd import surrogate as sg
    import ctypes
    rng = np.random.default_rng(B * 1000 + H + Cin + N + taps)
    x = _bf16(rng.standard_normal((B, H, W, Cin)))
    w = _bf16(rng.standard_normal((N, taps, Cin)) / np.sqrt(taps * Cin))
    bias = rng.standard_normal(N).astype(np.float32)
    dz = _bf16(rng.standard_normal((B, H, W, N)))
    k = 3 if taps == 9 else 1
    tw = torch.tensor(np.transpose(w, (0, 2, 1)).reshape(N, Cin, k, k), requires_grad=True)
    tx = torch.tensor(x).permute(0, 3, 1, 2).requires_grad_(True)
    ty = F.conv2d(tx, tw, torch.tensor(bias, dtype=torch.float64), padding=k // 2)
    ty.backward(torch.tensor(dz).permute(0, 3, 1, 2))
    ref_y = ty.detach().permute(0, 2, 3, 1).numpy()
    ref_dx = tx.grad.permute(0, 2, 3, 1).numpy()
    ref_dw = np.transpose(tw.grad.numpy().reshape(N, Cin, -1), (0, 2, 1))

    L = sg.nnlib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dx_, dw_, dz_ = _dev(x, torch.bfloat16), _dev(w, torch.bfloat16), _dev(dz, torch.bfloat16)
    db = torch.tensor(bias).cuda()
    for out_f32 in (False, True):
        y = torch.zeros(B * H * W * N, dtype=torch.float32 if out_f32 else torch.bfloat16).cuda()
        a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y, N, 0, B, H, W, taps, bias=db,
                         out_f32=out_f32)
        assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
        got = y.float().cpu().numpy().reshape(B, H, W, N)
        tol = 1e-4 if out_f32 else 6e-3
        assert _rel(got, ref_y) <= tol, (out_f32, _rel(got, ref_y))
    # data gradient: transposed weights, negated offsets
    wt = torch.zeros(N * taps * Cin, dtype=torch.bfloat16).cuda()
    assert L.lbfz_nn_transpose_w(sg._p(dw_), N, taps, Cin, sg._p(wt), st) == 0
    gx = torch.zeros(B * H * W * Cin, dtype=torch.bfloat16).cuda()
    a = sg.conv_args(dz_, N, 0, N, wt, Cin, gx, Cin, 0, B, H, W, taps, sign=-1)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
    assert _rel(gx.float().cpu().numpy().reshape(B, H, W, Cin), ref_dx) <= 6e-3
    # weight gradient (FP32, split over pixels)
    part = torch.zeros(16 * N * taps * Cin, dtype=torch.float32).cuda()
    gw = torch.zeros(N * taps * Cin, dtype=torch.float32).cuda()
    a = sg.conv_args(dx_, Cin, 0, Cin, dz_, N, None, 0, 0, B, H, W, taps, dz_cs=N)
    assert L.lbfz_nn_conv_wgrad(ctypes.byref(a), sg._p(part), 16, sg._p(gw), st) == 0
    assert _rel(gw.cpu().numpy().reshape(N, taps, Cin), ref_dw) <= 1e-4
    # bias gradient
    bpart = torch.zeros(8 * N, dtype=torch.float32).cuda()
    gb = torch.zeros(N, dtype=torch.float32).cuda()
    assert L.lbfz_nn_bias_grad(sg._p(dz_), B * H * W, N, N, sg._p(bpart), 8, sg._p(gb), st) == 0
    assert _rel(gb.cpu().numpy(), dz.sum(axis=(0, 1, 2))) <= 1e-5


@pytest.mark.parametrize("B,h,w,Cin,N", [(2, 6, 10, 64, 32), (1, 5, 8, 128, 64)])
def test_conv_reading_through_upsampling(B, h, w, Cin, N):
    """up = 1: the convolution of the nearest-2x-upsampled input, read from the
    half-resolution tensor, against upsample-then-convolve on the CPU (forward
    and weight gradient)."""
    import torch
    import torch.nn.functional as F
    from paper_2511_09422_amd import surrogate as sg
    import ctypes
    rng = np.random.default_rng(77 + Cin)
    H, W = 2 * h, 2 * w
    x = _bf16(rng.standard_normal((B, h, w, Cin)))
    w9 = _bf16(rng.standard_normal((N, 9, Cin)) / np.sqrt(9 * Cin))
    dz = _bf16(rng.standard_normal((B, H, W, N)))
    xu = torch.tensor(x).permute(0, 3, 1, 2)
    xu = F.interpolate(xu, scale_factor=2, mode="nearest").requires_grad_(True)
    tw = torch.tensor(np.transpose(w9, (0, 2, 1)).reshape(N, Cin, 3, 3), requires_grad=True)
    ty = F.conv2d(xu, tw, padding=1)
    ty.backward(torch.tensor(dz).permute(0, 3, 1, 2))
    ref_y = ty.detach().permute(0, 2, 3, 1).numpy()
    ref_dw = np.transpose(tw.grad.numpy().reshape(N, Cin, 9), (0, 2, 1))
    L = sg.nnlib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dx_, dw_, dz_ = _dev(x, torch.bfloat16), _dev(w9, torch.bfloat16), _dev(dz, torch.bfloat16)
    y = torch.zeros(B * H * W * N, dtype=torch.float32).cuda()
    a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y, N, 0, B, H, W, 9, out_f32=True, up=True)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
    assert _rel(y.cpu().numpy().reshape(B, H, W, N), ref_y) <= 1e-4
    part = torch.zeros(16 * N * 9 * Cin, dtype=torch.float32).cuda()
    gw = torch.zeros(N * 9 * Cin, dtype=torch.float32).cuda()
    a = sg.conv_args(dx_, Cin, 0, Cin, dz_, N, None, 0, 0, B, H, W, 9, dz_cs=N, up=True)
    assert L.lbfz_nn_conv_wgrad(ctypes.byref(a), sg._p(part), 16, sg._p(gw), st) == 0
    assert _rel(gw.cpu().numpy().reshape(N, 9, Cin), ref_dw) <= 1e-4
    # the data gradient has no upsampled form; odd sizes are refused
    a = sg.conv_args(dz_, N, 0, N, dw_, Cin, y, Cin, 0, B, H, W, 9, sign=-1, up=True)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == sg.LBFZ_NN_EINVAL
    a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y, N, 0, B, H - 1, W, 9, up=True)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == sg.LBFZ_NN_EINVAL


@pytest.mark.parametrize("B,H,W,Cin,N", [(2, 18, 22, 32, 32), (1, 10, 70, 32, 64)])
def test_conv_with_fused_pooling(B, H, W, Cin, N):
    """pool != NULL: the convolution also writes the 2 x 2 max pooling of its
    stored output; bit for bit lbfz_nn_maxpool2 of that output (ragged tiles
    in both directions; 32-wide and 64-wide tile shapes)."""
    import torch
    import ctypes
    from paper_2511_09422_amd import surrogate as sg
    rng = np.random.default_rng(H * W + N)
    x = _bf16(rng.standard_normal((B, H, W, Cin)))
    w9 = _bf16(rng.standard_normal((N, 9, Cin)) / np.sqrt(9 * Cin))
    bias = rng.standard_normal(N).astype(np.float32)
    L = sg.nnlib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dx_, dw_, db = _dev(x, torch.bfloat16), _dev(w9, torch.bfloat16), torch.tensor(bias).cuda()
    cs = N + 8   # output at a channel offset inside a wider tensor, as in the network
    y = torch.zeros(B * H * W * cs, dtype=torch.bfloat16).cuda()
    pooled = torch.full((B * (H // 2) * (W // 2) * N,), 7.0, dtype=torch.bfloat16).cuda()
    a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y, cs, 8, B, H, W, 9, bias=db, relu=True,
                     pool=pooled, pool_cs=N)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
    ref = torch.zeros_like(pooled)
    assert L.lbfz_nn_maxpool2(sg._p(y), cs, 8, sg._p(ref), N, B, H, W, N, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(pooled, ref)
    # odd sizes are refused
    a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y, cs, 8, B, H - 1, W, 9, bias=db,
                     pool=pooled, pool_cs=N)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == sg.LBFZ_NN_EINVAL


def test_pool_and_upsample():
    import torch
    import torch.nn.functional as F
    import ctypes
    from paper_2511_09422_amd import surrogate as sg
    rng = np.random.default_rng(5)
    B, H, W, C = 2, 8, 12, 16
    x = _bf16(rng.standard_normal((B, H, W, C)))
    g = _bf16(rng.standard_normal((B, H // 2, W // 2, C)))
    L = sg.nnlib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    tx = torch.tensor(x).permute(0, 3, 1, 2).requires_grad_(True)
    ty = F.max_pool2d(tx, 2)
    ty.backward(torch.tensor(g).permute(0, 3, 1, 2))
    dx_ = _dev(x, torch.bfloat16)
    y = torch.zeros(B * (H // 2) * (W // 2) * C, dtype=torch.bfloat16).cuda()
    assert L.lbfz_nn_maxpool2(sg._p(dx_), C, 0, sg._p(y), C, B, H, W, C, st) == 0
    assert np.array_equal(y.float().cpu().numpy().reshape(B, H // 2, W // 2, C),
                          ty.detach().permute(0, 2, 3, 1).numpy())
    gx = torch.zeros(B * H * W * C, dtype=torch.bfloat16).cuda()
    assert L.lbfz_nn_maxpool2_bwd(sg._p(dx_), C, 0, sg._p(_dev(g, torch.bfloat16)), C, sg._p(gx),
                                  C, 0, 0, B, H, W, C, st) == 0
    assert np.array_equal(gx.float().cpu().numpy().reshape(B, H, W, C),
                          tx.grad.permute(0, 2, 3, 1).numpy())
    # upsampling: forward and gradient
    up = torch.zeros(B * 4 * H * W * C, dtype=torch.bfloat16).cuda()
    assert L.lbfz_nn_upsample2(sg._p(dx_), B, H, W, C, sg._p(up), st) == 0
    ref = F.interpolate(torch.tensor(x).permute(0, 3, 1, 2), scale_factor=2, mode="nearest")
    assert np.array_equal(up.float().cpu().numpy().reshape(B, 2 * H, 2 * W, C),
                          ref.permute(0, 2, 3, 1).numpy())
    gu = _bf16(rng.standard_normal((B, 2 * H, 2 * W, C)))
    gd = torch.zeros(B * H * W * C, dtype=torch.bfloat16).cuda()
    assert L.lbfz_nn_upsample2_bwd(sg._p(_dev(gu, torch.bfloat16)), B, H, W, C, sg._p(gd), st) == 0
    refg = gu.reshape(B, H, 2, W, 2, C).sum(axis=(2, 4))
    assert _rel(gd.float().cpu().numpy().reshape(B, H, W, C), refg) <= 6e-3


def test_unet_loss_and_gradients_against_cpu_reference():
    import torch
    from oracle import unet_ref
    from paper_2511_09422_amd import surrogate as sg
    B, S = 2, 32
    rng = np.random.default_rng(11)
    w = sg.init_weights(3)
    for k in w:   # weights as the GPU sees them (bf16)
        w[k] = (_bf16(w[k][0]).astype(np.float32), w[k][1] + 0.01 * rng.standard_normal(
            w[k][1].shape).astype(np.float32))
    x = np.zeros((B, S, S, sg.CIN0))
    yy, xx = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    for c in range(sg.NF):
        x[..., c] = np.sin(0.2 * (c + 1) * xx + 0.3 * yy)[None] + 0.3 * rng.standard_normal((B, S, S))
    x = _bf16(x)
    tgt = rng.standard_normal((B, S, S, sg.NF)) * 0.5
    loss_ref, grads_ref, out_ref = unet_ref.loss_and_grads(x, w, tgt, sg.NF)

    net = sg.UNet(w, B, S)
    net.t["X0"].copy_(torch.tensor(x.reshape(-1), dtype=torch.float32).to(torch.bfloat16))
    net.target.copy_(torch.tensor(tgt.reshape(-1), dtype=torch.float32))
    net.forward()
    net.loss()
    net.backward()
    torch.cuda.synchronize()
    out = net.t["OUT"].cpu().numpy().reshape(B, S, S, sg.HEAD)
    loss = float(net.loss_t.cpu().numpy()[0])
    print(f"[unet] loss gpu {loss:.6f} cpu {loss_ref:.6f}; out rel {_rel(out, out_ref):.2e}",
          flush=True)
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    assert _rel(out, out_ref) <= 3e-2
    g = net.grads()
    bad = []
    for name in g:
        for j, part in enumerate(("w", "b")):
            a, r = g[name][j].ravel(), grads_ref[name][j].ravel()
            if name == "head":   # only the used outputs carry gradient
                a, r = g[name][j][:sg.NF].ravel(), grads_ref[name][j][:sg.NF].ravel()
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            cos = float(a @ r / max(np.linalg.norm(a) * np.linalg.norm(r), 1e-30))
            print(f"[unet] grad {name}.{part} rel L2 {rel:.2e} cos {cos:.5f}", flush=True)
            if rel > 0.1 or cos < 0.995:
                bad.append((name, part, rel, cos))
    assert not bad, bad


def test_training_reduces_loss():
    import torch
    from paper_2511_09422_amd import surrogate as sg
    B, S = 4, 64
    rng = np.random.default_rng(2)
    net = sg.UNet(sg.init_weights(0), B, S)
    yy, xx = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    x = np.zeros((B, S, S, sg.CIN0), np.float32)
    tgt = np.zeros((B, S, S, sg.NF), np.float32)
    for b in range(B):
        for c in range(sg.NF):
            ph = rng.uniform(0, 6)
            x[b, :, :, c] = np.sin(0.1 * (c + 1) * xx + 0.07 * yy + ph)
            tgt[b, :, :, c] = 0.5 * np.cos(0.1 * (c + 1) * xx + 0.07 * yy + ph)
    net.t["X0"].copy_(torch.tensor(x.reshape(-1)).to(torch.bfloat16))
    net.target.copy_(torch.tensor(tgt.reshape(-1)))
    losses = []
    for it in range(60):
        net.forward()
        net.loss()
        net.backward()
        net.adam(2e-3)
        losses.append(float(net.loss_t.cpu().numpy()[0]))
    print(f"[unet] training loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.25 * losses[0]


@pytest.mark.parametrize("B,S,Cin", [(3, 72, 32), (2, 20, 64)])
def test_conv_tail_fused_head_and_prediction(B, S, Cin):
    """lbfz_nn_conv_tail (the last 3 x 3 convolution, the 1 x 1 head and the
    prediction of whole grids in one launch) against (a) the CPU float64
    reference -- convolution of the bf16 operands, bias, ReLU, rounded to
    bf16 as the network stores it, head, prediction -- within the bf16 bar
    (6e-3 of the largest increment), and (b) the unfused kernels (convolution,
    1 x 1 head with FP32 output, lbfz_nn_apply_images) within 1e-5 of the
    largest increment (the two heads sum the same bf16 inputs in FP32 in
    different orders); the convolution output, when also requested, equals
    lbfz_nn_conv's bit for bit; nothing is written past a grid's planes.
    Ragged tiles: S = 72 (two tile columns, the second partial), S = 20
    (partial tile rows)."""
    import ctypes
    import torch
    import torch.nn.functional as F
    from paper_2511_09422_amd import surrogate as sg
    rng = np.random.default_rng(7 * B + S + Cin)
    N, NH, NF = 32, 8, 6
    npx = S * S
    x = _bf16(rng.standard_normal((B, S, S, Cin)))
    w = _bf16(rng.standard_normal((N, 9, Cin)) / np.sqrt(9 * Cin))
    bias = rng.standard_normal(N).astype(np.float32) * 0.1
    hw = _bf16(rng.standard_normal((NH, N)) / np.sqrt(N))
    hb = rng.standard_normal(NH).astype(np.float32) * 0.1
    shift = rng.standard_normal(NF).astype(np.float32) * 0.01
    scale = (1.0 + rng.random(NF)).astype(np.float32)
    resid = np.array([1, 1, 1, 1, 0, 0], np.float32)
    bstride, pstride = NF * npx + 40, NF * npx + 24
    before = np.full((B, bstride), np.nan, np.float32)
    before[:, :NF * npx] = rng.standard_normal((B, NF * npx))
    # CPU reference
    tw = torch.tensor(np.transpose(w, (0, 2, 1)).reshape(N, Cin, 3, 3))
    tx = torch.tensor(x).permute(0, 3, 1, 2)
    y = F.conv2d(tx, tw, torch.tensor(bias, dtype=torch.float64), padding=1)
    y = _bf16(np.maximum(y.permute(0, 2, 3, 1).numpy(), 0.0))          # B, S, S, N
    head = y @ hw.astype(np.float64).T + hb.astype(np.float64)          # B, S, S, NH
    inc_ref = np.stack([head[..., f] / scale[f] for f in range(NF)], 1).reshape(B, NF, npx)
    # GPU
    L = sg.nnlib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dx_, dw_ = _dev(x, torch.bfloat16), _dev(w, torch.bfloat16)
    db, dhw, dhb = torch.tensor(bias).cuda(), _dev(hw, torch.bfloat16), torch.tensor(hb).cuda()
    dsh, dsc, dre = torch.tensor(shift).cuda(), torch.tensor(scale).cuda(), torch.tensor(resid).cuda()
    dbefore = torch.tensor(before).cuda()

    def tail(out):
        pred = torch.full((B, pstride), float("nan"), dtype=torch.float32, device="cuda")
        a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, out, N, 0, B, S, S, 9, bias=db, relu=True)
        t = sg.lbfz_tail_args()
        t.head_w, t.head_b, t.nh, t.nf = dhw.data_ptr(), dhb.data_ptr(), NH, NF
        t.before, t.before_stride = dbefore.data_ptr(), bstride
        t.shift, t.scale, t.resid = dsh.data_ptr(), dsc.data_ptr(), dre.data_ptr()
        t.pred, t.pred_stride = pred.data_ptr(), pstride
        assert L.lbfz_nn_conv_tail(ctypes.byref(a), ctypes.byref(t), st) == 0
        torch.cuda.synchronize()
        return pred.cpu().numpy()

    y_tail = torch.zeros(B * npx * N, dtype=torch.bfloat16, device="cuda")
    p1 = tail(None)
    p2 = tail(y_tail)
    assert np.array_equal(p1, p2, equal_nan=True)
    assert np.isnan(p1[:, NF * npx:]).all()
    pf = p1[:, :NF * npx].reshape(B, NF, npx).astype(np.float64)
    bf = before[:, :NF * npx].reshape(B, NF, npx).astype(np.float64)
    inc = pf - resid[None, :, None] * bf - shift[None, :, None]
    assert _rel(inc, inc_ref) <= 6e-3, _rel(inc, inc_ref)
    # unfused kernels
    y_conv = torch.zeros(B * npx * N, dtype=torch.bfloat16, device="cuda")
    a = sg.conv_args(dx_, Cin, 0, Cin, dw_, N, y_conv, N, 0, B, S, S, 9, bias=db, relu=True)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
    out = torch.zeros(B * npx * NH, dtype=torch.float32, device="cuda")
    a = sg.conv_args(y_conv, N, 0, N, dhw, NH, out, NH, 0, B, S, S, 1, bias=dhb, out_f32=True)
    assert L.lbfz_nn_conv(ctypes.byref(a), st) == 0
    pred_u = torch.full((B, pstride), float("nan"), dtype=torch.float32, device="cuda")
    assert L.lbfz_nn_apply_images(sg._p(out), NH, sg._p(dbefore), B, bstride, NF, S, sg._p(dsh),
                                  sg._p(dsc), sg._p(dre), sg._p(pred_u), pstride, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(y_tail, y_conv)
    pu = pred_u.cpu().numpy()[:, :NF * npx].reshape(B, NF, npx).astype(np.float64)
    e = float(np.abs(pf - pu).max() / np.abs(inc_ref).max())
    assert e <= 1e-5, e


@pytest.mark.parametrize("nx,ny,walls,nimg", [(64, 48, 1, 3), (40, 72, 0, 2), (256, 256, 1, 2)])
def test_phi_div_sums_against_cpu(nx, ny, walls, nimg):
    """lbfz_nn_phi_div_sums (the screening check's sum of phi div u per grid)
    against the FP64 reference on the same FP32 fields: equal to FP64
    summation-order rounding (1e-12 of the sum of |phi div u|), for planes at
    a stride larger than the fields a grid holds."""
    import torch
    from paper_2511_09422_amd import surrogate as sg
    from tests.divergence_ref import div_d2q9
    rng = np.random.default_rng(nx + ny + walls)
    npx = nx * ny
    stride = 9 * npx
    host = rng.standard_normal((nimg, 9, ny, nx)).astype(np.float32)
    host[:, 4:6] *= 1e-3
    dev = torch.tensor(host.reshape(-1)).cuda()
    out = torch.zeros(nimg, dtype=torch.float64).cuda()
    parts = torch.zeros(nimg * 16, dtype=torch.float64).cuda()
    L = sg.nnlib()
    st = torch.cuda.current_stream().cuda_stream
    for nparts in (1, 3, 16):
        out.zero_()
        assert L.lbfz_nn_phi_div_sums(sg._p(dev), nimg, stride, nx, ny, walls, 0, 4, 5,
                                      sg._p(parts), nparts, sg._p(out), st) == 0
        got = out.cpu().numpy()
        for g in range(nimg):
            t = host[g, 0].astype(np.float64) * div_d2q9(host[g, 4], host[g, 5], walls)
            assert abs(got[g] - t.sum()) <= 1e-12 * np.abs(t).sum(), (nparts, g, got[g], t.sum())
    # argument checks: a stride too short for the highest plane, a bad side,
    # more parts than rows
    assert L.lbfz_nn_phi_div_sums(sg._p(dev), nimg, 5 * npx, nx, ny, walls, 0, 4, 5,
                                  sg._p(parts), 4, sg._p(out), st) == sg.LBFZ_NN_EINVAL
    assert L.lbfz_nn_phi_div_sums(sg._p(dev), nimg, stride, 1, ny, walls, 0, 4, 5,
                                  sg._p(parts), 4, sg._p(out), st) == sg.LBFZ_NN_EINVAL
    assert L.lbfz_nn_phi_div_sums(sg._p(dev), nimg, stride, nx, ny, walls, 0, 4, 5,
                                  sg._p(parts), ny + 1, sg._p(out), st) == sg.LBFZ_NN_EINVAL


@pytest.mark.parametrize("nimg,n,stride,plane", [(3, 1000, 4100, 2), (5, 4096, 4 * 4096, 3)])
def test_scale_planes_by_grid_sums(nimg, n, stride, plane):
    """lbfz_nn_scale_planes (a grid's solute over its mean, and back): plane
    `plane` of every image times n / sums[i], then times sums[i] / n, each
    factor formed in FP64 and applied in FP32 -- equal to that arithmetic bit
    for bit; the other planes untouched."""
    import torch
    from paper_2511_09422_amd import surrogate as sg
    rng = np.random.default_rng(nimg + n)
    host = rng.uniform(0.01, 0.1, size=nimg * stride).astype(np.float32)
    sums = np.array([host[i * stride + plane * n:i * stride + (plane + 1) * n].astype(np.float64).sum()
                     for i in range(nimg)])
    dev = torch.tensor(host).cuda()
    dsum = torch.tensor(sums).cuda()
    L = sg.nnlib()
    st = torch.cuda.current_stream().cuda_stream
    assert L.lbfz_nn_scale_planes(sg._p(dev), nimg, stride, plane, n, sg._p(dsum), 0, st) == 0
    got = dev.cpu().numpy()
    want = host.copy()
    for i in range(nimg):
        sl = slice(i * stride + plane * n, i * stride + (plane + 1) * n)
        want[sl] = host[sl] * np.float32(n / sums[i])
    assert np.array_equal(got, want)
    assert L.lbfz_nn_scale_planes(sg._p(dev), nimg, stride, plane, n, sg._p(dsum), 1, st) == 0
    back = dev.cpu().numpy()
    for i in range(nimg):
        sl = slice(i * stride + plane * n, i * stride + (plane + 1) * n)
        want[sl] = want[sl] * np.float32(sums[i] / n)
    assert np.array_equal(back, want)
    assert np.abs(back - host).max() <= 1e-6 * np.abs(host).max()
    assert L.lbfz_nn_scale_planes(sg._p(dev), nimg, plane * n, plane, n, sg._p(dsum), 0,
                                  st) == sg.LBFZ_NN_EINVAL
