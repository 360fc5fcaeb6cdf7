"""CPU reference of the surrogate network (test infrastructure only): the same
3-level U-Net in plain PyTorch CPU ops in float64 -- conv2d with zero padding,
ReLU, 2x2 max pooling, nearest 2x upsampling, channel concatenation -- used
to check the forward pass and every gradient of the GPU kernels.  Weights in
the GPU layout [out][tap][in] (tap t = 3 * ky + kx) are reshaped to PyTorch's
[out][in][ky][kx]; activations are NHWC on input and output."""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

# name, taps, relu (the order of the forward pass)
ORDER = (("L1a", 9, True), ("L1b", 9, True), ("L2a", 9, True), ("L2b", 9, True),
         ("L3a", 9, True), ("L3b", 9, True), ("U2", 9, True), ("L4a", 9, True),
         ("L4b", 9, True), ("U1", 9, True), ("L5a", 9, True), ("L5b", 9, True),
         ("head", 1, False))


def to_torch_weight(w: np.ndarray, taps: int) -> torch.Tensor:
    """[out][tap][in] -> [out][in][k][k]."""
    co, t, ci = w.shape
    k = 3 if taps == 9 else 1
    return torch.tensor(np.transpose(w, (0, 2, 1)).reshape(co, ci, k, k), dtype=torch.float64)


def conv(x, w, b, taps, relu):
    y = F.conv2d(x, w, b, padding=1 if taps == 9 else 0)
    return F.relu(y) if relu else y


def forward(x0_nhwc: np.ndarray, weights: dict, requires_grad: bool = False):
    """x0: [B, H, W, Cin0]; weights: name -> (w [out][tap][in], b [out]).
    Returns (OUT [B, H, W, head channels] tensor, parameter tensors)."""
    params = {}
    for name, taps, _ in ORDER:
        w, b = weights[name]
        tw = to_torch_weight(np.asarray(w, np.float64), taps).requires_grad_(requires_grad)
        tb = torch.tensor(np.asarray(b, np.float64)).requires_grad_(requires_grad)
        params[name] = (tw, tb)
    spec = {name: (taps, relu) for name, taps, relu in ORDER}

    def c(name, x):
        taps, relu = spec[name]
        return conv(x, params[name][0], params[name][1], taps, relu)

    x = torch.tensor(np.asarray(x0_nhwc, np.float64)).permute(0, 3, 1, 2)
    a1 = c("L1a", x)
    s1 = c("L1b", a1)
    a2 = c("L2a", F.max_pool2d(s1, 2))
    s2 = c("L2b", a2)
    a3 = c("L3a", F.max_pool2d(s2, 2))
    a3b = c("L3b", a3)
    u2 = c("U2", F.interpolate(a3b, scale_factor=2, mode="nearest"))
    a4 = c("L4a", torch.cat([u2, s2], dim=1))
    a4b = c("L4b", a4)
    u1 = c("U1", F.interpolate(a4b, scale_factor=2, mode="nearest"))
    a5 = c("L5a", torch.cat([u1, s1], dim=1))
    a5b = c("L5b", a5)
    out = c("head", a5b)
    return out.permute(0, 2, 3, 1), params


def loss_and_grads(x0_nhwc, weights, target, nf: int):
    """Mean squared error of the first nf output channels against target
    [B, H, W, nf]; returns (loss, name -> (dW [out][tap][in], db))."""
    out, params = forward(x0_nhwc, weights, requires_grad=True)
    t = torch.tensor(np.asarray(target, np.float64))
    loss = ((out[..., :nf] - t) ** 2).mean()
    loss.backward()
    grads = {}
    for name, taps, _ in ORDER:
        tw, tb = params[name]
        g = tw.grad.numpy()                       # [out][in][k][k]
        co, ci = g.shape[:2]
        grads[name] = (np.transpose(g.reshape(co, ci, -1), (0, 2, 1)), tb.grad.numpy())
    return float(loss.detach()), grads, out.detach().numpy()
