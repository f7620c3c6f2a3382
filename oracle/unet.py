"""FP64 CPU oracle of the 3D U-Net surrogate (paper Sec. 4, Table 2; the
architecture of App. A.2), in plain PyTorch CPU operations.

TEST INFRASTRUCTURE ONLY (see the package docstring): only the tests, the
smoke check and the benchmark's CPU baseline use it.  It shares nothing with
the HIP implementation.

Architecture (App. A.2: a standard 3D encoder-decoder with skip connections):
  encoder   four stages of widths (32, 64, 128, 256); each stage two blocks
            of 3x3x3 convolution, batch normalisation and ReLU, then 2x2x2
            max pooling;
  bottleneck two such blocks at 512 channels;
  decoder   mirrors the encoder: trilinear upsampling by 2, concatenation
            with the skip connection of the same resolution, two blocks;
  head      1x1x1 convolution to the output channels and a sigmoid.
Readings of what the appendix leaves open:
  - convolutions pad by one cell (same size) and carry no bias: the batch
    normalisation that follows has its own shift;
  - batch normalisation uses the batch statistics while training (biased
    variance, eps = 1e-5) and updates running statistics with momentum 0.1
    (unbiased variance), which evaluation uses;
  - trilinear upsampling with half-pixel centres (align_corners = False),
    clamped at the faces;
  - the concatenation puts the upsampled channels first, then the skip;
  - the head has a bias.
Parameters are one FP64 vector in the order of ``layout``; convolution
weights are [out][in][27] with tap t = 9 (dx + 1) + 3 (dy + 1) + (dz + 1)
for the input at (x + dx, y + dy, z + dz) (cross-correlation, x the slowest
spatial axis).
"""
from dataclasses import dataclass, field

import numpy as np
import torch
import torch.nn.functional as F


@dataclass
class Shape:
    nx: int = 128
    ny: int = 64
    nz: int = 64
    cin: int = 4
    cout: int = 4
    widths: tuple = field(default_factory=lambda: (32, 64, 128, 256))
    bottleneck: int = 512


def blocks(s: Shape):
    """(name, in_channels, out_channels) of every conv-BN-ReLU block in
    forward order: encoder stages, bottleneck, decoder stages."""
    out = []
    c = s.cin
    for l, w in enumerate(s.widths):
        out += [(f"enc{l}a", c, w), (f"enc{l}b", w, w)]
        c = w
    out += [("bota", c, s.bottleneck), ("botb", s.bottleneck, s.bottleneck)]
    c = s.bottleneck
    for l in reversed(range(len(s.widths))):
        w = s.widths[l]
        out += [(f"dec{l}a", c + w, w), (f"dec{l}b", w, w)]
        c = w
    return out


def layout(s: Shape):
    """(name, shape) of every parameter tensor in vector order: per block the
    convolution weight [out][in][27], the BN scale and shift [out]; then the
    head weight [cout][widths[0]] and bias [cout]."""
    out = []
    for name, ci, co in blocks(s):
        out += [(name + ".W", (co, ci, 27)), (name + ".gamma", (co,)), (name + ".beta", (co,))]
    out += [("head.W", (s.cout, s.widths[0])), ("head.b", (s.cout,))]
    return out


def param_count(s: Shape) -> int:
    return int(sum(np.prod(sh) for _, sh in layout(s)))


def unpack(theta, s: Shape):
    """Dict of torch FP64 tensors (views of a copy of theta)."""
    t = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone()
    p, o = {}, 0
    for name, sh in layout(s):
        n = int(np.prod(sh))
        p[name] = t[o:o + n].view(*sh)
        o += n
    return p


def running_stats(s: Shape):
    """Initial running statistics of every BN layer: mean 0, variance 1."""
    return {name: (torch.zeros(co, dtype=torch.float64), torch.ones(co, dtype=torch.float64))
            for name, _, co in blocks(s)}


def _block(x, p, name, stats, training):
    W = p[name + ".W"]
    co, ci, _ = W.shape
    z = F.conv3d(x, W.reshape(co, ci, 3, 3, 3), padding=1)
    rm, rv = stats[name]
    y = F.batch_norm(z, rm, rv, p[name + ".gamma"], p[name + ".beta"], training=training, momentum=0.1, eps=1e-5)
    return F.relu(y)


def forward(params, x, s: Shape, stats=None, training=True):
    """x: [B][cin][nx][ny][nz]; params: dict from unpack (tensors may require
    grad); stats: running statistics, updated in place when training.
    Returns the sigmoid output [B][cout][nx][ny][nz]."""
    if stats is None:
        stats = running_stats(s)
    h = torch.as_tensor(x, dtype=torch.float64)
    skips = []
    for l in range(len(s.widths)):
        h = _block(h, params, f"enc{l}a", stats, training)
        h = _block(h, params, f"enc{l}b", stats, training)
        skips.append(h)
        h = F.max_pool3d(h, 2)
    h = _block(h, params, "bota", stats, training)
    h = _block(h, params, "botb", stats, training)
    for l in reversed(range(len(s.widths))):
        h = F.interpolate(h, scale_factor=2, mode="trilinear", align_corners=False)
        h = torch.cat([h, skips[l]], dim=1)
        h = _block(h, params, f"dec{l}a", stats, training)
        h = _block(h, params, f"dec{l}b", stats, training)
    Wh = params["head.W"]
    y = torch.einsum("oc,bcxyz->boxyz", Wh, h) + params["head.b"][None, :, None, None, None]
    return torch.sigmoid(y)


def masked_mse(y, t, mask):
    """Mean of (y - t)^2 over the mask cells, all samples and channels (the
    loss of App. A.2 on the inner box)."""
    m = torch.as_tensor(np.asarray(mask), dtype=torch.float64)[None, None]
    cnt = y.shape[0] * y.shape[1] * m.sum()
    d = (y - torch.as_tensor(t, dtype=torch.float64)) * m
    return (d * d).sum() / cnt


def loss_and_grad(theta, x, t, mask, s: Shape, stats=None):
    """Loss and its gradient with respect to the parameter vector (training
    mode), plus the running statistics after the step."""
    p = unpack(theta, s)
    for v in p.values():
        v.requires_grad_(True)
    if stats is None:
        stats = running_stats(s)
    y = forward(p, x, s, stats, training=True)
    loss = masked_mse(y, t, mask)
    loss.backward()
    g = np.concatenate([p[name].grad.detach().numpy().ravel() for name, _ in layout(s)])
    return float(loss.item()), g, stats


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


__all__ = ["Shape", "blocks", "layout", "param_count", "unpack", "running_stats", "forward", "masked_mse",
           "loss_and_grad", "adam"]
