"""Pins of the FP64 U-Net oracle (App. A.2 architecture) against definitions
written out independently of the library calls it is built from."""
import numpy as np
import pytest
import torch

from oracle import unet as U

RNG = np.random.default_rng(77)


def _conv_direct(x, W):
    """Cross-correlation with one cell of zero padding, written out as the
    sum over taps t = 9 (dx+1) + 3 (dy+1) + (dz+1)."""
    B, ci, X, Y, Z = x.shape
    co = W.shape[0]
    xp = np.zeros((B, ci, X + 2, Y + 2, Z + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((B, co, X, Y, Z))
    for t in range(27):
        dx, dy, dz = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
        sl = xp[:, :, 1 + dx:1 + dx + X, 1 + dy:1 + dy + Y, 1 + dz:1 + dz + Z]
        out += np.einsum("oc,bcxyz->boxyz", W[:, :, t], sl)
    return out


def test_block_convolution_is_the_padded_tap_sum():
    """The oracle's convolution (inside a block, with BN made the identity)
    is the direct tap sum of the weight layout [out][in][27]."""
    s = U.Shape(nx=4, ny=5, nz=6, cin=2, cout=1, widths=(3,), bottleneck=4)
    x = RNG.standard_normal((2, 2, 4, 5, 6))
    W = RNG.standard_normal((3, 2, 27))
    p = {"b.W": torch.tensor(W), "b.gamma": torch.ones(3, dtype=torch.float64),
         "b.beta": torch.zeros(3, dtype=torch.float64)}
    # evaluation-mode BN with mean 0, variance 1 - eps: the identity
    stats = {"b": (torch.zeros(3, dtype=torch.float64), torch.full((3,), 1.0 - 1e-5, dtype=torch.float64))}
    got = U._block(torch.tensor(x), p, "b", stats, training=False).numpy()
    want = np.maximum(_conv_direct(x, W), 0.0)
    assert np.abs(got - want).max() < 1e-12


def test_training_batch_norm_standardises_each_channel():
    """Training-mode BN: before the ReLU every channel has mean beta and
    biased standard deviation gamma over batch and space; the running mean
    moves 10% of the way to the batch mean, the running variance to the
    unbiased batch variance."""
    x = torch.tensor(RNG.standard_normal((3, 2, 4, 4, 5)) * 2.0 + 1.5)
    W = torch.tensor(RNG.standard_normal((4, 2, 27)))
    gamma = torch.tensor([0.5, 2.0, 1.0, 3.0], dtype=torch.float64)
    beta = torch.tensor([0.1, -0.4, 2.0, 0.0], dtype=torch.float64)
    p = {"b.W": W, "b.gamma": gamma, "b.beta": beta}
    stats = {"b": (torch.zeros(4, dtype=torch.float64), torch.ones(4, dtype=torch.float64))}
    z = torch.tensor(_conv_direct(x.numpy(), W.numpy()))
    n = z[:, 0].numel()
    U._block(x, p, "b", stats, training=True)
    # undo the ReLU on a shifted copy: choose beta large so nothing is cut
    p2 = dict(p, **{"b.beta": beta + 100.0})
    stats2 = {"b": (torch.zeros(4, dtype=torch.float64), torch.ones(4, dtype=torch.float64))}
    y = U._block(x, p2, "b", stats2, training=True) - 100.0
    for c in range(4):
        yc = y[:, c]
        assert abs(float(yc.mean()) - float(beta[c])) < 1e-12
        assert abs(float(((yc - yc.mean()) ** 2).mean().sqrt()) - float(gamma[c])) < 1e-5 * float(gamma[c])
        zc = z[:, c]
        assert abs(float(stats["b"][0][c]) - 0.1 * float(zc.mean())) < 1e-12
        var_unb = float(((zc - zc.mean()) ** 2).sum() / (n - 1))
        assert abs(float(stats["b"][1][c]) - (0.9 + 0.1 * var_unb)) < 1e-12


def _up1d(a, axis):
    """Linear upsampling by 2 with half-pixel centres along one axis: output
    2i takes 3/4 of input i and 1/4 of input i - 1, output 2i + 1 3/4 of i
    and 1/4 of i + 1, the neighbour index clamped at the faces."""
    a = np.moveaxis(a, axis, -1)
    n = a.shape[-1]
    lo = a[..., np.maximum(np.arange(n) - 1, 0)]
    hi = a[..., np.minimum(np.arange(n) + 1, n - 1)]
    out = np.empty(a.shape[:-1] + (2 * n,))
    out[..., 0::2] = 0.75 * a + 0.25 * lo
    out[..., 1::2] = 0.75 * a + 0.25 * hi
    return np.moveaxis(out, -1, axis)


def test_trilinear_upsampling_is_separable_half_pixel_interpolation():
    """The decoder's upsampling (library interpolation, align_corners False)
    equals the separable half-pixel linear interpolation written out, and
    reproduces a linear field exactly away from the faces."""
    import torch.nn.functional as F
    a = RNG.standard_normal((2, 3, 4, 5, 6))
    got = F.interpolate(torch.tensor(a), scale_factor=2, mode="trilinear", align_corners=False).numpy()
    want = _up1d(_up1d(_up1d(a, 2), 3), 4)
    assert np.abs(got - want).max() < 1e-13
    x = np.arange(8.0)[:, None, None] * 0.3 + np.arange(6.0)[None, :, None] * -0.7 + np.arange(5.0)[None, None, :] * 0.2
    up = F.interpolate(torch.tensor(x)[None, None], scale_factor=2, mode="trilinear",
                       align_corners=False).numpy()[0, 0]
    # output cell i' sits at input coordinate (i' + 1/2)/2 - 1/2
    xi = (np.arange(16) + 0.5) / 2 - 0.5
    yi = (np.arange(12) + 0.5) / 2 - 0.5
    zi = (np.arange(10) + 0.5) / 2 - 0.5
    lin = xi[:, None, None] * 0.3 + yi[None, :, None] * -0.7 + zi[None, None, :] * 0.2
    assert np.abs(up[1:-1, 1:-1, 1:-1] - lin[1:-1, 1:-1, 1:-1]).max() < 1e-12


def test_max_pooling_is_the_block_maximum():
    import torch.nn.functional as F
    a = RNG.standard_normal((2, 3, 4, 6, 8))
    got = F.max_pool3d(torch.tensor(a), 2).numpy()
    want = a.reshape(2, 3, 2, 2, 3, 2, 4, 2).max(axis=(3, 5, 7))
    assert np.array_equal(got, want)


def test_layout_and_counts():
    """Parameter count of the App. A.2 network at 4 inputs and outputs:
    27-tap convolutions of every block, BN scale and shift, the head."""
    s = U.Shape()
    n = 0
    for name, ci, co in U.blocks(s):
        n += co * ci * 27 + 2 * co
    n += 4 * 32 + 4
    assert U.param_count(s) == n
    names = [b[0] for b in U.blocks(s)]
    assert names[:2] == ["enc0a", "enc0b"] and names[8:10] == ["bota", "botb"] and names[-2:] == ["dec0a", "dec0b"]
    chans = {b[0]: (b[1], b[2]) for b in U.blocks(s)}
    assert chans["dec3a"] == (512 + 256, 256) and chans["dec0a"] == (64 + 32, 32) and chans["enc0a"] == (4, 32)


def _tiny():
    s = U.Shape(nx=8, ny=8, nz=8, cin=2, cout=2, widths=(2, 3), bottleneck=4)
    theta = RNG.standard_normal(U.param_count(s)) * 0.5
    x = RNG.standard_normal((2, 2, 8, 8, 8))
    t = RNG.uniform(0.2, 0.8, (2, 2, 8, 8, 8))
    mask = np.zeros((8, 8, 8), np.uint8)
    mask[1:7, 2:6, 2:6] = 1
    return s, theta, x, t, mask


def test_gradient_matches_finite_differences():
    """The oracle's gradient (reverse mode) against central differences of
    its own loss on a two-stage network, over a sample of parameters from
    every group (training-mode BN, so the batch statistics are
    differentiated too)."""
    s, theta, x, t, mask = _tiny()
    loss, g, _ = U.loss_and_grad(theta, x, t, mask, s)

    def L(th):
        p = U.unpack(th, s)
        return float(U.masked_mse(U.forward(p, x, s, U.running_stats(s), training=True), t, mask))

    off = 0
    checked = 0
    for name, sh in U.layout(s):
        n = int(np.prod(sh))
        for k in RNG.choice(n, size=min(n, 3), replace=False):
            i = off + int(k)
            e = np.zeros_like(theta)
            h = 1e-5
            e[i] = h
            fd = (L(theta + e) - L(theta - e)) / (2 * h)
            assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd)) + 1e-9, (name, k, fd, g[i])
            checked += 1
        off += n
    assert checked > 20


def test_head_output_in_unit_interval_and_loss_zero_on_own_output():
    s, theta, x, t, mask = _tiny()
    p = U.unpack(theta, s)
    y = U.forward(p, x, s)
    assert float(y.min()) > 0.0 and float(y.max()) < 1.0
    assert float(U.masked_mse(y, y.detach().numpy(), mask)) == 0.0
