"""Pins of the FP64 Fourier-neural-operator oracle against numpy's FFTs,
linear-algebra identities and finite differences."""
import math

import numpy as np
import pytest

from oracle import fno

RNG = np.random.default_rng(42)
SMALL = fno.Shape(nx=8, ny=8, nz=8, cin=2, cout=2, width=3, layers=2, mx=2, my=2, mz=2, hidden=5)
SMALL_SIREN = fno.Shape(nx=8, ny=8, nz=8, cin=2, cout=2, width=3, layers=2, mx=2, my=2, mz=2, hidden=5,
                        proj="siren", w0=30.0)
SMALL_HYBRID = fno.Shape(nx=8, ny=8, nz=8, cin=2, cout=2, width=3, layers=2, mx=2, my=2, mz=2, hidden=5,
                         arch="hybrid", ff_hidden=4)


def corner(Vfull, s):
    kx = fno.mode_indices(s.mx) % s.nx
    ky = fno.mode_indices(s.my) % s.ny
    return Vfull[..., kx, :, :][..., :, ky, :][..., :s.mz]


def test_forward_dft_is_rfftn_corner_modes():
    s = fno.Shape(nx=16, ny=8, nz=12, mx=3, my=2, mz=4)
    v = RNG.standard_normal((2, 3, s.nx, s.ny, s.nz))
    V = fno.forward_dft(v, fno.dft_matrices(s))
    ref = corner(np.fft.rfftn(v, axes=(2, 3, 4)), s)
    assert np.abs(V - ref).max() < 1e-11


def test_inverse_dft_is_irfftn_of_zero_padded_spectrum():
    s = fno.Shape(nx=16, ny=8, nz=12, mx=3, my=2, mz=4)
    Y = RNG.standard_normal((2, 3, 2 * s.mx, 2 * s.my, s.mz)) + 1j * RNG.standard_normal((2, 3, 2 * s.mx, 2 * s.my, s.mz))
    full = np.zeros((2, 3, s.nx, s.ny, s.nz // 2 + 1), complex)
    kx = fno.mode_indices(s.mx) % s.nx
    ky = fno.mode_indices(s.my) % s.ny
    for a, i in enumerate(kx):
        for b, j in enumerate(ky):
            full[:, :, i, j, :s.mz] = Y[:, :, a, b, :]
    ref = np.fft.irfftn(full, s=(s.nx, s.ny, s.nz), axes=(2, 3, 4))
    out = fno.inverse_dft(Y, fno.dft_matrices(s), s)
    assert np.abs(out - ref).max() < 1e-12


def test_identity_spectral_weights_low_pass_convention():
    """R(T v) with identity mixing keeps a field made of retained modes whose
    conjugate partners are also retained, and halves a kz = 0 mode whose
    partner is not retained (kx = -m is kept, +m is not: the c2r real part
    of the corner convention)."""
    s = fno.Shape(nx=16, ny=8, nz=8, mx=3, my=2, mz=3)
    mats = fno.dft_matrices(s)

    def lp(u):
        return fno.inverse_dft(fno.forward_dft(u, mats), mats, s)

    x, y, z = np.meshgrid(np.arange(s.nx), np.arange(s.ny), np.arange(s.nz), indexing="ij")
    band = np.cos(2 * np.pi * (2 * x / s.nx + 1 * y / s.ny + 2 * z / s.nz)) + 0.3 * np.sin(2 * np.pi * x / s.nx)
    assert np.abs(lp(band[None, None]) - band).max() < 1e-12
    edge = np.cos(2 * np.pi * 3 * x / s.nx)  # kx = +-3 = +-mx, kz = 0
    assert np.abs(lp(edge[None, None]) - 0.5 * edge).max() < 1e-12
    v = RNG.standard_normal((1, 2, s.nx, s.ny, s.nz))
    assert np.abs(lp(lp(v)) - lp(v)).max() > 1e-3  # not a projection


@pytest.mark.parametrize("which", ["forward", "inverse"])
def test_adjoint_dot_product_identities(which):
    s = fno.Shape(nx=8, ny=8, nz=8, mx=2, my=2, mz=3)
    mats = fno.dft_matrices(s)
    v = RNG.standard_normal((1, 1, 8, 8, 8))
    G = RNG.standard_normal((1, 1, 4, 4, 3)) + 1j * RNG.standard_normal((1, 1, 4, 4, 3))
    if which == "forward":
        lhs = np.sum((fno.forward_dft(v, mats) * np.conj(G)).real)
        rhs = np.sum(v * fno.adjoint_forward_dft(G, mats))
    else:
        lhs = np.sum(fno.inverse_dft(G, mats, s) * v)
        rhs = np.sum((np.conj(fno.adjoint_inverse_dft(v, mats, s)) * G).real)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert abs(fno.gelu(np.array(0.0))) == 0.0
    assert np.abs(fno.gelu(np.array([10.0])) - 10.0).max() < 1e-12
    h = 1e-6
    fd = (fno.gelu(x + h) - fno.gelu(x - h)) / (2 * h)
    assert np.abs(fd - fno.gelu_grad(x)).max() < 1e-8
    # GELU(x) = x Phi(x) with the normal CDF
    phi = np.array([0.5 * (1 + math.erf(v / math.sqrt(2))) for v in x])
    assert np.abs(fno.gelu(x) - x * phi).max() < 1e-14


def test_siren_activation_and_derivative():
    s = SMALL_SIREN
    x = np.linspace(-0.3, 0.3, 101)
    assert np.array_equal(fno.proj_act(x, s), np.sin(30.0 * x))
    h = 1e-7
    fd = (fno.proj_act(x + h, s) - fno.proj_act(x - h, s)) / (2 * h)
    assert np.abs(fd - fno.proj_act_grad(x, s)).max() < 1e-5 * 30.0
    # the default projection is GELU
    assert np.array_equal(fno.proj_act(x, SMALL), fno.gelu(x))


def test_siren_initialisation_scales():
    s = fno.Shape(width=32, hidden=128, proj="siren")
    p = fno.unpack(fno.init_params(s, 0), s)
    assert np.abs(p["Q1"]).max() <= 1.0 / 32 and np.abs(p["Q1"]).max() > 0.9 / 32
    bound = math.sqrt(6.0 / 128) / 30.0
    assert np.abs(p["Q2"]).max() <= bound and np.abs(p["Q2"]).max() > 0.9 * bound


def test_parameter_pack_round_trip_and_count():
    th = fno.init_params(SMALL, 3)
    assert th.size == fno.param_count(SMALL)
    assert np.array_equal(fno.pack(fno.unpack(th, SMALL), SMALL), th)
    full = fno.Shape()
    # width 32, 4 layers, 32x32x16 modes: 134,217,728 spectral reals
    assert fno.param_count(full) - 4 * (32 * 32 + 32) - 32 * 4 - 32 - 128 * 32 - 128 - 4 * 128 - 4 == 134217728


def _loss(th, x, t, mask, s):
    y, _ = fno.forward(th, x, s)
    return fno.masked_mse(y, t, mask)[0]


@pytest.mark.parametrize("s", [SMALL, SMALL_SIREN, SMALL_HYBRID], ids=["gelu", "siren", "hybrid"])
def test_backward_matches_finite_differences(s):
    th = fno.init_params(s, 1)
    x = RNG.standard_normal((2, s.cin, s.nx, s.ny, s.nz))
    t = RNG.standard_normal((2, s.cout, s.nx, s.ny, s.nz))
    mask = np.ones((s.nx, s.ny, s.nz), np.uint8)
    mask[:2] = 0
    y, c = fno.forward(th, x, s)
    _, gy = fno.masked_mse(y, t, mask)
    g = fno.backward(th, c, gy, s)
    # every parameter group is sampled: lift, spectral, pointwise, projection
    nproj = s.hidden * s.width + s.hidden + s.cout * s.hidden + s.cout
    parts = [np.arange(0, 6), RNG.choice(th.size, 40, replace=False), np.arange(th.size - nproj, th.size)]
    if s.arch == "hybrid":
        # every feed-forward parameter of every layer (W1, b1, W2, b2 follow
        # the layer's spectral weights)
        nlift, nspec = s.width * s.cin + s.width, 4 * s.mx * s.my * s.mz * s.width * s.width * 2
        nff = 2 * s.ff_hidden * s.width + s.ff_hidden + s.width
        for l in range(s.layers):
            o = nlift + l * (nspec + nff) + nspec
            parts.append(np.arange(o, o + nff))
    idx = np.unique(np.concatenate(parts))
    # central differences: truncation O(h^2), rounding O(eps L / h); the
    # bound leaves room for both and still fails on any wrong term (O(1))
    h = 1e-5
    err = []
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (_loss(th + e, x, t, mask, s) - _loss(th - e, x, t, mask, s)) / (2 * h)
        err.append(abs(g[i] - fd) / (abs(fd) + 1e-3 * np.abs(g).max()))
    assert max(err) < 5e-5, max(err)


def _ffn(v, L):
    """The hybrid's residual block without its spectral part, written out
    per point: v + W2 GELU(W1 v + b1) + b2."""
    z = np.einsum("hc,bc...->bh...", L["W1"], v) + L["b1"].reshape(1, -1, 1, 1, 1)
    return v + np.einsum("ch,bh...->bc...", L["W2"], fno.gelu(z)) + L["b2"].reshape(1, -1, 1, 1, 1)


def test_hybrid_with_identity_spectral_weights_is_a_pointwise_residual_block():
    """Identity mixing on a lifted input made of retained modes reproduces
    the field (s = v), so one hybrid layer equals the pointwise residual
    feed-forward block, followed by the projection."""
    s = fno.Shape(nx=16, ny=8, nz=8, cin=2, cout=2, width=3, layers=1, mx=3, my=2, mz=3, hidden=5,
                  arch="hybrid", ff_hidden=6)
    p = fno.unpack(fno.init_params(s, 4), s)
    p["p"] = RNG.standard_normal(s.width)
    L = p["layers"][0]
    L["W"] = np.broadcast_to(np.eye(s.width)[:, :, None, None, None], L["W"].shape).astype(complex)
    L["b1"], L["b2"] = RNG.standard_normal(s.ff_hidden), RNG.standard_normal(s.width)
    x, y, z = np.meshgrid(np.arange(s.nx), np.arange(s.ny), np.arange(s.nz), indexing="ij")
    xin = np.stack([np.cos(2 * np.pi * (2 * x / s.nx + y / s.ny + 2 * z / s.nz)),
                    np.sin(2 * np.pi * (x / s.nx - z / s.nz))])[None]
    out, _ = fno.forward(fno.pack(p, s), xin, s)
    v0 = np.einsum("wc,bc...->bw...", p["P"], xin) + p["p"].reshape(1, -1, 1, 1, 1)
    v1 = _ffn(v0, L)
    h1 = np.einsum("hw,bw...->bh...", p["Q1"], v1) + p["q1"].reshape(1, -1, 1, 1, 1)
    ref = np.einsum("oh,bh...->bo...", p["Q2"], fno.gelu(h1)) + p["q2"].reshape(1, -1, 1, 1, 1)
    assert np.abs(out - ref).max() < 1e-11 * np.abs(ref).max()


def test_hybrid_with_zero_output_weights_adds_its_biases():
    """With W2 = 0 every hybrid layer adds b2 whatever its spectral weights:
    v_L = P x + p + sum_l b2_l."""
    s = SMALL_HYBRID
    p = fno.unpack(fno.init_params(s, 2), s)
    shift = np.zeros(s.width)
    for L in p["layers"]:
        L["W2"] = np.zeros_like(L["W2"])
        L["b2"] = RNG.standard_normal(s.width)
        shift += L["b2"]
    x = RNG.standard_normal((2, s.cin, s.nx, s.ny, s.nz))
    out, c = fno.forward(fno.pack(p, s), x, s)
    v = np.einsum("wc,bc...->bw...", p["P"], x) + (p["p"] + shift).reshape(1, -1, 1, 1, 1)
    assert np.abs(c["vL"] - v).max() < 1e-12
    h1 = np.einsum("hw,bw...->bh...", p["Q1"], v) + p["q1"].reshape(1, -1, 1, 1, 1)
    ref = np.einsum("oh,bh...->bo...", p["Q2"], fno.gelu(h1)) + p["q2"].reshape(1, -1, 1, 1, 1)
    assert np.abs(out - ref).max() < 1e-12


def test_hybrid_parameter_count():
    s = fno.Shape(arch="hybrid", ff_hidden=128)
    th = fno.init_params(fno.Shape(nx=8, ny=8, nz=8, mx=2, my=2, mz=2, arch="hybrid", ff_hidden=8), 0)
    assert th.size == fno.param_count(fno.Shape(nx=8, ny=8, nz=8, mx=2, my=2, mz=2, arch="hybrid", ff_hidden=8))
    # width 32, 4 layers, 32x32x16 modes, feed-forward 32 -> 128 -> 32
    assert fno.param_count(s) - 134217728 == 4 * (2 * 128 * 32 + 128 + 32) + 32 * 4 + 32 + 128 * 32 + 128 + 4 * 128 + 4


def test_masked_mse_only_counts_mask_cells():
    y = RNG.standard_normal((2, 3, 4, 4, 4))
    t = y.copy()
    mask = np.zeros((4, 4, 4), np.uint8)
    mask[1, 2, 3] = 1
    t[:, :, 0, 0, 0] += 5.0
    loss, g = fno.masked_mse(y, t, mask)
    assert loss == 0.0 and np.abs(g).max() == 0.0
    t[:, :, 1, 2, 3] += 1.0
    loss, g = fno.masked_mse(y, t, mask)
    assert abs(loss - 1.0) < 1e-15


def test_adam_first_step_is_lr_times_sign():
    th = RNG.standard_normal(10)
    g = RNG.standard_normal(10)
    new, m, v = fno.adam(th, g, np.zeros(10), np.zeros(10), 1, 0.01)
    assert np.abs((th - new) - 0.01 * np.sign(g)).max() < 1e-8
    # and it minimises a quadratic
    x = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 2001):
        x, m, v = fno.adam(x, 2 * x, m, v, t, 0.05)
    assert np.abs(x).max() < 1e-3


def test_inner_box_mask_extent():
    s = fno.Shape()
    m = fno.inner_box_mask(s)
    assert m.sum() == (int(0.9 * 128) - int(0.1 * 128)) * 32 * 32
    assert m[11, 16, 16] == 0 and m[12, 16, 16] == 1 and m[115, 16, 16] == 0
