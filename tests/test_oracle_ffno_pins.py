"""Pins of the factorized-FNO part of the FP64 oracle (Table 2 and App. A.2,
per-axis spectral convolutions after Tran et al.): numpy's 1D real FFTs,
band-limited round trips, a single-mode closed form and finite
differences."""
import numpy as np
import pytest

from oracle import fno

RNG = np.random.default_rng(7)
SMALL_FFNO = fno.Shape(nx=16, ny=8, nz=8, cin=2, cout=2, width=3, layers=2, mx=4, my=3, mz=2, hidden=5,
                       arch="ffno", ff_hidden=4)


@pytest.mark.parametrize("axis", [2, 3, 4])
def test_axis_dft_is_numpy_rfft_truncated(axis):
    v = RNG.standard_normal((2, 3, 16, 8, 12))
    m = 3
    ref = np.take(np.fft.rfft(v, axis=axis), np.arange(m), axis=axis)
    assert np.abs(fno.axis_dft(v, axis, m) - ref).max() < 1e-11


@pytest.mark.parametrize("axis", [2, 3, 4])
def test_axis_idft_inverts_band_limited_fields(axis):
    """A field whose spectrum along the axis lies in k < m comes back
    exactly; numpy's irfft of the same coefficients gives the same field."""
    shape = [2, 3, 16, 8, 12]
    N, m = shape[axis], 3
    cshape = list(shape)
    cshape[axis] = N // 2 + 1
    C = RNG.standard_normal(cshape) + 1j * RNG.standard_normal(cshape)
    C = np.where((np.arange(N // 2 + 1) < m).reshape([-1 if i == axis else 1 for i in range(5)]), C, 0)
    v = np.fft.irfft(C, n=N, axis=axis)   # drops Im of k = 0 as the c2r convention does
    V = fno.axis_dft(v, axis, m)
    assert np.abs(fno.axis_idft(V, axis, N) - v).max() < 1e-12
    assert np.abs(fno.axis_idft(np.take(C, np.arange(m), axis=axis), axis, N) - v).max() < 1e-12


@pytest.mark.parametrize("axis", [2, 3, 4])
def test_single_mode_closed_form(axis):
    """v[c](n) = delta(c, c0) cos(2 pi k0 n_d / N_d) with k0 >= 1: the axis-d
    term is Re(W_d[k0][c0][o] exp(i theta)) = Wr cos - Wi sin; the field is
    constant along the two other axes, which see only their k = 0 mode and
    add Re(W_e[0][c0][o]) v."""
    s = fno.Shape(nx=16, ny=8, nz=12, width=3, mx=5, my=3, mz=4, arch="ffno")
    L = {"W" + a: RNG.standard_normal((m, 3, 3)) + 1j * RNG.standard_normal((m, 3, 3))
         for a, m in fno.axis_modes(s).items()}
    names = {2: "x", 3: "y", 4: "z"}
    N = (s.nx, s.ny, s.nz)[axis - 2]
    k0, c0 = 2, 1
    th = 2 * np.pi * k0 * np.arange(N) / N
    along = [-1 if i == axis else 1 for i in range(5)]   # broadcast a line along the axis
    v = np.zeros((1, 3, s.nx, s.ny, s.nz))
    v[:, c0:c0 + 1] = np.cos(th).reshape(along)
    out = fno.ffno_spectral(v, L, s)
    W = L["W" + names[axis]][k0, c0]                     # [o]
    ref = np.zeros_like(v)
    for o in range(3):
        dc = sum(L["W" + names[e]][0, c0, o].real for e in (2, 3, 4) if e != axis)
        term = W[o].real * np.cos(th) - W[o].imag * np.sin(th) + dc * np.cos(th)
        ref[:, o:o + 1] = term.reshape(along)
    assert np.abs(out - ref).max() < 1e-12


def test_zero_spectral_weights_give_a_constant_shift():
    """With every axis weight zero, s = 0 and each layer adds
    W2 GELU(b1) + b2 at every point."""
    s = SMALL_FFNO
    p = fno.unpack(fno.init_params(s, 3), s)
    shift = np.zeros(s.width)
    for L in p["layers"]:
        for a, _ in fno.AXES:
            L["W" + a] = np.zeros_like(L["W" + a])
        L["b1"], L["b2"] = RNG.standard_normal(s.ff_hidden), RNG.standard_normal(s.width)
        shift += L["W2"] @ fno.gelu(L["b1"]) + L["b2"]
    x = RNG.standard_normal((2, s.cin, s.nx, s.ny, s.nz))
    _, c = fno.forward(fno.pack(p, s), x, s)
    v = np.einsum("wc,bc...->bw...", p["P"], x) + (p["p"] + shift).reshape(1, -1, 1, 1, 1)
    assert np.abs(c["vL"] - v).max() < 1e-12


def _loss(th, x, t, mask, s):
    y, _ = fno.forward(th, x, s)
    return fno.masked_mse(y, t, mask)[0]


def test_ffno_backward_matches_finite_differences():
    s = SMALL_FFNO
    th = fno.init_params(s, 1)
    x = RNG.standard_normal((2, s.cin, s.nx, s.ny, s.nz))
    t = RNG.standard_normal((2, s.cout, s.nx, s.ny, s.nz))
    mask = np.ones((s.nx, s.ny, s.nz), np.uint8)
    mask[:3] = 0
    y, c = fno.forward(th, x, s)
    _, gy = fno.masked_mse(y, t, mask)
    g = fno.backward(th, c, gy, s)
    # every parameter of the first layer (three axis weights, re and im, and
    # the feed-forward block), the lift, the projection, and a random sample
    nlift = s.width * s.cin + s.width
    nlayer = (fno.param_count(s) - nlift - (s.hidden * s.width + s.hidden + s.cout * s.hidden + s.cout)) // s.layers
    idx = np.unique(np.concatenate([np.arange(nlift + nlayer), RNG.choice(th.size, 40, replace=False),
                                    np.arange(th.size - 20, th.size)]))
    h = 1e-5
    err = []
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (_loss(th + e, x, t, mask, s) - _loss(th - e, x, t, mask, s)) / (2 * h)
        err.append(abs(g[i] - fd) / (abs(fd) + 1e-3 * np.abs(g).max()))
    assert max(err) < 5e-5, max(err)


def test_ffno_parameter_count_and_layout():
    small = fno.Shape(nx=8, ny=8, nz=8, mx=2, my=3, mz=4, width=5, arch="ffno", ff_hidden=8)
    th = fno.init_params(small, 0)
    assert th.size == fno.param_count(small)
    assert np.array_equal(fno.pack(fno.unpack(th, small), small), th)
    # layer 0 after the lift: Wx [mx][w][w][2], then Wy [my][...], Wz [mz][...]
    L = fno.unpack(th, small)["layers"][0]
    o = 5 * small.cin + 5
    for a, m in (("x", 2), ("y", 3), ("z", 4)):
        blk = th[o:o + m * 25 * 2].reshape(m, 5, 5, 2)
        assert L["W" + a].shape == (m, 5, 5)
        assert np.array_equal(L["W" + a], blk[..., 0] + 1j * blk[..., 1])
        o += m * 25 * 2
    # width 32, 4 layers, 16 modes per axis, feed-forward 32 -> 128 -> 32
    s = fno.Shape(arch="ffno", ff_hidden=128)
    per_layer = 48 * 32 * 32 * 2 + 2 * 128 * 32 + 128 + 32
    assert fno.param_count(s) == 32 * 4 + 32 + 4 * per_layer + 128 * 32 + 128 + 4 * 128 + 4
