"""FP64 numpy oracle of the 3D Fourier neural operator surrogate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Architecture (paper Sec. 4 and App. A.2: FNO with 32 channels, 4 layers, a
feed-forward lifting; predicts mean flow fields from geometry and Re):
  v0 = P x + p                                  lifting cin -> width
  for l in layers:
      V = T(v)        truncated 3D real DFT: kx, ky in {0..m-1, -m..-1},
                      kz in {0..m-1} (corner modes of the half spectrum)
      Y[b,o,k] = sum_c V[b,c,k] W_l[c,o,k]     per-mode complex mixing
      s = R(Y)        truncated inverse (the c2r convention of irfftn: the
                      kz = 0 term enters with its real part, kz >= 1 doubled,
                      normalised by 1/(X Y Z))
      h = s + Wp_l v + bp_l
      v = GELU(h) except after the last layer (GELU with erf)
  y = Q2 act(Q1 v + q1) + q2                    projection width -> hidden -> cout
                      act = GELU, or for the SIREN projection of App. A.2
                      act(h) = sin(w0 h) (w0 = 30)
Hybrid F/FNO (arch = "hybrid", App. A.2: the factorized FNO's layer
structure with the unfactorized 3D spectral convolution of the FNO): each
layer is a residual block around a pointwise feed-forward network,
      s = R(W_l . T(v))                         the same spectral convolution
      v = v + W2_l GELU(W1_l s + b1_l) + b2_l   width -> ff_hidden -> width
with no bypass channel map and no activation on the residual stream.
Factorized FNO (arch = "ffno", Table 2 and App. A.2 after Tran et al.): the
same residual feed-forward block as the hybrid, with the spectral
convolution split into one 1D convolution per axis and summed,
      s = sum_{d in x, y, z} R_d(W_{d,l} . T_d(v))
      T_d  1D real DFT along axis d, modes k = 0..m_d - 1
           (V_k = sum_n v_n exp(-2 pi i k n / N_d))
      W    per-mode complex mixing of the channels, Y_k[o] = sum_c V_k[c] W[k][c][o]
      R_d  1D c2r inverse along d: (1/N_d) sum_k c_k Re(Y_k exp(+2 pi i k n / N_d)),
           c_0 = 1, c_k = 2 for k >= 1 (m_d <= N_d / 2, so no Nyquist term)
Loss: mean squared error over the cells of a mask (App. A.2, inner region),
all samples and output channels.  Optimiser: Adam (beta 0.9, 0.999,
eps 1e-8).  The projection is a GELU MLP by default; proj = "siren" gives
the paper's SIREN (sine activation with frequency w0).

Parameter vector layout (shared with the GPU library's C ABI):
  lift W [width][cin], lift b [width];
  per layer: spectral W [2mx][2my][mz][width][width][2] (re, im; first
  index j -> kx = j for j < mx else j - 2mx, likewise ky), then for the
  FNO the pointwise W [width][width] (out, in) and bias [width], for the
  hybrid W1 [ff_hidden][width], b1 [ff_hidden], W2 [width][ff_hidden],
  b2 [width]; for the factorized FNO the spectral block is the three axis
  weights Wx [mx][width][width][2], Wy [my][...], Wz [mz][...] (mode, in,
  out, re/im) followed by the hybrid's W1, b1, W2, b2;
  proj W1 [hidden][width], b1 [hidden], W2 [cout][hidden], b2 [cout].
"""
from dataclasses import dataclass
import math

import numpy as np
from scipy.special import erf


@dataclass(frozen=True)
class Shape:
    nx: int = 128
    ny: int = 64
    nz: int = 64
    cin: int = 4
    cout: int = 4
    width: int = 32
    layers: int = 4
    mx: int = 16
    my: int = 16
    mz: int = 16
    hidden: int = 128
    proj: str = "gelu"
    w0: float = 30.0
    arch: str = "fno"
    ff_hidden: int = 128


AXES = (("x", 2), ("y", 3), ("z", 4))  # factorized FNO: weight name suffix, array axis of [B][C][X][Y][Z]


def axis_modes(s: Shape):
    """Retained modes per axis of the factorized FNO."""
    return {"x": s.mx, "y": s.my, "z": s.mz}


def param_count(s: Shape) -> int:
    w = s.width
    n = w * s.cin + w
    spec = (2 * s.mx) * (2 * s.my) * s.mz * w * w * 2
    if s.arch == "ffno":
        spec = (s.mx + s.my + s.mz) * w * w * 2
    if s.arch in ("hybrid", "ffno"):
        n += s.layers * (spec + 2 * s.ff_hidden * w + s.ff_hidden + w)
    else:
        n += s.layers * (spec + w * w + w)
    n += s.hidden * w + s.hidden + s.cout * s.hidden + s.cout
    return n


def unpack(theta, s: Shape):
    theta = np.asarray(theta, dtype=np.float64)
    w = s.width
    o = 0

    def take(*shape):
        nonlocal o
        k = int(np.prod(shape))
        a = theta[o:o + k].reshape(shape)
        o += k
        return a

    p = {"P": take(w, s.cin), "p": take(w)}
    p["layers"] = []
    for _ in range(s.layers):
        if s.arch == "ffno":
            L = {}
            for a, m in axis_modes(s).items():
                wa = take(m, w, w, 2)
                L["W" + a] = wa[..., 0] + 1j * wa[..., 1]          # [k][c_in][c_out]
            H = s.ff_hidden
            L.update({"W1": take(H, w), "b1": take(H), "W2": take(w, H), "b2": take(w)})
            p["layers"].append(L)
            continue
        ws = take(2 * s.mx, 2 * s.my, s.mz, w, w, 2)
        # complex weights as [c_in][c_out][kx][ky][kz]
        W = (ws[..., 0] + 1j * ws[..., 1]).transpose(3, 4, 0, 1, 2)
        if s.arch == "hybrid":
            H = s.ff_hidden
            p["layers"].append({"W": W, "W1": take(H, w), "b1": take(H), "W2": take(w, H), "b2": take(w)})
        else:
            p["layers"].append({"W": W, "Wp": take(w, w), "bp": take(w)})
    p["Q1"] = take(s.hidden, w)
    p["q1"] = take(s.hidden)
    p["Q2"] = take(s.cout, s.hidden)
    p["q2"] = take(s.cout)
    assert o == theta.size
    return p


def pack(p, s: Shape):
    parts = [p["P"].ravel(), p["p"].ravel()]
    for L in p["layers"]:
        if s.arch == "ffno":
            parts += [np.stack([L["W" + a].real, L["W" + a].imag], -1).ravel() for a, _ in AXES]
            parts += [L["W1"].ravel(), L["b1"].ravel(), L["W2"].ravel(), L["b2"].ravel()]
            continue
        W = L["W"].transpose(2, 3, 4, 0, 1)
        ws = np.stack([W.real, W.imag], -1)
        if s.arch == "hybrid":
            parts += [ws.ravel(), L["W1"].ravel(), L["b1"].ravel(), L["W2"].ravel(), L["b2"].ravel()]
        else:
            parts += [ws.ravel(), L["Wp"].ravel(), L["bp"].ravel()]
    parts += [p["Q1"].ravel(), p["q1"].ravel(), p["Q2"].ravel(), p["q2"].ravel()]
    return np.concatenate(parts)


def mode_indices(m):
    """Retained wavenumbers of a full axis: 0..m-1, -m..-1."""
    return np.concatenate([np.arange(m), np.arange(-m, 0)])


def dft_matrices(s: Shape):
    """Forward truncated DFT matrices: F[k, n] = exp(-2 pi i k n / N)."""
    kx, ky, kz = mode_indices(s.mx), mode_indices(s.my), np.arange(s.mz)
    Fx = np.exp(-2j * np.pi * np.outer(kx, np.arange(s.nx)) / s.nx)
    Fy = np.exp(-2j * np.pi * np.outer(ky, np.arange(s.ny)) / s.ny)
    Fz = np.exp(-2j * np.pi * np.outer(kz, np.arange(s.nz)) / s.nz)
    return Fx, Fy, Fz


def forward_dft(v, mats):
    """V[..., kx, ky, kz] = sum_{x,y,z} v[..., x, y, z] exp(-2 pi i k.n / N),
    the separable sum taken one axis at a time."""
    Fx, Fy, Fz = mats
    t = np.tensordot(v, Fz, axes=([-1], [1]))                        # [..., x, y, kz]
    t = np.moveaxis(np.tensordot(t, Fy, axes=([-2], [1])), -1, -2)   # [..., x, ky, kz]
    t = np.moveaxis(np.tensordot(t, Fx, axes=([-3], [1])), -1, -3)   # [..., kx, ky, kz]
    return t


def inverse_dft(Y, mats, s: Shape):
    """s[..., x, y, z] = (1/(XYZ)) sum_k c_kz Re(Y[..., k] exp(+2 pi i k.n/N)),
    c_0 = 1, c_kz = 2 for kz >= 1."""
    Fx, Fy, Fz = mats
    ckz = np.where(np.arange(s.mz) == 0, 1.0, 2.0)
    t = Y * ckz
    t = np.tensordot(t, np.conj(Fz), axes=([-1], [0]))                       # [..., kx, ky, z]
    t = np.moveaxis(np.tensordot(t, np.conj(Fy), axes=([-2], [0])), -1, -2)  # [..., kx, y, z]
    t = np.moveaxis(np.tensordot(t, np.conj(Fx), axes=([-3], [0])), -1, -3)  # [..., x, y, z]
    return t.real / (s.nx * s.ny * s.nz)


def adjoint_forward_dft(G, mats):
    """Adjoint of forward_dft as a real-linear map (complex gradient G on
    the modes -> real gradient on the grid): Re(sum_k G[k] exp(+i k.n))."""
    Fx, Fy, Fz = mats
    t = np.tensordot(G, np.conj(Fz), axes=([-1], [0]))
    t = np.moveaxis(np.tensordot(t, np.conj(Fy), axes=([-2], [0])), -1, -2)
    t = np.moveaxis(np.tensordot(t, np.conj(Fx), axes=([-3], [0])), -1, -3)
    return t.real


def adjoint_inverse_dft(g, mats, s: Shape):
    """Adjoint of inverse_dft: (c_kz/(XYZ)) times the forward DFT of g."""
    ckz = np.where(np.arange(s.mz) == 0, 1.0, 2.0)
    return forward_dft(g, mats) * ckz / (s.nx * s.ny * s.nz)


def axis_dft(v, axis, m):
    """V[..., k, ...] = sum_n v[..., n, ...] exp(-2 pi i k n / N), k = 0..m-1,
    along one axis (the factorized FNO's per-axis transform)."""
    N = v.shape[axis]
    F = np.exp(-2j * np.pi * np.outer(np.arange(m), np.arange(N)) / N)
    return np.moveaxis(np.tensordot(v, F, axes=([axis], [1])), -1, axis)


def axis_idft(Y, axis, N):
    """c2r inverse along one axis: (1/N) sum_k c_k Re(Y_k exp(+2 pi i k n / N)),
    c_0 = 1, c_k = 2 for k >= 1."""
    m = Y.shape[axis]
    ck = np.where(np.arange(m) == 0, 1.0, 2.0)
    E = np.exp(2j * np.pi * np.outer(np.arange(m), np.arange(N)) / N) * ck[:, None]
    return np.moveaxis(np.tensordot(Y, E, axes=([axis], [0])), -1, axis).real / N


def axis_adjoint_dft(G, axis, N):
    """Adjoint of axis_dft as a real-linear map: Re(sum_k G_k exp(+i theta))."""
    m = G.shape[axis]
    E = np.exp(2j * np.pi * np.outer(np.arange(m), np.arange(N)) / N)
    return np.moveaxis(np.tensordot(G, E, axes=([axis], [0])), -1, axis).real


def axis_adjoint_idft(g, axis, m):
    """Adjoint of axis_idft: (c_k / N) times the forward transform of g."""
    N = g.shape[axis]
    ck = np.where(np.arange(m) == 0, 1.0, 2.0)
    shape = [1] * g.ndim
    shape[axis] = m
    return axis_dft(g, axis, m) * (ck / N).reshape(shape)


def axis_mix(V, W, axis):
    """Y[b, o, .., k, ..] = sum_c V[b, c, .., k, ..] W[k][c][o] (mode along axis)."""
    Vm = np.moveaxis(V, axis, -1)
    return np.moveaxis(np.einsum("bcijk,kco->boijk", Vm, W), -1, axis)


def ffno_spectral(v, L, s: Shape, cache=None):
    """s = sum over the three axes of R_d(W_d . T_d(v)); the per-axis modes
    are kept in cache["Vd"] when a cache list is given."""
    out = np.zeros_like(v)
    modes = axis_modes(s)
    for a, ax in AXES:
        V = axis_dft(v, ax, modes[a])
        if cache is not None:
            cache.append(V)
        out = out + axis_idft(axis_mix(V, L["W" + a], ax), ax, v.shape[ax])
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def proj_act(h, s: Shape):
    """Hidden activation of the projection: GELU, or sin(w0 h) (SIREN)."""
    return np.sin(s.w0 * h) if s.proj == "siren" else gelu(h)


def proj_act_grad(h, s: Shape):
    return s.w0 * np.cos(s.w0 * h) if s.proj == "siren" else gelu_grad(h)


def pointwise(W, v, b=None):
    """(W v)[b, o, ...] = sum_c W[o, c] v[b, c, ...] (+ bias)."""
    out = np.tensordot(W, v, axes=([1], [1]))  # [o, b, ...]
    out = np.moveaxis(out, 0, 1)
    if b is not None:
        out = out + b.reshape((1, -1) + (1,) * (v.ndim - 2))
    return out


def forward(theta, x, s: Shape, mats=None):
    """x [B][cin][X][Y][Z] -> y [B][cout][X][Y][Z] and the saved activations."""
    p = unpack(theta, s)
    mats = mats or dft_matrices(s)
    cache = {"x": x}
    v = pointwise(p["P"], x, p["p"])
    cache["v"] = []
    for li, L in enumerate(p["layers"]):
        cache["v"].append(v)
        if s.arch == "ffno":
            Vd = []
            sc = ffno_spectral(v, L, s, Vd)
            z = pointwise(L["W1"], sc, L["b1"])
            cache.setdefault("Vd", []).append(Vd)
            cache.setdefault("s", []).append(sc)
            cache.setdefault("z", []).append(z)
            v = v + pointwise(L["W2"], gelu(z), L["b2"])
            continue
        V = forward_dft(v, mats)
        Y = np.einsum("bck...,cok...->bok...", V, L["W"])
        cache.setdefault("V", []).append(V)
        if s.arch == "hybrid":
            sc = inverse_dft(Y, mats, s)
            z = pointwise(L["W1"], sc, L["b1"])
            cache.setdefault("s", []).append(sc)
            cache.setdefault("z", []).append(z)
            v = v + pointwise(L["W2"], gelu(z), L["b2"])
            continue
        h = inverse_dft(Y, mats, s) + pointwise(L["Wp"], v, L["bp"])
        cache.setdefault("h", []).append(h)
        v = gelu(h) if li < s.layers - 1 else h
    cache["vL"] = v
    h1 = pointwise(p["Q1"], v, p["q1"])
    cache["h1"] = h1
    y = pointwise(p["Q2"], proj_act(h1, s), p["q2"])
    return y, cache


def masked_mse(y, t, mask):
    """Mean of (y - t)^2 over mask cells, all samples and channels; returns
    the loss and dL/dy."""
    m = np.asarray(mask, dtype=np.float64)[None, None]
    cnt = y.shape[0] * y.shape[1] * m.sum()
    d = (y - t) * m
    return float((d * d).sum() / cnt), 2.0 * d / cnt


def backward(theta, cache, gy, s: Shape, mats=None):
    """Gradient of the loss with respect to the parameter vector, given
    dL/dy, by the chain rule through the saved activations."""
    p = unpack(theta, s)
    mats = mats or dft_matrices(s)
    g = {"layers": [None] * s.layers}
    # projection
    h1 = cache["h1"]
    a = proj_act(h1, s)
    red = tuple(i for i in range(gy.ndim) if i != 1)
    g["Q2"] = np.tensordot(gy, a, axes=(red, red))
    g["q2"] = gy.sum(axis=red)
    ga = pointwise(p["Q2"].T, gy)
    gh1 = ga * proj_act_grad(h1, s)
    vL = cache["vL"]
    g["Q1"] = np.tensordot(gh1, vL, axes=(red, red))
    g["q1"] = gh1.sum(axis=red)
    gv = pointwise(p["Q1"].T, gh1)
    # Fourier layers in reverse
    for li in range(s.layers - 1, -1, -1):
        L = p["layers"][li]
        if s.arch == "ffno":
            z, sc = cache["z"][li], cache["s"][li]
            gL = {"W2": np.tensordot(gv, gelu(z), axes=(red, red)), "b2": gv.sum(axis=red)}
            gz = pointwise(L["W2"].T, gv) * gelu_grad(z)
            gL["W1"] = np.tensordot(gz, sc, axes=(red, red))
            gL["b1"] = gz.sum(axis=red)
            gs = pointwise(L["W1"].T, gz)
            modes = axis_modes(s)
            for (a, ax), V in zip(AXES, cache["Vd"][li]):
                gY = axis_adjoint_idft(gs, ax, modes[a])
                Vm, gYm = np.moveaxis(V, ax, -1), np.moveaxis(gY, ax, -1)
                gL["W" + a] = np.einsum("bcijk,boijk->kco", np.conj(Vm), gYm)
                gV = np.moveaxis(np.einsum("boijk,kco->bcijk", gYm, np.conj(L["W" + a])), -1, ax)
                gv = gv + axis_adjoint_dft(gV, ax, gs.shape[ax])
            g["layers"][li] = gL
            continue
        if s.arch == "hybrid":
            # v' = v + W2 GELU(z) + b2, z = W1 s + b1, s = R(W . T(v))
            z, sc = cache["z"][li], cache["s"][li]
            gL = {"W2": np.tensordot(gv, gelu(z), axes=(red, red)), "b2": gv.sum(axis=red)}
            gz = pointwise(L["W2"].T, gv) * gelu_grad(z)
            gL["W1"] = np.tensordot(gz, sc, axes=(red, red))
            gL["b1"] = gz.sum(axis=red)
            gs = pointwise(L["W1"].T, gz)
            gY = adjoint_inverse_dft(gs, mats, s)
            V = cache["V"][li]
            gL["W"] = np.einsum("bck...,bok...->cok...", np.conj(V), gY)
            gV = np.einsum("bok...,cok...->bck...", gY, np.conj(L["W"]))
            gv = gv + adjoint_forward_dft(gV, mats)
            g["layers"][li] = gL
            continue
        h = cache["h"][li]
        gh = gv * gelu_grad(h) if li < s.layers - 1 else gv
        v = cache["v"][li]
        gL = {}
        gL["Wp"] = np.tensordot(gh, v, axes=(red, red))
        gL["bp"] = gh.sum(axis=red)
        gvp = pointwise(L["Wp"].T, gh)
        gY = adjoint_inverse_dft(gh, mats, s)                 # complex gradient on the modes
        V = cache["V"][li]
        gL["W"] = np.einsum("bck...,bok...->cok...", np.conj(V), gY)
        gV = np.einsum("bok...,cok...->bck...", gY, np.conj(L["W"]))
        gv = gvp + adjoint_forward_dft(gV, mats)
        g["layers"][li] = gL
    x = cache["x"]
    g["P"] = np.tensordot(gv, x, axes=(red, red))
    g["p"] = gv.sum(axis=red)
    return pack(g, s)


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(s: Shape, seed=0):
    """Seeded initial parameters (uniform fan-in scaling; spectral weights
    uniform with scale 1/width^2)."""
    rng = np.random.default_rng(seed)
    w = s.width
    p = {"P": rng.uniform(-1, 1, (w, s.cin)) / math.sqrt(s.cin), "p": np.zeros(w), "layers": []}
    for _ in range(s.layers):
        if s.arch == "ffno":
            H = s.ff_hidden
            L = {"W" + a: (rng.uniform(0, 1, (m, w, w)) + 1j * rng.uniform(0, 1, (m, w, w))) / (w * w)
                 for a, m in axis_modes(s).items()}
            L.update({"W1": rng.uniform(-1, 1, (H, w)) / math.sqrt(w), "b1": np.zeros(H),
                      "W2": rng.uniform(-1, 1, (w, H)) / math.sqrt(H), "b2": np.zeros(w)})
            p["layers"].append(L)
            continue
        W = (rng.uniform(0, 1, (w, w, 2 * s.mx, 2 * s.my, s.mz)) + 1j * rng.uniform(0, 1, (w, w, 2 * s.mx, 2 * s.my, s.mz)))
        if s.arch == "hybrid":
            H = s.ff_hidden
            p["layers"].append({"W": W / (w * w), "W1": rng.uniform(-1, 1, (H, w)) / math.sqrt(w), "b1": np.zeros(H),
                                "W2": rng.uniform(-1, 1, (w, H)) / math.sqrt(H), "b2": np.zeros(w)})
        else:
            p["layers"].append({"W": W / (w * w), "Wp": rng.uniform(-1, 1, (w, w)) / math.sqrt(w),
                                "bp": np.zeros(w)})
    if s.proj == "siren":  # Sitzmann et al.: first layer U(+-1/n), later U(+-sqrt(6/n)/w0)
        p["Q1"] = rng.uniform(-1, 1, (s.hidden, w)) / w
        p["Q2"] = rng.uniform(-1, 1, (s.cout, s.hidden)) * math.sqrt(6.0 / s.hidden) / s.w0
    else:
        p["Q1"] = rng.uniform(-1, 1, (s.hidden, w)) / math.sqrt(w)
        p["Q2"] = rng.uniform(-1, 1, (s.cout, s.hidden)) / math.sqrt(s.hidden)
    p["q1"] = np.zeros(s.hidden)
    p["q2"] = np.zeros(s.cout)
    return pack(p, s)


def inner_box_mask(s: Shape):
    """Loss region of App. A.2 (inner box of the 2x1x1 domain): x in
    [0.1, 0.9) of X (i.e. [0.2, 1.8) of 2L), y and z in [0.25, 0.75)."""
    m = np.zeros((s.nx, s.ny, s.nz), np.uint8)
    m[int(0.1 * s.nx):int(0.9 * s.nx), int(0.25 * s.ny):int(0.75 * s.ny), int(0.25 * s.nz):int(0.75 * s.nz)] = 1
    return m


__all__ = ["Shape", "param_count", "unpack", "pack", "dft_matrices", "forward_dft", "inverse_dft", "forward",
           "backward", "masked_mse", "adam", "init_params", "gelu", "gelu_grad", "proj_act", "proj_act_grad",
           "inner_box_mask", "mode_indices",
           "adjoint_forward_dft", "adjoint_inverse_dft", "axis_dft", "axis_idft", "axis_adjoint_dft",
           "axis_adjoint_idft", "axis_mix", "ffno_spectral", "axis_modes", "AXES"]
