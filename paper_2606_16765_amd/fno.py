"""Python binding of the Fourier-neural-operator part of the C ABI (argument
marshalling only; every contraction, activation, reduction and update runs
in the HIP library).  Device tensors are torch CUDA tensors: inputs BF16
[B][cin][nx][ny][nz], targets and outputs FP32, the loss mask uint8
[nx][ny][nz].
"""
import ctypes
import time

import numpy as np

from ._lib import FnoParams, load


class FnoError(RuntimeError):
    pass


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Fno:
    """3D FNO: lifting, Fourier layers with truncated corner modes, GELU MLP
    projection; trained with masked MSE and Adam.  arch="hybrid" gives the
    hybrid F/FNO: residual layers v + W2 GELU(W1 s + b1) + b2 around the same
    spectral convolution s (feed-forward width ff_hidden); arch="ffno" the
    factorized FNO, the same residual layers with s the sum of 1D spectral
    convolutions along x, y and z (mx, my, mz modes each)."""

    def __init__(self, nx=128, ny=64, nz=64, cin=4, cout=4, width=32, layers=4, mx=16, my=16, mz=16, hidden=128,
                 max_batch=16, seed=0, proj="gelu", w0=30.0, arch="fno", ff_hidden=128):
        L = load()
        p = FnoParams()
        p.nx, p.ny, p.nz, p.cin, p.cout = nx, ny, nz, cin, cout
        p.width, p.layers, p.mx, p.my, p.mz = width, layers, mx, my, mz
        p.proj_hidden, p.max_batch = hidden, max_batch
        p.proj_act = {"gelu": 0, "siren": 1}[proj]
        p.proj_w0 = w0
        p.arch = {"fno": 0, "hybrid": 1, "ffno": 2}[arch]
        p.ff_hidden = ff_hidden
        self.p = p
        self.shape = (nx, ny, nz)
        self._L = L
        self._h = None
        h = ctypes.c_void_p()
        rc = L.fno_create(ctypes.byref(p), ctypes.c_uint64(seed), _stream(), ctypes.byref(h))
        self._check(rc, "fno_create", None)
        self._h = h
        self.nparam = int(L.fno_param_count(ctypes.byref(p)))

    def _check(self, rc, what, h="self"):
        if rc != 0:
            msg = self._L.fno_last_error(self._h if h == "self" else None)
            raise FnoError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def close(self):
        if self._h is not None:
            self._L.fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        a = np.empty(self.nparam, np.float32)
        self._check(self._L.fno_get_params(self._h, ctypes.c_void_p(a.ctypes.data), self.nparam), "fno_get_params")
        return a

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.nparam
        self._check(self._L.fno_set_params(self._h, ctypes.c_void_p(a.ctypes.data), self.nparam), "fno_set_params")

    def forward(self, x, y=None):
        import torch
        assert x.dtype == torch.bfloat16 and x.is_cuda and x.is_contiguous()
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, self.p.cout) + self.shape, dtype=torch.float32, device=x.device)
        self._check(self._L.fno_forward(self._h, ctypes.c_void_p(x.data_ptr()), B, ctypes.c_void_p(y.data_ptr())),
                    "fno_forward")
        return y

    def loss_grad(self, x, target, mask, grads=True):
        B = x.shape[0]
        loss = ctypes.c_float()
        g = np.empty(self.nparam, np.float32) if grads else None
        self._check(self._L.fno_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                          ctypes.c_void_p(mask.data_ptr()), B, ctypes.byref(loss),
                                          None if g is None else ctypes.c_void_p(g.ctypes.data)), "fno_loss_grad")
        return loss.value, g

    def adam_step(self, lr):
        self._check(self._L.fno_adam_step(self._h, ctypes.c_float(lr)), "fno_adam_step")

    def train_step(self, x, target, mask, lr, want_loss=True):
        """One Adam step; returns the loss, or None without want_loss (then
        nothing waits for the device)."""
        loss = ctypes.c_float()
        self._check(self._L.fno_train_step(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                           ctypes.c_void_p(mask.data_ptr()), x.shape[0], ctypes.c_float(lr),
                                           ctypes.byref(loss) if want_loss else None), "fno_train_step")
        return loss.value if want_loss else None


def _fields_check(x):
    import torch
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous() and x.dim() >= 3
    S, C = x.shape[0], x.shape[1]
    return S, C, x[0, 0].numel()


def field_minmax(x):
    """Per-channel (min, max) over samples and points of device float
    x [S][C][...]; returns two numpy arrays."""
    L = load()
    S, C, P = _fields_check(x)
    lo = np.empty(C, np.float32)
    hi = np.empty(C, np.float32)
    rc = L.fno_field_minmax(ctypes.c_void_p(x.data_ptr()), S, C, P, _stream(), ctypes.c_void_p(lo.ctypes.data),
                            ctypes.c_void_p(hi.ctypes.data))
    if rc:
        raise FnoError(f"fno_field_minmax failed ({rc}): {L.fno_last_error(None).decode()}")
    return lo, hi


def field_scale(x, lo, hi, inverse=False):
    """In place: per-channel (x - lo) / (hi - lo), or its inverse."""
    L = load()
    S, C, P = _fields_check(x)
    lo = np.ascontiguousarray(lo, np.float32)
    hi = np.ascontiguousarray(hi, np.float32)
    assert lo.size == C and hi.size == C
    rc = L.fno_field_scale(ctypes.c_void_p(x.data_ptr()), S, C, P, ctypes.c_void_p(lo.ctypes.data),
                           ctypes.c_void_p(hi.ctypes.data), 1 if inverse else 0, _stream())
    if rc:
        raise FnoError(f"fno_field_scale failed ({rc}): {L.fno_last_error(None).decode()}")
    return x


def forward_cost(batch=16, nx=128, ny=64, nz=64, cin=4, cout=4, width=32, layers=4, mx=16, my=16, mz=16,
                 hidden=128):
    """Work of one forward pass, for the roofline of the surrogate.

    flops: the real contractions as the kernels execute them (complex values
    as re/im pairs): per Fourier layer the z, y and x stages of the truncated
    forward DFT, the per-mode complex channel mixing, the inverse x and y
    stages, the c2r stage along z and the pointwise channel map; plus the
    lift and the two-stage projection.  Zero padding of the MFMA tiles is not
    counted.
    min_bytes: the least HBM traffic of any implementation that keeps each
    layer's intermediates on chip: every activation read and written once in
    BF16, the network input (BF16) and output (FP32), and the BF16 spectral
    weights once per pass."""
    P = nx * ny * nz
    MX, MY, MZ = 2 * mx, 2 * my, mz
    M = MX * MY * MZ
    W = width
    per_layer = 2 * (W * nx * ny * nz * 2 * MZ            # z stage (r2c)
                     + W * nx * MZ * 2 * ny * 2 * MY      # y stage
                     + W * MY * MZ * 2 * nx * 2 * MX      # x stage
                     + M * W * W * 4                      # complex mixing
                     + W * MY * MZ * 2 * MX * 2 * nx      # inverse x
                     + W * nx * MZ * 2 * MY * 2 * ny      # inverse y
                     + W * nx * ny * 2 * MZ * nz          # c2r along z
                     + P * W * W)                         # channel map
    flops = batch * (layers * per_layer + 2 * P * cin * W + 2 * P * (W * hidden + hidden * cout))
    act = W * P * 2
    min_bytes = batch * (cin * P * 2 + act + layers * 2 * act + act + cout * P * 4) + layers * W * W * M * 2 * 2
    return {"flops": int(flops), "min_bytes": int(min_bytes)}


def bench_inference(batch=16, reps=10, proj="gelu", arch="fno"):
    """Forward time per batch at the full surrogate shape (128x64x64, width
    32, 4 layers, 32x32x16 retained modes, hidden 128), random input."""
    import torch
    net = Fno(max_batch=batch, proj=proj, arch=arch)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((batch, 4, 128, 64, 64), device="cuda", generator=g).to(torch.bfloat16)
    y = torch.empty((batch, 4, 128, 64, 64), device="cuda")
    net.forward(x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.forward(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    net.close()
    return {"batch": batch, "ms_per_batch": round(ms, 3), "samples_per_s": round(batch / ms * 1e3, 1)}


def bench_train(batch=16, reps=5, arch="fno"):
    """One training step (masked-MSE forward, backward, Adam) per batch at the
    full surrogate shape, random input and target; the paper reports its
    training rate in samples per second."""
    import torch
    net = Fno(max_batch=batch, arch=arch)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((batch, 4, 128, 64, 64), device="cuda", generator=g).to(torch.bfloat16)
    t = torch.rand((batch, 4, 128, 64, 64), device="cuda", generator=g)
    m = torch.zeros((128, 64, 64), dtype=torch.uint8, device="cuda")
    m[12:115, 16:48, 16:48] = 1
    net.train_step(x, t, m, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, t, m, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    net.close()
    return {"batch": batch, "ms_per_step": round(ms, 3), "train_samples_per_s": round(batch / ms * 1e3, 1)}
