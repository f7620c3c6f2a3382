"""Python binding of the 3D U-Net part of the C ABI (argument marshalling
only; every convolution, normalisation, pooling, upsampling, reduction and
update runs in the HIP library).  Device tensors are torch CUDA tensors:
inputs BF16 [B][cin][nx][ny][nz], targets and outputs FP32, the loss mask
uint8 [nx][ny][nz] -- the same interface as the Fourier operator.
"""
import ctypes
import time

import numpy as np

from ._lib import UnetParams, load


class UnetError(RuntimeError):
    pass


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Unet:
    """3D U-Net of App. A.2: encoder widths (32, 64, 128, 256) with two
    conv-BN-ReLU blocks per stage and max pooling, bottleneck 512, decoder
    with trilinear upsampling and skip concatenation, 1x1x1 sigmoid head."""

    def __init__(self, nx=128, ny=64, nz=64, cin=4, cout=4, widths=(32, 64, 128, 256), bottleneck=512,
                 max_batch=16, seed=0):
        L = load()
        p = UnetParams()
        p.nx, p.ny, p.nz, p.cin, p.cout = nx, ny, nz, cin, cout
        for i in range(4):
            p.widths[i] = int(widths[i])
        p.bottleneck, p.max_batch = int(bottleneck), int(max_batch)
        self.p = p
        self.shape = (nx, ny, nz)
        self.widths = tuple(int(w) for w in widths)
        self.bottleneck = int(bottleneck)
        self._L = L
        self._h = None
        h = ctypes.c_void_p()
        rc = L.unet_create(ctypes.byref(p), ctypes.c_uint64(seed), _stream(), ctypes.byref(h))
        self._check(rc, "unet_create", None)
        self._h = h
        self.nparam = int(L.unet_param_count(ctypes.byref(p)))
        # batch-norm channels: two blocks per encoder and decoder stage, two in the bottleneck
        self.nbn = 4 * sum(self.widths) + 2 * self.bottleneck

    def _check(self, rc, what, h="self"):
        if rc != 0:
            msg = self._L.unet_last_error(self._h if h == "self" else None)
            raise UnetError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def close(self):
        if self._h is not None:
            self._L.unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        a = np.empty(self.nparam, np.float32)
        self._check(self._L.unet_get_params(self._h, ctypes.c_void_p(a.ctypes.data), self.nparam), "unet_get_params")
        return a

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.nparam
        self._check(self._L.unet_set_params(self._h, ctypes.c_void_p(a.ctypes.data), self.nparam), "unet_set_params")

    def bn_stats(self):
        """Running (means, variances) of every batch-norm layer, block order."""
        a = np.empty(2 * self.nbn, np.float32)
        self._check(self._L.unet_bn_stats(self._h, ctypes.c_void_p(a.ctypes.data), a.size), "unet_bn_stats")
        return a[: self.nbn], a[self.nbn:]

    def forward(self, x, y=None, training=False):
        import torch
        assert x.dtype == torch.bfloat16 and x.is_cuda and x.is_contiguous()
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, self.p.cout) + self.shape, dtype=torch.float32, device=x.device)
        self._check(self._L.unet_forward(self._h, ctypes.c_void_p(x.data_ptr()), B, 1 if training else 0,
                                         ctypes.c_void_p(y.data_ptr())), "unet_forward")
        return y

    def loss_grad(self, x, target, mask, grads=True):
        B = x.shape[0]
        loss = ctypes.c_float()
        g = np.empty(self.nparam, np.float32) if grads else None
        self._check(self._L.unet_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                           ctypes.c_void_p(mask.data_ptr()), B, ctypes.byref(loss),
                                           None if g is None else ctypes.c_void_p(g.ctypes.data)), "unet_loss_grad")
        return loss.value, g

    def adam_step(self, lr):
        self._check(self._L.unet_adam_step(self._h, ctypes.c_float(lr)), "unet_adam_step")

    def train_step(self, x, target, mask, lr, want_loss=True):
        """One Adam step; returns the loss, or None without want_loss (then
        nothing waits for the device)."""
        loss = ctypes.c_float()
        self._check(self._L.unet_train_step(self._h, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                            x.shape[0], ctypes.c_float(lr),
                                            ctypes.byref(loss) if want_loss else None), "unet_train_step")
        return loss.value if want_loss else None


def forward_flops(nx=128, ny=64, nz=64, cin=4, cout=4, widths=(32, 64, 128, 256), bottleneck=512, batch=16):
    """Multiply-add FLOPs of one forward pass (the 27-tap convolutions at
    their real input widths and the head)."""
    f = 0
    c = cin
    P = nx * ny * nz
    for l, w in enumerate(widths):
        v = P >> (3 * l)
        f += 2 * 27 * v * (c * w + w * w)
        c = w
    vb = P >> 12
    f += 2 * 27 * vb * (c * bottleneck + bottleneck * bottleneck)
    c = bottleneck
    for l in reversed(range(len(widths))):
        w = widths[l]
        v = P >> (3 * l)
        f += 2 * 27 * v * ((c + w) * w + w * w)
        c = w
    f += 2 * P * widths[0] * cout
    return batch * f


def bench_inference(batch=16, reps=10):
    """Forward time per batch at the full surrogate shape (128x64x64, App.
    A.2 widths), evaluation mode."""
    import torch
    net = Unet(max_batch=batch)
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
    fl = forward_flops(batch=batch)
    return {"batch": batch, "ms_per_batch": round(ms, 3), "samples_per_s": round(batch / ms * 1e3, 1),
            "tflops": round(fl / (ms / 1e3) / 1e12, 1)}


def bench_train(batch=16, reps=5):
    """One training step (forward, masked MSE, backward, Adam) per batch at
    the full surrogate shape."""
    import torch
    net = Unet(max_batch=batch)
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
