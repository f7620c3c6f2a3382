"""Dataset generation, training and evaluation of the FNO surrogate on one
GPU (paper Sec. 2, Sec. 4 and App. A.2).

Pipeline, all device work in this library's kernels:
  1. per seeded obstacle: an LBM run of `steps` steps with averaging over
     the second half (the mean after a settling time), then the mean fields
     pooled factor^3 and turned 0..3 quarter turns about x (App. A.2's
     augmentation) straight into the dataset tensor;
  2. per-field min-max scaling with the training samples' extremes;
  3. training with masked MSE on the inner box, Adam, cosine learning rate;
  4. held-out evaluation (samples of whole simulations never seen in
     training), the gain over the training-set mean field, and the
     time-to-field of the LBM against the surrogate's inference.

Host work is limited to geometry and input-channel generation (inputs/),
which runs while the GPU steps the previous simulation.

    python -m paper_2606_16765_amd.surrogate --sims 128 --out result.json
"""
import argparse
import json
import math
import os
import sys
import time
from dataclasses import asdict, dataclass, field

import numpy as np


@dataclass
class Config:
    shape: tuple = (256, 128, 128)
    factor: int = 2
    sims: int = 128
    held_out: int = 16
    steps: int = 20000
    turns: int = 4
    storage: str = "f32"
    u_in: float = 0.05
    obstacle_bc: int = 1
    epochs: int = 50
    batch: int = 16
    lr: float = 1e-3
    width: int = 32
    layers: int = 4
    modes: tuple = (16, 16, 16)
    hidden: int = 128
    proj: str = "gelu"          # projection hidden activation: "gelu" or "siren" (sine, w0)
    w0: float = 30.0
    also_proj: tuple = ()       # further projections trained and evaluated on the same data
    arch: str = "fno"           # "fno" or "hybrid" (hybrid F/FNO: residual feed-forward layers)
                                # or "ffno" (factorized FNO: per-axis spectral convolutions)
    ff_hidden: int = 128        # hybrid feed-forward width
    also_arch: tuple = ()       # further architectures trained and evaluated on the same data
                                # ("fno", "hybrid", "ffno", or "unet": the 3D U-Net of App. A.2)
    seed: int = 0
    curve_sims: int = 4
    curve_steps: tuple = (1000, 2000, 5000, 10000)
    log_every: int = 1
    extra: dict = field(default_factory=dict)


def log(msg):
    print(f"[surrogate] {msg}", flush=True)


def _event():
    import torch
    return torch.cuda.Event(enable_timing=True)


def inner_mask(X, Y, Z):
    m = np.zeros((X, Y, Z), np.uint8)
    m[int(0.1 * X):int(0.9 * X), int(0.25 * Y):int(0.75 * Y), int(0.25 * Z):int(0.75 * Z)] = 1
    return m


def run_lbm(cfg, seed, steps, out=None, turns=1, geo=None):
    """One LBM run of the seeded obstacle; pooled means (turns 0..turns-1)
    written to out[t] (device float [turns][4][X][Y][Z]).  Returns the
    device time of steps + pooling in ms and the run's status."""
    import torch
    from inputs import random_obstacle
    from .lbm import Lbm, nu_from_re
    nx, ny, nz = cfg.shape
    if geo is None:
        geo = random_obstacle(cfg.shape, seed)
    re = geo.params["re"]
    sim = Lbm(cfg.shape, storage=cfg.storage, u_in=cfg.u_in, nu=nu_from_re(cfg.u_in, ny, re), mode="auto",
              solid=geo.solid, links=geo.links, obstacle_bc=cfg.obstacle_bc, avg_start=steps // 2, force_every=0,
              perturb=(seed, 0.01 * cfg.u_in))
    f = cfg.factor
    if out is None:
        out = torch.empty((turns, 4, nx // f, ny // f, nz // f), dtype=torch.float32, device="cuda")
    e0, e1 = _event(), _event()
    e0.record()
    sim.step(steps)
    for t in range(turns):
        sim.mean_fields_pooled(f, t, out=out[t])
    e1.record()
    return sim, out, (e0, e1), re


def generate(cfg):
    """Dataset tensors on the device: x BF16 [S][4][X][Y][Z], y FP32
    physical pooled means, S = sims * turns; per-simulation timings."""
    import torch
    from inputs import coarse_inputs, random_obstacle, to_bf16_bits
    nx, ny, nz = cfg.shape
    f = cfg.factor
    X, Y, Z = nx // f, ny // f, nz // f
    S = cfg.sims * cfg.turns
    x = torch.empty((S, 4, X, Y, Z), dtype=torch.bfloat16, device="cuda")
    y = torch.empty((S, 4, X, Y, Z), dtype=torch.float32, device="cuda")
    xv = x.view(torch.int16)
    recs = []
    t_start = time.time()
    geo = random_obstacle(cfg.shape, cfg.seed)
    for k in range(cfg.sims):
        seed = cfg.seed + k
        tg = time.time()
        sim, _, (e0, e1), re = run_lbm(cfg, seed, cfg.steps, out=y[k * cfg.turns:(k + 1) * cfg.turns],
                                       turns=cfg.turns, geo=geo)
        # host work while the GPU steps: input channels of this run, geometry of the next
        th = time.time()
        feats = []
        for t in range(cfg.turns):
            a, obj = coarse_inputs(cfg.shape, seed, f, turns=t)
            feats.append(to_bf16_bits(a))
        nxt = random_obstacle(cfg.shape, seed + 1) if k + 1 < cfg.sims else None
        host_s = time.time() - th
        for t in range(cfg.turns):
            xv[k * cfg.turns + t].copy_(torch.from_numpy(feats[t].view(np.int16)))
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        mass = sim.mass()
        ok = bool(np.isfinite(mass))
        sim.close()
        recs.append(dict(seed=seed, re=float(re), aoa=float(obj["aoa"]), n_prims=len(obj["prims"]),
                         kinds=[p_["kind"] for p_ in obj["prims"]], gpu_ms=ms, host_s=host_s, stable=ok,
                         solid_cells=int(geo.n_solid)))
        geo = nxt
        if k % cfg.log_every == 0 or k == cfg.sims - 1:
            log(f"sim {k + 1}/{cfg.sims} seed {seed} Re {re:.0f}: {ms / 1e3:.2f} s GPU "
                f"({cfg.shape[0] * cfg.shape[1] * cfg.shape[2] * cfg.steps / ms / 1e3:.0f} MLUPS), "
                f"host {host_s:.2f} s, stable {ok}, elapsed {time.time() - t_start:.0f} s")
    torch.cuda.synchronize()
    return x, y, recs


def metrics(pred, true, mask):
    """Errors of pred against true (numpy [S][4][X][Y][Z]): relative L2 over
    the whole domain and the inner box (all four fields stacked), per field
    inner-box relative L2, and MSE / max-sample MAE / NRMSE / MAPE over the
    inner box."""
    m = mask.astype(bool)
    d = pred - true
    out = {}
    whole = np.sqrt((d ** 2).sum(axis=(1, 2, 3, 4)) / (true ** 2).sum(axis=(1, 2, 3, 4)))
    di, ti = d[:, :, m], true[:, :, m]
    inner = np.sqrt((di ** 2).sum(axis=(1, 2)) / (ti ** 2).sum(axis=(1, 2)))
    out["rel_l2_whole"] = float(whole.mean())
    out["rel_l2_inner"] = float(inner.mean())
    out["rel_l2_inner_per_field"] = [float(np.sqrt((di[:, c] ** 2).sum() / (ti[:, c] ** 2).sum())) for c in range(4)]
    out["mse_inner"] = float((di ** 2).mean())
    out["max_sample_mae_inner"] = float(np.abs(di).mean(axis=(1, 2)).max())
    rng = ti.max() - ti.min()
    out["nrmse_inner"] = float(np.sqrt((di ** 2).mean()) / rng) if rng > 0 else None
    big = np.abs(ti) > 0.05 * np.abs(ti).max()
    out["mape_inner_pct"] = float(100.0 * (np.abs(di)[big] / np.abs(ti)[big]).mean())
    return out


def train(cfg, net, xs, ys, n_train, mask_d):
    import torch
    steps_per_epoch = n_train // cfg.batch
    total = steps_per_epoch * cfg.epochs
    rng = np.random.default_rng(cfg.seed + 12345)
    xb = torch.empty((cfg.batch,) + tuple(xs.shape[1:]), dtype=xs.dtype, device="cuda")
    yb = torch.empty((cfg.batch,) + tuple(ys.shape[1:]), dtype=ys.dtype, device="cuda")
    hist = []
    e0, e1 = _event(), _event()
    e0.record()
    step = 0
    for ep in range(cfg.epochs):
        perm = torch.from_numpy(rng.permutation(n_train)).to("cuda")
        losses = []
        for b in range(steps_per_epoch):
            idx = perm[b * cfg.batch:(b + 1) * cfg.batch]
            torch.index_select(xs, 0, idx, out=xb)
            torch.index_select(ys, 0, idx, out=yb)
            lr = cfg.lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            # the loss is read back (a device wait) on every 8th step only
            want = b % 8 == 7 or b == steps_per_epoch - 1
            loss = net.train_step(xb, yb, mask_d, lr, want_loss=want)
            if want:
                losses.append(loss)
            step += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{cfg.epochs}: loss {hist[-1]:.3e}")
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    return dict(epochs=cfg.epochs, steps=total, loss_history=hist, train_s=ms / 1e3,
                train_samples_per_s=total * cfg.batch / (ms / 1e3))


def predict(cfg, net, xs, idx, lo, hi):
    """Physical-unit predictions for samples idx (numpy), and the forward
    time per batch of cfg.batch."""
    import torch
    from .fno import field_scale
    xb = torch.empty((cfg.batch,) + tuple(xs.shape[1:]), dtype=xs.dtype, device="cuda")
    yb = torch.empty((cfg.batch, 4) + tuple(xs.shape[2:]), dtype=torch.float32, device="cuda")
    out = []
    times = []
    for b0 in range(0, len(idx), cfg.batch):
        sel = idx[b0:b0 + cfg.batch]
        for j, i in enumerate(sel):
            xb[j].copy_(xs[int(i)])
        B = len(sel)
        e0, e1 = _event(), _event()
        e0.record()
        net.forward(xb[:B], yb[:B])
        field_scale(yb[:B], lo, hi, inverse=True)
        e1.record()
        e1.synchronize()
        times.append((e0.elapsed_time(e1), B))
        out.append(yb[:B].cpu().numpy())
    return np.concatenate(out), times


class FieldModel:
    """Mean fields of a seeded obstacle at a given Reynolds number and angle
    of attack.  Inside the parameter range the network was trained on
    (Re_c in [1000, 10000], |AoA| <= 15 degrees by default) the trained FNO
    answers; outside it the LBM runs the case (the fallback of the gain
    test).  Fields are physical-unit numpy [4][X][Y][Z] (u, v, w, p) on the
    coarse grid."""

    def __init__(self, cfg, net, lo, hi, re_range=(1000.0, 10000.0), aoa_max=15.0):
        self.cfg, self.net, self.lo, self.hi = cfg, net, lo, hi
        self.re_range, self.aoa_max = (float(re_range[0]), float(re_range[1])), float(aoa_max)

    def in_range(self, re, aoa):
        return self.re_range[0] <= float(re) <= self.re_range[1] and abs(float(aoa)) <= self.aoa_max

    def mean_field(self, seed, re=None, aoa=None):
        """(fields, source) with source "fno" or "lbm"; re and aoa default to
        the seeded values."""
        import torch
        from inputs import coarse_inputs, random_obstacle, to_bf16_bits
        from .fno import field_scale
        cfg = self.cfg
        feats, obj = coarse_inputs(cfg.shape, seed, cfg.factor, re=re, aoa=aoa)
        if self.in_range(obj["re"], obj["aoa"]):
            x = torch.from_numpy(to_bf16_bits(feats).view(np.int16)).to("cuda").view(torch.bfloat16)
            y = self.net.forward(x.unsqueeze(0).contiguous())
            field_scale(y, self.lo, self.hi, inverse=True)
            return y[0].cpu().numpy(), "fno"
        geo = random_obstacle(cfg.shape, seed, re=obj["re"], aoa=obj["aoa"])
        sim, out, (_, e1), _ = run_lbm(cfg, seed, cfg.steps, turns=1, geo=geo)
        e1.synchronize()
        sim.close()
        return out[0].cpu().numpy(), "lbm"


def _dump(path, obj):
    if path:
        with open(path, "w") as fh:
            fh.write(json.dumps(obj) + "\n")


def run(cfg, out_path=None):
    import torch
    from .fno import Fno, field_minmax, field_scale
    torch.cuda.set_device(0)
    nx, ny, nz = cfg.shape
    f = cfg.factor
    X, Y, Z = nx // f, ny // f, nz // f
    t0 = time.time()
    log(f"config {asdict(cfg)}")
    xs, yphys, recs = generate(cfg)
    stable = np.array([r["stable"] for r in recs for _ in range(cfg.turns)])
    n_train_sims = cfg.sims - cfg.held_out
    tr = np.arange(n_train_sims * cfg.turns)
    te = np.arange(n_train_sims * cfg.turns, cfg.sims * cfg.turns)
    tr = tr[stable[tr]]
    te = te[stable[te]]
    log(f"dataset: {len(tr)} training and {len(te)} held-out samples ({time.time() - t0:.0f} s)")
    _dump(out_path, dict(partial="dataset", sims=recs))
    # scaling with the training samples' extremes; training copies in place order
    ytr = torch.empty((len(tr),) + tuple(yphys.shape[1:]), dtype=torch.float32, device="cuda")
    xtr = torch.empty((len(tr),) + tuple(xs.shape[1:]), dtype=xs.dtype, device="cuda")
    for j, i in enumerate(tr):
        ytr[j].copy_(yphys[int(i)])
        xtr[j].copy_(xs[int(i)])
    lo, hi = field_minmax(ytr)
    field_scale(ytr, lo, hi)
    mask = inner_mask(X, Y, Z)
    mask_d = torch.from_numpy(mask).cuda()
    mx, my, mz = cfg.modes
    net = Fno(nx=X, ny=Y, nz=Z, width=cfg.width, layers=cfg.layers, mx=mx, my=my, mz=mz, hidden=cfg.hidden,
              max_batch=cfg.batch, seed=cfg.seed, proj=cfg.proj, w0=cfg.w0, arch=cfg.arch, ff_hidden=cfg.ff_hidden)
    tinfo = train(cfg, net, xtr, ytr, len(tr) - len(tr) % cfg.batch if len(tr) >= cfg.batch else len(tr), mask_d)
    log(f"trained: {tinfo['train_s']:.1f} s, {tinfo['train_samples_per_s']:.1f} samples/s")
    _dump(out_path, dict(partial="trained", sims=recs, train=tinfo))
    # held-out evaluation in physical units and in scaled units
    pred, times = predict(cfg, net, xs, te, lo, hi)
    true = np.stack([yphys[int(i)].cpu().numpy() for i in te])
    res_fno = metrics(pred, true, mask)
    sc = lambda a: ((a - lo[None, :, None, None, None]) / (hi - lo)[None, :, None, None, None])
    res_fno_scaled = metrics(sc(pred), sc(true), mask)
    # gain test (i): the training-set mean field as the prediction
    mean_field = np.zeros(true.shape[1:])
    for i in tr:
        mean_field += yphys[int(i)].cpu().numpy()
    mean_field /= len(tr)
    base = np.broadcast_to(mean_field, true.shape)
    res_mean = metrics(base, true, mask)
    res_mean_scaled = metrics(sc(base), sc(true), mask)
    fwd_ms = sum(t for t, _ in times) / sum(b for _, b in times)
    full = [t / b for t, b in times if b == cfg.batch]
    log(f"held-out rel L2 inner: FNO {res_fno['rel_l2_inner']:.4f} vs mean field {res_mean['rel_l2_inner']:.4f}")
    variants, arch_variants = {}, {}
    specs = [("proj", v, dict(proj=v, arch=cfg.arch)) for v in cfg.also_proj]
    specs += [("arch", v, dict(proj=cfg.proj, arch=v)) for v in cfg.also_arch]
    for kind, name, kw in specs:
        # the same data, scaling, seed and schedule with another projection
        # or architecture
        if kw["arch"] == "unet":
            from .unet import Unet
            vnet = Unet(nx=X, ny=Y, nz=Z, max_batch=cfg.batch, seed=cfg.seed)
        else:
            vnet = Fno(nx=X, ny=Y, nz=Z, width=cfg.width, layers=cfg.layers, mx=mx, my=my, mz=mz,
                       hidden=cfg.hidden, max_batch=cfg.batch, seed=cfg.seed, w0=cfg.w0, ff_hidden=cfg.ff_hidden,
                       **kw)
        vinfo = train(cfg, vnet, xtr, ytr, len(tr) - len(tr) % cfg.batch if len(tr) >= cfg.batch else len(tr), mask_d)
        vpred, vtimes = predict(cfg, vnet, xs, te, lo, hi)
        vnet.close()
        row = dict(held_out=metrics(vpred, true, mask), held_out_scaled=metrics(sc(vpred), sc(true), mask),
                   train_samples_per_s=vinfo["train_samples_per_s"], train_s=vinfo["train_s"],
                   loss_history=vinfo["loss_history"],
                   forward_ms_per_sample=sum(t for t, _ in vtimes) / sum(b for _, b in vtimes))
        (variants if kind == "proj" else arch_variants)[name] = row
        log(f"{'projection' if kind == 'proj' else 'architecture'} {name}: held-out rel L2 inner "
            f"{row['held_out']['rel_l2_inner']:.4f}, {row['train_samples_per_s']:.1f} training samples/s")
    # gain test (ii) and time-to-field: shorter LBM runs of held-out obstacles
    curve = []
    held_seeds = [r["seed"] for r in recs[n_train_sims:] if r["stable"]][:cfg.curve_sims]
    for seed in held_seeds:
        k = seed - cfg.seed
        ref = yphys[k * cfg.turns].cpu().numpy()[None]
        for T in cfg.curve_steps:
            sim, out, (e0, e1), _ = run_lbm(cfg, seed, T, turns=1)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            sim.close()
            err = metrics(out.cpu().numpy(), ref, mask)
            curve.append(dict(seed=seed, steps=T, gpu_ms=ms, rel_l2_inner=err["rel_l2_inner"],
                              rel_l2_whole=err["rel_l2_whole"]))
            log(f"lbm curve seed {seed} steps {T}: {ms:.0f} ms, rel L2 inner {err['rel_l2_inner']:.4f}")
    lbm_ms = float(np.mean([r["gpu_ms"] for r in recs if r["stable"]]))
    per_steps = {}
    for c in curve:
        per_steps.setdefault(c["steps"], []).append(c)
    curve_summary = [dict(steps=T, gpu_ms=float(np.mean([c["gpu_ms"] for c in v])),
                          rel_l2_inner=float(np.mean([c["rel_l2_inner"] for c in v])))
                     for T, v in sorted(per_steps.items())]
    reach = [c for c in curve_summary if c["rel_l2_inner"] <= res_fno["rel_l2_inner"]]
    result = dict(
        config=dict(asdict(cfg), shape=list(cfg.shape), modes=list(cfg.modes), coarse=[X, Y, Z],
                    n_train=int(len(tr)), n_held_out=int(len(te)), unstable_sims=int(sum(not r["stable"] for r in recs))),
        fno=dict(held_out=res_fno, held_out_scaled=res_fno_scaled, forward_ms_per_sample=fwd_ms,
                 forward_ms_per_batch=float(np.mean(full)) * cfg.batch if full else None, **tinfo),
        mean_field_baseline=dict(held_out=res_mean, held_out_scaled=res_mean_scaled),
        projection_variants=variants,
        architecture_variants=arch_variants,
        gain=dict(rel_l2_inner_ratio_mean_over_fno=res_mean["rel_l2_inner"] / res_fno["rel_l2_inner"],
                  rel_l2_whole_ratio_mean_over_fno=res_mean["rel_l2_whole"] / res_fno["rel_l2_whole"]),
        time_to_field=dict(
            lbm_ms_per_field=lbm_ms, lbm_steps=cfg.steps, fno_ms_per_field=fwd_ms,
            speedup=lbm_ms / fwd_ms,
            lbm_curve=curve_summary,
            lbm_min_ms_to_fno_error=(reach[0]["gpu_ms"] if reach else None),
            note="GPU time only: LBM steps + pooling vs FNO forward + unscaling, per field; host geometry "
                 "generation excluded from both"),
        sims=recs,
        wall_s=time.time() - t0,
    )
    net.close()
    return result


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sims", type=int, default=128)
    ap.add_argument("--held-out", type=int, default=16)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--shape", type=int, nargs=3, default=[256, 128, 128])
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, nargs=3, default=[16, 16, 16])
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--proj", choices=["gelu", "siren"], default="gelu")
    ap.add_argument("--w0", type=float, default=30.0)
    ap.add_argument("--also-proj", choices=["gelu", "siren"], nargs="*", default=[],
                    help="also train and evaluate networks with these projections on the same data")
    ap.add_argument("--arch", choices=["fno", "hybrid"], default="fno")
    ap.add_argument("--ff-hidden", type=int, default=128)
    ap.add_argument("--also-arch", choices=["fno", "hybrid", "ffno", "unet"], nargs="*", default=[],
                    help="also train and evaluate these architectures on the same data")
    ap.add_argument("--curve-sims", type=int, default=4)
    ap.add_argument("--curve-steps", type=int, nargs="*", default=[1000, 2000, 5000, 10000])
    ap.add_argument("--log-every", type=int, default=1)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    cfg = Config(shape=tuple(a.shape), sims=a.sims, held_out=a.held_out, steps=a.steps, epochs=a.epochs,
                 batch=a.batch, lr=a.lr, width=a.width, modes=tuple(a.modes), hidden=a.hidden, layers=a.layers,
                 proj=a.proj, w0=a.w0, also_proj=tuple(a.also_proj), arch=a.arch, ff_hidden=a.ff_hidden,
                 also_arch=tuple(a.also_arch),
                 curve_sims=a.curve_sims, curve_steps=tuple(a.curve_steps), log_every=a.log_every)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    res = run(cfg, a.out)
    _dump(a.out, res)
    summ = dict(fno=res["fno"]["held_out"]["rel_l2_inner"], mean=res["mean_field_baseline"]["held_out"]["rel_l2_inner"],
                lbm_ms=res["time_to_field"]["lbm_ms_per_field"], fno_ms=res["time_to_field"]["fno_ms_per_field"])
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
