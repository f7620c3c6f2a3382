"""Storage-precision study of the stream-collide path (FP32 populations and
shifted FP16/BF16 populations with FP32 arithmetic, FP64 means).

error_table: the seeded random obstacle of the 256x128x128 generator scaled
to a channel of the given size, run at several Re with FP64, FP32, FP16 and
BF16 storage; the mean fields over the second half of the run are compared
with a reference: the FP64 CPU oracle's means of the same configuration where
the caller passes them (the laminar Re 1000 case), else this library's FP64
run (which agrees with the oracle to 1e-11 at every size the parity tests
cover).  Two noise floors bound what any arithmetic can reach once the flow
is chaotic: a second FP64 run whose initial populations are rounded to FP32
(a perturbation of FP32 rounding size), and one whose initial perturbation
amplitude differs by a relative 1e-10.

throughput: MLUPS and the stream-collide kernel's HBM rate per storage type
on a larger channel, from the library's own per-launch event timing.
"""
import numpy as np

from .lbm import Lbm, bytes_per_cell_update, nu_from_re

HBM_PEAK_GBS = 8000.0


def _run(geo, re, storage, steps, amp, u_in=0.05, round_f32=False):
    nx, ny, nz = geo.shape
    sim = Lbm(geo.shape, storage=storage, u_in=u_in, re=re, mode="auto", solid=geo.solid,
              links=geo.links, obstacle_bc=1, avg_start=steps // 2, force_every=0, perturb=(0, amp))
    if round_f32:
        # the initial state with every population rounded to FP32
        sim.set_populations(sim.populations().astype(np.float32).astype(np.float64))
    sim.step(steps)
    m, n = sim.mean_fields()
    mass = sim.mass()
    sim.close()
    return m, mass


def _errors(m, ref, fluid):
    U = m[:3, fluid]
    R = ref[:3, fluid]
    out = {"e_vel": float(np.linalg.norm(U - R) / np.linalg.norm(R))}
    for k, name in enumerate("uvwp"):
        r = ref[k, fluid]
        out["e_" + name] = float(np.linalg.norm(m[k, fluid] - r) / np.linalg.norm(r))
    return out


def error_table(shape=(128, 64, 64), res=(1000.0, 5000.0, 10000.0), steps=10000, seed=0, log=print,
                oracle_means=None):
    """oracle_means: {re: [4][nz][ny][nx] mean fields of the FP64 oracle for
    this configuration}; those Re are measured against the oracle (the FP64
    storage run of this library is then one more row), the others against
    the library's FP64 run."""
    from inputs import random_obstacle
    geo = random_obstacle(shape, seed)
    fluid = geo.solid.reshape(-1) == 0
    amp = 0.01 * 0.05
    oracle_means = oracle_means or {}
    rows = []
    for re in res:
        f64, _ = _run(geo, re, "f64", steps, amp)
        f64 = f64.reshape(4, -1)
        row = {"re": re, "mode": "k17" if 0.05 * shape[1] / nu_from_re(0.05, shape[1], re) >= 3000 else "plain"}
        if re in oracle_means:
            ref = np.asarray(oracle_means[re], dtype=np.float64).reshape(4, -1)
            row["reference"] = "FP64 CPU oracle (means stored in float32)"
            row["f64"] = _errors(f64, ref, fluid)
        else:
            ref = f64
            row["reference"] = "FP64 storage run of this library"
        rf, _ = _run(geo, re, "f64", steps, amp, round_f32=True)
        row["noise_floor_f32_rounded_start"] = _errors(rf.reshape(4, -1), f64, fluid)
        noise, _ = _run(geo, re, "f64", steps, amp * (1.0 + 1e-10))
        row["noise_floor_f64"] = _errors(noise.reshape(4, -1), f64, fluid)
        for st in ("f32", "f16", "bf16"):
            m, mass = _run(geo, re, st, steps, amp)
            row[st] = _errors(m.reshape(4, -1), ref, fluid)
            row[st]["mass"] = float(mass)
        rows.append(row)
        log(f"precision Re {re:.0f} vs {row['reference']}: e_vel f32 {row['f32']['e_vel']:.2e} "
            f"f16 {row['f16']['e_vel']:.2e} bf16 {row['bf16']['e_vel']:.2e} floor (FP32-rounded start) "
            f"{row['noise_floor_f32_rounded_start']['e_vel']:.2e}")
    return dict(shape=list(shape), steps=steps, window=[steps // 2, steps], obstacle_seed=seed, rows=rows,
                reference="per row: the FP64 CPU oracle where given, else this library's FP64 run",
                noise_floors="FP64 runs from the initial populations rounded to FP32, and from a 1e-10 "
                             "relative change of the perturbation amplitude, against the FP64 run")


def throughput(shape=(512, 256, 256), storages=("f32", "f16", "bf16"), steps=400, warmup=20, seed=0, re=5500.0,
               log=print):
    import torch
    from inputs import random_obstacle
    geo = random_obstacle(shape, seed)
    N = shape[0] * shape[1] * shape[2]
    out = []
    for st in storages:
        sim = Lbm(shape, storage=st, u_in=0.05, nu=nu_from_re(0.05, shape[1], re), mode="auto", solid=geo.solid,
                  links=geo.links, obstacle_bc=1, avg_start=None, force_every=1, perturb=(seed, 0.0005))
        sim.step(warmup)
        torch.cuda.synchronize()
        sim.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        kms, launches = sim.profile_read()
        sim.close()
        bpc = bytes_per_cell_update(st, averaging=False)
        bytes_launch = (N - geo.n_solid) * (bpc - 1) + N
        gbs = bytes_launch / (kms / launches / 1e3) / 1e9
        rec = dict(storage=st, mlups=N * steps / (ms / 1e3) / 1e6, kernel_ms=kms / launches,
                   bytes_per_cell_update=bpc, achieved_gbs=gbs, frac=gbs / HBM_PEAK_GBS)
        out.append(rec)
        log(f"throughput {st} {shape}: {rec['mlups']:.0f} MLUPS, kernel {rec['kernel_ms']:.3f} ms, {gbs:.0f} GB/s")
    return dict(shape=list(shape), steps=steps, re=re, obstacle_seed=seed, rows=out)
