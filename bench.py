"""Benchmark of the hot path on one MI355X.

Workload (default "c2"): the paper-scale channel, 1024 x 512 x 512 cells, a
spanwise cylinder of diameter 64 at x = 307.2, Re_D = 3900 at u_in = 0.05,
FP32 populations, fourth-order parametrised cumulant mode (Re_c on the
channel height is 31200 >= 3000), seeded 1% perturbation, drag and lift
recorded in FP64 every step, averaging off.  A step is one fused
stream-and-collide launch plus the force reduction.

Prints one JSON line: MLUPS (million lattice-cell updates per second) for
the whole job; the roofline of the stream-collide kernel (algorithmic bytes
per launch over its event-timed duration, against 8 TB/s, next to a
same-pattern probe and a plain copy); the 256x128x128 dataset configuration
with the running mean on; the Fourier neural operator's forward time per
batch of 16 with its MFMA and HBM rates, and its training step; the storage
precision study; and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("lbm.hip", "lbm_device.h"):
        with open(os.path.join(ROOT, "paper_2606_16765_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload):
    """HBM traffic per launch measured with rocprofv3 counters for the
    current kernel source (profiles/lbm_step_<workload>_traffic.txt), or
    None when absent or taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", f"lbm_step_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_surrogate_result():
    """Summary of the full surrogate pipeline runs (dataset of LBM runs,
    training, held-out errors, time-to-field), committed under profiles/ by
    the runs that produced them; None when absent.  Both runs use the same
    seeds, hence the same LBM fields: the first trains the FNO with both
    projections and the hybrid, the second the FNO, the U-Net and the
    factorized FNO."""
    files = ("fno_surrogate_c4.json", "surrogate_c4_nets.json")
    keep = None
    for name in files:
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            r = json.load(fh)
        if keep is None:
            keep = {k: r[k] for k in ("config", "gain", "time_to_field") if k in r}
            if "fno" in r:
                keep["fno_held_out"] = r["fno"].get("held_out")
                keep["fno_train_samples_per_s"] = r["fno"].get("train_samples_per_s")
            if "mean_field_baseline" in r:
                keep["mean_field_held_out"] = r["mean_field_baseline"].get("held_out")
            keep["source"] = []
        for proj, v in r.get("projection_variants", {}).items():
            keep[f"fno_{proj}_projection_held_out"] = v.get("held_out")
        for arch, v in r.get("architecture_variants", {}).items():
            keep[f"{arch}_held_out"] = v.get("held_out")
            keep[f"{arch}_train_samples_per_s"] = v.get("train_samples_per_s")
        keep["source"].append(f"profiles/{name} (python -m paper_2606_16765_amd.surrogate)")
    return keep


def read_validation_result():
    """Sphere drag against the paper's Table 1 and the cylinder's Strouhal
    number from the committed validation runs (profiles/validation_*.json);
    None when absent."""
    out = {}
    for name in ("validation_sphere_periodic", "validation_sphere_walls", "validation_sphere_periodic_l384",
                 "validation_c2_cylinder"):
        path = os.path.join(ROOT, "profiles", name + ".json")
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            r = json.load(fh)
        key = "sphere_periodic" if "periodic" in name else "sphere"
        rows = []
        for blk in r.get(key, []):
            for row in blk["rows"]:
                rows.append({"L": blk["resolution"], "re_s": row["re_s"], "cd": round(row["cd"], 4),
                             "cd_paper": row["cd_paper"]})
        out.setdefault(key, []).extend(rows)
        if "cylinder" in r:
            cy = r["cylinder"]
            out.setdefault("cylinder", []).append({"shape": cy["shape"], "steps": cy["steps"],
                                                   "strouhal": round(cy["strouhal"], 4), "cd": round(cy["cd"], 4)})
    if not out:
        return None
    out["source"] = "profiles/validation_*.json (python -m paper_2606_16765_amd.validation)"
    return out


WORKLOADS = {
    # name: (shape, storage, description)
    "c2": ((1024, 512, 512), "f32", "cylinder D=64, Re_D=3900, K17, FP32, 1024x512x512"),
    "c1": ((256, 128, 128), "f32", "random obstacle seed 0, FP32 with running mean, 256x128x128"),
    "c3-f16": ((512, 256, 256), "f16", "random obstacle seed 0, FP16 shifted storage, 512x256x256"),
    "c3-bf16": ((512, 256, 256), "bf16", "random obstacle seed 0, BF16 shifted storage, 512x256x256"),
}


def make_workload(name):
    from inputs import random_obstacle, spanwise_cylinder
    import paper_2606_16765_amd as P
    shape, storage, desc = WORKLOADS[name]
    if name == "c2":
        geo = spanwise_cylinder(shape, center=(307.2, 255.5), diameter=64.0)
        nu = P.nu_from_re(0.05, 64.0, 3900.0)
        kw = dict(avg_start=None, force_every=1)
        char_len, area = 64.0, 64.0 * shape[2]
    else:
        geo = random_obstacle(shape, 0)
        re = 1000.0 + 9000.0 * 0.5
        nu = P.nu_from_re(0.05, shape[1], re)
        kw = dict(avg_start=0, force_every=1, snap_every=25, snap_count=20) if name == "c1" else \
            dict(avg_start=0, force_every=1)
        char_len, area = None, geo.frontal_area
    return geo, nu, storage, kw, desc, char_len, area


def run_lbm(name, steps, warmup, probe=True):
    import numpy as np
    import torch
    import paper_2606_16765_amd as P

    t0 = time.time()
    geo, nu, storage, kw, desc, char_len, area = make_workload(name)
    log(f"geometry {geo.name} {geo.shape}: {geo.n_solid} solid cells, {len(geo.links[0])} links "
        f"({time.time() - t0:.1f} s)")
    sim = P.Lbm(geo.shape, storage=storage, u_in=0.05, nu=nu, mode="auto", solid=geo.solid, links=geo.links,
                obstacle_bc=1,
                perturb=(0, 0.01 * 0.05), **kw)
    info = sim.info()
    log(f"created: omega1={info['omega1']:.6f} mode={'k17' if info['mode'] else 'plain'}")
    N = geo.shape[0] * geo.shape[1] * geo.shape[2]
    n_solid = geo.n_solid
    del geo
    sim.step(warmup)
    torch.cuda.synchronize()
    log(f"warmup {warmup} steps done")
    sim.profile(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    # chunks keep progress lines flowing during a long timed region
    done = 0
    chunk = max(1, steps // 5)
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        if done < steps:
            log(f"enqueued {done}/{steps} steps")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    kern_ms, launches = sim.profile_read()
    sim.profile(False)
    # same memory traffic without the collision: the attainable rate of this
    # access pattern on this device
    probe_ms = sim.bandwidth_probe(20) if probe else float("nan")
    mass = sim.mass()
    forces, fsteps = sim.forces()
    sim.close()
    mlups = N * steps / elapsed / 1e6
    avg_kernel_s = kern_ms / launches / 1e3
    bpc = P.bytes_per_cell_update(storage, averaging=kw.get("avg_start") is not None)
    # solid cells read only their flag byte
    bytes_per_launch = (N - n_solid) * (bpc - 1) + N * 1
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    log(f"timed {steps} steps in {elapsed:.3f} s: {mlups:.1f} MLUPS; kernel avg {avg_kernel_s * 1e3:.3f} ms "
        f"-> {achieved:.0f} GB/s")
    esize = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
    probe_gbs = N * 2 * 27 * esize / (probe_ms / 1e3) / 1e9
    if probe:
        log(f"same-pattern probe (no collision): {probe_ms:.3f} ms per pass -> {probe_gbs:.0f} GB/s")
    out = dict(mlups=mlups, elapsed=elapsed, N=N, n_solid=n_solid, desc=desc, storage=storage,
               probe_ms=probe_ms, probe_gbs=probe_gbs,
               kernel_ms=avg_kernel_s * 1e3, bytes_per_launch=bytes_per_launch, achieved=achieved,
               bytes_per_cell=bpc, mass=mass, launches=launches)
    if len(forces):
        half = forces[len(forces) // 2:]
        u = 0.05
        out["cd"] = float(2.0 * half[:, 0].mean() / (u * u * area))
        out["cl_rms"] = float(2.0 * np.sqrt((half[:, 1] ** 2).mean()) / (u * u * area))
    return out


def copy_rate(reps=10):
    """Rate of the library's plain streaming copy of 4 GiB (one 16-byte
    vector per lane, non-temporal stores), the attainable bandwidth of a
    streaming kernel on this device."""
    from paper_2606_16765_amd.lbm import copy_bandwidth
    return copy_bandwidth(4 * 2 ** 30, reps)


def torch_copy_rate(reps=10):
    """Rate of a plain 4 GiB device-to-device copy with torch's copy kernel,
    for comparison."""
    import torch
    a = torch.empty(2 ** 30, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * 2 ** 30 / dt / 1e9


def fno_leg():
    """FNO forward and training step at batch 16 on the full surrogate shape,
    with the forward pass's MFMA and HBM rates."""
    from paper_2606_16765_amd import fno as pfno
    out = pfno.bench_inference(batch=16, reps=20)
    out["train"] = pfno.bench_train(batch=16)
    out["siren_projection"] = pfno.bench_inference(batch=16, reps=20, proj="siren")
    # the hybrid F/FNO (residual feed-forward layers, width 32 -> 128 -> 32)
    out["hybrid"] = pfno.bench_inference(batch=16, reps=20, arch="hybrid")
    out["hybrid"]["train"] = pfno.bench_train(batch=16, arch="hybrid")
    # the factorized FNO (per-axis spectral convolutions, 16 modes per axis)
    out["ffno"] = pfno.bench_inference(batch=16, reps=20, arch="ffno")
    out["ffno"]["train"] = pfno.bench_train(batch=16, arch="ffno")
    # the 3D U-Net of App. A.2 (implicit-GEMM convolutions on BF16 MFMA)
    from paper_2606_16765_amd import unet as punet
    u = punet.bench_inference(batch=16, reps=10)
    u["frac_mfma"] = round(u["tflops"] / MFMA_BF16_PEAK_TFLOPS, 4)
    u["train"] = punet.bench_train(batch=16, reps=5)
    out["unet"] = u
    cost = pfno.forward_cost(batch=16)
    s = out["ms_per_batch"] / 1e3
    out["roofline"] = {
        "flops_per_batch": cost["flops"], "tflops": round(cost["flops"] / s / 1e12, 2),
        "mfma_bf16_peak_tflops": MFMA_BF16_PEAK_TFLOPS,
        "frac_mfma": round(cost["flops"] / s / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4),
        "min_bytes_per_batch": cost["min_bytes"], "gbs_at_min_bytes": round(cost["min_bytes"] / s / 1e9, 1),
        "frac_hbm_at_min_bytes": round(cost["min_bytes"] / s / 1e9 / HBM_PEAK_GBS, 4),
        "note": "flops: the real contractions as executed; min_bytes: BF16 activations read and written once per "
                "layer, input, output and spectral weights once",
    }
    return out


def fno_cpu_baseline():
    """The FP64 numpy oracle of the FNO, as it stands: one forward pass at
    batch 1 on the full surrogate shape, on this host's cores (threaded
    BLAS)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import fno as ofno
    s = ofno.Shape()
    th = ofno.init_params(s, 0)
    x = np.random.default_rng(0).standard_normal((1, s.cin, s.nx, s.ny, s.nz))
    mats = ofno.dft_matrices(s)
    t = time.perf_counter()
    ofno.forward(th, x, s, mats)
    dt = time.perf_counter() - t
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return dict(value=1.0 / dt, unit="samples/s", cores=threads, kind="oracle",
                sample=f"one FP64 forward pass at batch 1, 128x64x64, width 32, 4 layers, 32x32x16 modes: {dt:.1f} s")


def precision_oracle_means():
    """The FP64 CPU oracle's mean fields of the precision study's laminar
    case (Re 1000, 128x64x64, 10,000 steps), written by
    tests/golden/make_precision_reference.py; {} when absent."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "precision_ref_re1000.npz")
    if not os.path.exists(path):
        return {}
    d = np.load(path)
    return {float(d["re"]): d["means"]}


def c1_leg(steps=2000, warmup=50):
    """The dataset configuration (256x128x128, FP32, random obstacle seed 0,
    Re_c 5500) with the FP64 running mean and snapshots on, as every dataset
    run executes it: MLUPS and the step kernel's rate at 281 B per cell."""
    r = run_lbm("c1", steps, warmup, probe=False)
    return {"workload": r["desc"], "steps": steps, "mlups": round(r["mlups"], 1),
            "kernel_ms": round(r["kernel_ms"], 4), "bytes_per_cell_update": r["bytes_per_cell"],
            "achieved_gbs": round(r["achieved"], 1), "frac": round(r["achieved"] / HBM_PEAK_GBS, 4)}


def cpu_baseline(name, budget_s=15.0, one_core=False):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    the same configuration at 128 x 64 x 64 (geometry scaled by 1/8), timed
    on this host's cores."""
    from inputs import random_obstacle, spanwise_cylinder
    from oracle import lbm as olbm
    shape = (128, 64, 64)
    if name == "c2":
        geo = spanwise_cylinder(shape, center=(38.4, 31.5), diameter=8.0)
        nu = 0.05 * 8.0 / 3900.0
        mode = 1
    else:
        geo = random_obstacle(shape, 0)
        nu = 0.05 * 64 / 5500.0
        mode = 1
    p = olbm.make_params(shape, nu=nu, u_in=0.05, mode=mode, avg_start=10 ** 9)
    r = olbm.Run(p, solid=geo.solid)
    t = time.perf_counter()
    r.step(2)
    probe = time.perf_counter() - t
    n = max(2, int(budget_s / max(probe / 2, 1e-3)))
    t = time.perf_counter()
    r.step(n)
    dt = time.perf_counter() - t
    N = shape[0] * shape[1] * shape[2]
    out = dict(value=N * n / dt / 1e6, unit="MLUPS", cores=olbm.threads(), kind="oracle",
               sample=f"{name} configuration at 128x64x64 (geometry scaled 1/8), FP64 oracle, {n} steps, "
                      f"{dt:.1f} s")
    if not one_core:
        out["single_core"] = cpu_baseline_one_core(name)
    return out


def cpu_baseline_one_core(name, budget_s=6.0):
    """The same oracle sample on one core: a child process with
    OMP_NUM_THREADS=1 (the oracle library fixes its thread count when it
    loads), so that nothing in it touches the GPU."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.cpu_baseline(%r, %r, one_core=True)))" % (ROOT, name, budget_s))
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fno", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the 256x128x128 run with the running mean on")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32/FP16/BF16 storage study")
    ap.add_argument("--copy-calib", action="store_true", help="only run a plain device copy of known size")
    ap.add_argument("--fno-only", action="store_true", help="only time the FNO forward and training step at batch 16")
    ap.add_argument("--fno-forward-reps", type=int, default=0,
                    help="only run this many timed FNO forward passes at batch 16 (a profiling target)")
    ap.add_argument("--unet-forward-reps", type=int, default=0,
                    help="only run this many timed U-Net forward passes at batch 16 (a profiling target)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the x-slab "
              "decomposition across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    sys.path.insert(0, ROOT)
    from paper_2606_16765_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    if args.copy_calib:
        # plain copy kernel of known size, for scaling the HBM counters
        print(json.dumps({"copy_bytes_read": 4 * 2 ** 30, "copy_bytes_written": 4 * 2 ** 30,
                          "copy_GBps": copy_rate()}), flush=True)
        return

    if args.unet_forward_reps:
        # a profiling target: only U-Net forward passes at batch 16
        from paper_2606_16765_amd import unet as punet
        print(json.dumps({"unet_forward": punet.bench_inference(batch=16, reps=args.unet_forward_reps)}), flush=True)
        return
    if args.fno_forward_reps:
        # a profiling target: only FNO forward passes at batch 16
        from paper_2606_16765_amd import fno as pfno
        print(json.dumps({"fno_forward": pfno.bench_inference(batch=16, reps=args.fno_forward_reps)}), flush=True)
        return
    if args.fno_only:
        print(json.dumps({"fno": fno_leg()}), flush=True)
        return

    res = run_lbm(args.workload, args.steps, args.warmup)
    traffic = read_traffic(args.workload)
    line = {
        "metric": "D3Q27 cumulant MLUPS + % HBM roofline; FNO vs LBM mean-field time at L2 err",
        "value": round(res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["storage"],
        "data": "synthetic (seeded geometry and perturbation; no dataset)",
        "config": {"workload": res["desc"], "cells": res["N"], "solid_cells": res["n_solid"],
                   "u_in": 0.05, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(res["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(res["achieved"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "lbm_step_kernel (stream-collide, two-lattice pull)",
                     "bytes_per_launch": res["bytes_per_launch"], "bytes_per_cell_update": res["bytes_per_cell"],
                     "kernel_ms": round(res["kernel_ms"], 4),
                     "same_pattern_probe_gbs": round(res["probe_gbs"], 1),
                     "frac_of_probe": round(res["achieved"] / res["probe_gbs"], 4),
                     "probe_note": "lbm_bandwidth_probe: the pull step's loads and stores of every cell with the "
                                   "collision left out, same kernel layout and tile order"},
    }
    cgbs = copy_rate()
    line["roofline"]["plain_copy_gbs"] = round(cgbs, 1)
    line["roofline"]["frac_of_copy"] = round(res["achieved"] / cgbs, 4)
    line["roofline"]["plain_copy_note"] = ("lbm_copy_bandwidth: 4 GiB read + 4 GiB written, one 16-byte vector per "
                                           "lane, non-temporal stores")
    tgbs = torch_copy_rate()
    line["roofline"]["torch_copy_gbs"] = round(tgbs, 1)
    log(f"plain 4 GiB copy: {cgbs:.0f} GB/s (library), {tgbs:.0f} GB/s (torch)")
    if "cd" in res:
        line["physics"] = {"cd_mean_second_half": round(res["cd"], 4), "cl_rms_second_half": round(res["cl_rms"], 4),
                           "strouhal": None,
                           "strouhal_note": "one shedding period is about 6000 steps at this size; not "
                                            "resolvable within the timed steps (the 66,000-step run of this "
                                            "workload is under validation.cylinder)"}
    if not args.no_c1:
        line["c1_running_mean"] = c1_leg()
        log(f"c1 with running mean: {line['c1_running_mean']}")
    if not args.no_fno:
        line["fno"] = fno_leg()
        log(f"fno: {line['fno']}")
    if not args.no_fno:
        sur = read_surrogate_result()
        if sur is not None:
            line.setdefault("fno", {})["surrogate_run"] = sur
    val = read_validation_result()
    if val is not None:
        line["validation"] = val
    if not args.no_precision:
        from paper_2606_16765_amd import precision
        log("precision study ...")
        line["precision"] = {
            "error_vs_f64": precision.error_table(log=log, oracle_means=precision_oracle_means()),
            "throughput": precision.throughput(log=log),
        }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(args.workload)
        log(f"cpu baseline: {line['cpu_baseline']}")
        if "fno" in line:
            line["fno"]["cpu_oracle"] = fno_cpu_baseline()
            log(f"fno oracle: {line['fno']['cpu_oracle']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
