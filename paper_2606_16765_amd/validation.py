"""Physics validation runs on the GPU path (paper Sec. 3.3 and Table 1).

sphere_drag: the sphere of the paper's drag study in the 2L x L x L channel,
D = L/6 (Re_c = 6 Re_s on the channel height), centred at x = 0.3 * 2L, at
channel resolution L; FP32, interpolated bounce-back, the K17 switch at
Re_c 3000.  The drag coefficient is c_d = 2 <F_x> / (u_in^2 pi D^2 / 4)
with <F_x> the mean momentum-exchange force over the second half of the
run (FP64 series, every step); the Strouhal number St = f D / u_in comes
from the dominant frequency of the lift (F_y and F_z power spectra summed,
Hann window, second half).

cylinder_strouhal: the spanwise cylinder of the 1024x512x512 workload at a
reduced resolution (same blockage D/H = 1/8, Re_D 3900), St from the lift
F_y over the second half of the run.

    python -m paper_2606_16765_amd.validation --res 128 256 --out result.json
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from .lbm import Lbm, nu_from_re


def _run_steps(sim, steps, log, label, parts=10):
    """Step in chunks, waiting for each, with a progress line per chunk
    (long runs at large L print something every minute or so)."""
    import torch
    chunk = max(1, -(-steps // parts))
    done = 0
    t0 = time.time()
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        torch.cuda.synchronize()
        done += k
        if done < steps:
            log(f"{label}: {done}/{steps} steps ({time.time() - t0:.0f} s)")

# paper Table 1 (drag coefficient of the sphere at channel resolution L)
TABLE1 = {
    100: {128: 1.122, 256: 1.108, 384: 1.106, 512: 1.106, "ref": 1.08},
    500: {128: 0.573, 256: 0.562, 384: 0.563, 512: 0.562, "ref": 0.547},
    1000: {128: 0.479, 256: 0.460, 384: 0.466, 512: 0.467, 1024: 0.472, "ref": 0.472},
    2000: {128: 0.434, 256: 0.407, 384: 0.407, 512: 0.404, "ref": 0.430},
}


def dominant_frequency(signals, dt=1.0, band=None):
    """Frequency (cycles per step) of the largest peak of the summed power
    spectra of zero-mean, Hann-windowed signals, excluding the two lowest
    bins and, when band = (fmin, fmax) is given, everything outside it."""
    n = len(signals[0])
    w = np.hanning(n)
    power = np.zeros(n // 2 + 1)
    for s in signals:
        s = np.asarray(s, np.float64)
        power += np.abs(np.fft.rfft((s - s.mean()) * w)) ** 2
    freqs = np.fft.rfftfreq(n, dt)
    sel = np.arange(len(power)) >= 2
    if band is not None:
        sel &= (freqs >= band[0]) & (freqs <= band[1])
    idx = np.nonzero(sel)[0]
    k = int(idx[np.argmax(power[idx])])
    # parabolic interpolation of the peak on the log power
    if 1 <= k < len(power) - 1:
        a, b, c = np.log(power[k - 1] + 1e-300), np.log(power[k] + 1e-300), np.log(power[k + 1] + 1e-300)
        den = a - 2 * b + c
        off = 0.5 * (a - c) / den if den != 0 else 0.0
        return float((k + off) * (freqs[1] - freqs[0]))
    return float(freqs[k])


def approach_velocity(res=128, re_s=(100, 500, 1000, 2000), ftt=6.0, u_in=0.05, storage="f32", log=print):
    """Mean streamwise velocity at the sphere's centre in the empty duct
    (same inlet, walls, Re and run length, averaged over the second half):
    the uniform inlet profile accelerates in the core as the wall boundary
    layers grow, so the sphere meets a faster stream than u_in."""
    L = int(res)
    shape = (2 * L, L, L)
    D = L / 6.0
    steps = int(round(ftt * 2 * L / u_in))
    xc, yc = 0.3 * 2 * L, (L - 1) / 2.0
    out = {}
    for re in re_s:
        sim = Lbm(shape, storage=storage, u_in=u_in, nu=nu_from_re(u_in, D, re), mode="auto", obstacle_bc=1,
                  avg_start=steps // 2, force_every=0, perturb=(0, 0.01 * u_in))
        sim.step(steps)
        m, _ = sim.mean_fields()
        sim.close()
        x0 = int(math.floor(xc))
        wx = xc - x0
        y0 = int(math.floor(yc))
        u = m[0][y0:y0 + 2, y0:y0 + 2, :]  # [z][y][x], z and y both centred
        uc = float((1 - wx) * u[:, :, x0].mean() + wx * u[:, :, x0 + 1].mean())
        out[re] = uc
        log(f"empty duct L={L} Re_s {re}: u at the sphere centre {uc:.5f} = {uc / u_in:.4f} u_in")
    return out


def sphere_drag(res=128, re_s=(100, 500, 1000, 2000), ftt=6.0, u_in=0.05, storage="f32", log=print,
                approach=None, lateral="walls"):
    """lateral = "walls" (no-slip side walls, the channel of the dataset) or
    "periodic" (periodic in y and z: no wall confinement, only the blockage
    of the periodic images)."""
    from inputs import sphere_channel
    L = int(res)
    shape = (2 * L, L, L)
    D = L / 6.0
    geo = sphere_channel(shape, center=(0.3 * 2 * L, (L - 1) / 2.0, (L - 1) / 2.0), radius=D / 2.0)
    area = math.pi * D * D / 4.0
    steps = int(round(ftt * 2 * L / u_in))
    rows = []
    for re in re_s:
        t0 = time.time()
        per = (0, 1, 1) if lateral == "periodic" else (0, 0, 0)
        sim = Lbm(shape, storage=storage, periodic=per, u_in=u_in, nu=nu_from_re(u_in, D, re), mode="auto",
                  solid=geo.solid, links=geo.links, obstacle_bc=1, avg_start=None, force_every=1,
                  perturb=(0, 0.01 * u_in))
        mode = sim.info()["mode"]
        _run_steps(sim, steps, log, f"sphere L={L} Re_s {re}")
        F, _ = sim.forces()
        mass = sim.mass()
        sim.close()
        half = F[len(F) // 2:]
        cd = float(2.0 * half[:, 0].mean() / (u_in * u_in * area))
        # shedding band St 0.05 - 0.5; the transverse acoustic mode of the
        # duct (c_s / 2L, St near 1 at L = 6D) lies above it
        f = dominant_frequency([half[:, 1], half[:, 2]], band=(0.05 * u_in / D, 0.5 * u_in / D))
        lift_rms = float(np.sqrt(((half[:, 1:] - half[:, 1:].mean(0)) ** 2).sum(1).mean()) * 2 / (u_in ** 2 * area))
        row = dict(re_s=re, re_c=6 * re, mode="k17" if mode else "plain", steps=steps, cd=cd,
                   cd_paper=TABLE1.get(re, {}).get(L), cd_reference=TABLE1.get(re, {}).get("ref"),
                   strouhal=f * D / u_in, lift_rms_coefficient=lift_rms, stable=bool(np.isfinite(mass)),
                   seconds=time.time() - t0)
        if approach and re in approach:
            ua = approach[re]
            row["approach_velocity"] = ua
            row["cd_at_approach_velocity"] = float(2.0 * half[:, 0].mean() / (ua * ua * area))
        rows.append(row)
        log(f"sphere L={L} ({lateral}) Re_s {re}: c_d {cd:.4f} (paper {row['cd_paper']}, reference {row['cd_reference']}), "
            f"c_d at approach velocity {row.get('cd_at_approach_velocity', float('nan')):.4f}, "
            f"St {row['strouhal']:.3f}, {steps} steps in {row['seconds']:.1f} s")
    return dict(case="sphere", resolution=L, shape=list(shape), diameter=D, u_in=u_in, storage=storage,
                lateral=lateral, rows=rows)


def cylinder_strouhal(scale=0.5, steps=40000, re_d=3900.0, u_in=0.05, storage="f32", log=print):
    from inputs import spanwise_cylinder
    shape = (int(1024 * scale), int(512 * scale), int(512 * scale))
    D = 64.0 * scale
    geo = spanwise_cylinder(shape, center=(307.2 * scale, (shape[1] - 1) / 2.0), diameter=D)
    t0 = time.time()
    sim = Lbm(shape, storage=storage, u_in=u_in, nu=nu_from_re(u_in, D, re_d), mode="auto", solid=geo.solid,
              links=geo.links, obstacle_bc=1, avg_start=None, force_every=1, perturb=(0, 0.01 * u_in))
    _run_steps(sim, steps, log, f"cylinder {shape}")
    F, _ = sim.forces()
    sim.close()
    half = F[len(F) // 2:]
    area = D * shape[2]
    # shedding band St 0.05 - 0.5: the duct's transverse acoustic mode
    # (c_s / 2 ny, St = 0.72 at 1024x512x512) lies above it and can carry
    # more lift power than the shedding
    f = dominant_frequency([half[:, 1]], band=(0.05 * u_in / D, 0.5 * u_in / D))
    f_all = dominant_frequency([half[:, 1]])
    out = dict(case="spanwise cylinder", shape=list(shape), diameter=D, re_d=re_d, steps=steps,
               cd=float(2.0 * half[:, 0].mean() / (u_in * u_in * area)),
               cl_rms=float(2.0 * half[:, 1].std() / (u_in * u_in * area)),
               strouhal=f * D / u_in, periods_in_window=f * len(half),
               strouhal_unbanded_peak=f_all * D / u_in,
               strouhal_acoustic_mode=(1.0 / math.sqrt(3.0)) / (2.0 * shape[1]) * D / u_in,
               lift_every_50_steps_second_half=[float(v) for v in half[::50, 1]],
               seconds=time.time() - t0)
    log(f"cylinder {shape} D={D}: c_d {out['cd']:.3f}, c_l rms {out['cl_rms']:.3f}, St {out['strouhal']:.3f} "
        f"({out['periods_in_window']:.1f} periods), {out['seconds']:.1f} s")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--res", type=int, nargs="*", default=[128, 256])
    ap.add_argument("--re", type=int, nargs="*", default=[100, 500, 1000, 2000])
    ap.add_argument("--ftt", type=float, default=6.0)
    ap.add_argument("--cylinder-scale", type=float, default=0.5)
    ap.add_argument("--cylinder-steps", type=int, default=40000)
    ap.add_argument("--no-cylinder", action="store_true")
    ap.add_argument("--periodic-res", type=int, nargs="*", default=[128],
                    help="resolutions of the extra runs with periodic lateral boundaries")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(f"[validation] {m}", flush=True)
    appr = approach_velocity(min(a.res), tuple(a.re), a.ftt, log=log) if a.res else {}
    res = {"approach_velocity": {str(k): v for k, v in appr.items()},
           "sphere": [sphere_drag(r, tuple(a.re), a.ftt, log=log, approach=appr) for r in a.res],
           "sphere_periodic": [sphere_drag(r, tuple(a.re), a.ftt, log=log, lateral="periodic")
                               for r in a.periodic_res]}
    if not a.no_cylinder:
        res["cylinder"] = cylinder_strouhal(a.cylinder_scale, a.cylinder_steps, log=log)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as fh:
            fh.write(json.dumps(res) + "\n")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
