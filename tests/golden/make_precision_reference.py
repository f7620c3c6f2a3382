"""Write the FP64 oracle's mean fields of the storage-precision study's
laminar case, the reference of the GPU's FP32, FP16 and BF16 storage errors.

Configuration (the precision study's): the seeded random obstacle of the
256x128x128 generator (seed 0) scaled to a 128x64x64 channel, u_in = 0.05,
Re 1000 on the channel height (nu = 0.05 * 64 / 1000, plain cumulant mode,
Sec. 3.2: the fourth-order mode is off below Re_c 3000), interpolated
bounce-back with the generator's wall distances, initial velocity the
seeded 1% perturbation (seed 0, amplitude 0.01 u_in), 10,000 steps, means
of u, v, w, p over steps [5000, 10000) (Sec. 2).

Output: precision_ref_re1000.npz beside this script, the four mean fields
[4][nz][ny][nx] rounded to float32 (the comparison is at the 1e-6 level;
float32 adds at most 6e-8 relative), plus the configuration.  Calls only
the oracle and the seeded input generators.

    python tests/golden/make_precision_reference.py     # ~15 min on 8 cores
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from inputs import perturbation, random_obstacle  # noqa: E402
from oracle import lbm as olbm  # noqa: E402

SHAPE = (128, 64, 64)
RE = 1000.0
STEPS = 10000
U_IN = 0.05
AMP = 0.01 * U_IN
OUT = os.path.join(HERE, "precision_ref_re1000.npz")


def main():
    geo = random_obstacle(SHAPE, 0)
    u0 = perturbation(SHAPE, 0, AMP, geo.solid)
    nu = U_IN * SHAPE[1] / RE
    p = olbm.make_params(SHAPE, nu=nu, u_in=U_IN, mode=0, obstacle_bc=1, avg_start=STEPS // 2)
    r = olbm.Run(p, solid=geo.solid, links=geo.links, u0=u0)
    t0 = time.time()
    chunk = 500
    for k in range(0, STEPS, chunk):
        r.step(chunk, forces=False)
        print(f"{k + chunk}/{STEPS} steps, {time.time() - t0:.0f} s", flush=True)
    m = r.mean_fields()
    assert r.count == STEPS - STEPS // 2
    np.savez_compressed(OUT, means=m.astype(np.float32), shape=np.array(SHAPE), re=RE, steps=STEPS,
                        window=np.array([STEPS // 2, STEPS]), u_in=U_IN, amp=AMP, obstacle_seed=0, perturb_seed=0,
                        threads=olbm.threads())
    print(OUT, os.path.getsize(OUT), "bytes", flush=True)


if __name__ == "__main__":
    main()
