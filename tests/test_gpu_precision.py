"""Storage precision against the FP64 CPU oracle at the precision study's
full length: the seeded random obstacle at 128x64x64, Re 1000 on the channel
height (plain mode, laminar), interpolated bounce-back, 10,000 steps, means
over [5000, 10000).  The oracle's means come from
tests/golden/make_precision_reference.py (stored in float32, which adds at
most 6e-8 relative).

Bounds: FP64 storage 1e-7 on every field (measured 2.0e-8 to 2.5e-8; the
float32 storage of the reference dominates).  FP32 storage: 1e-5 relative L2
on the stacked mean velocity, the target of the FP32 path (measured 2.9e-6),
and on u and p (2.9e-6, 2.8e-6); the transverse means v and w are an order
of magnitude smaller than u, so the same absolute rounding is a larger
relative error: bound 3.6e-5, twice the measured 1.8e-5 and 1.4e-5.  FP16
and BF16 shifted storage: twice the measured stacked-velocity error (5.8e-3,
5.7e-2)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REF = os.path.join(HERE, "golden", "precision_ref_re1000.npz")


@pytest.fixture(scope="module")
def case():
    from inputs import random_obstacle
    d = np.load(REF)
    shape = tuple(int(v) for v in d["shape"])
    geo = random_obstacle(shape, int(d["obstacle_seed"]))
    return d, geo


def _means(geo, d, storage):
    import paper_2606_16765_amd as P
    steps = int(d["steps"])
    sim = P.Lbm(geo.shape, storage=storage, u_in=float(d["u_in"]), re=float(d["re"]), mode="auto",
                solid=geo.solid, links=geo.links, obstacle_bc=1, avg_start=int(d["window"][0]), force_every=0,
                perturb=(int(d["perturb_seed"]), float(d["amp"])))
    assert sim.info()["mode"] == 0
    sim.step(steps)
    m, n = sim.mean_fields()
    sim.close()
    assert n == steps - int(d["window"][0])
    return m.reshape(4, -1)


def _err(m, ref, fluid):
    e = {"vel": float(np.linalg.norm(m[:3, fluid] - ref[:3, fluid]) / np.linalg.norm(ref[:3, fluid]))}
    for k, name in enumerate("uvwp"):
        e[name] = float(np.linalg.norm(m[k, fluid] - ref[k, fluid]) / np.linalg.norm(ref[k, fluid]))
    return e


@pytest.mark.parametrize("storage,bound", [("f64", 1e-7), ("f32", 1e-5), ("f16", 1.2e-2), ("bf16", 1.2e-1)])
def test_storage_precision_against_the_oracle_at_re1000(case, storage, bound):
    d, geo = case
    ref = d["means"].astype(np.float64).reshape(4, -1)
    fluid = geo.solid.reshape(-1) == 0
    e = _err(_means(geo, d, storage), ref, fluid)
    print(storage, {k: float(f"{v:.3e}") for k, v in e.items()}, flush=True)
    assert e["vel"] < bound, e
    if storage == "f64":
        assert max(e.values()) < bound, e
    if storage == "f32":
        assert e["u"] < 1e-5 and e["p"] < 1e-5, e
        assert e["v"] < 3.6e-5 and e["w"] < 3.6e-5, e
