"""Host logic of bench.py: the readers of the committed profiles (no GPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import pytest  # noqa: E402


def test_traffic_file_belongs_to_the_current_step_kernel_sources():
    """roofline.traffic is reported only while the counter summary was taken
    on the current lbm.hip / lbm_device.h; the committed summary must match
    them, and its bytes lie within a few percent of the algorithmic count."""
    t = bench.read_traffic("c2")
    if t is None:
        pytest.skip("profiles/lbm_step_c2_traffic.txt predates the current LBM sources: retake the counters")
    alg = 57894608896
    assert 0.95 < t / alg < 1.10


def test_surrogate_and_validation_summaries_parse():
    s = bench.read_surrogate_result()
    assert s is not None and 0 < s["fno_held_out"]["rel_l2_inner"] < s["mean_field_held_out"]["rel_l2_inner"]
    assert "hybrid_held_out" in s and "fno_siren_projection_held_out" in s
    # the U-Net beats the FNO inside the loss box, as in the paper's Table 2
    assert s["unet_held_out"]["rel_l2_inner"] < s["fno_held_out"]["rel_l2_inner"]
    v = bench.read_validation_result()
    Ls = {(r["L"], r["re_s"]) for r in v["sphere_periodic"]}
    assert {(128, 1000), (256, 1000), (384, 1000)} <= Ls
    full = [c for c in v["cylinder"] if c["shape"] == [1024, 512, 512]]
    assert full and 0.19 < full[0]["strouhal"] < 0.23
