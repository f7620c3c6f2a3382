"""Seeded input generators: counter-based RNG and obstacle geometry."""
import math

import numpy as np

from inputs import perturbation, random_obstacle, sphere_channel, spanwise_cylinder, splitmix64
from inputs.geometry import directions


def test_splitmix64_published_first_output():
    # first output of SplitMix64 seeded with 0
    assert int(splitmix64(0, 0)) == 0xE220A8397B1DCDAF


def test_perturbation_is_seeded_and_bounded():
    a = perturbation((8, 4, 4), 3, 5e-4)
    b = perturbation((8, 4, 4), 3, 5e-4)
    c = perturbation((8, 4, 4), 4, 5e-4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.abs(a).max() <= 5e-4 and abs(a.mean()) < 1e-4


def test_sphere_geometry_links_are_exact_distances():
    g = sphere_channel((64, 32, 32), center=(16.0, 15.5, 15.5), radius=4.0)
    zz, yy, xx = np.nonzero(g.solid)
    d = np.sqrt((xx - 16.0) ** 2 + (yy - 15.5) ** 2 + (zz - 15.5) ** 2)
    assert d.max() <= 4.0 and g.n_solid > 4 / 3 * math.pi * 3.0 ** 3
    c = directions()
    cell, dr, q = g.links
    x, y, z = cell % 64, (cell // 64) % 32, cell // (64 * 32)
    # the crossing point lies on the sphere
    px = x + q * c[dr, 0]
    py = y + q * c[dr, 1]
    pz = z + q * c[dr, 2]
    r = np.sqrt((px - 16.0) ** 2 + (py - 15.5) ** 2 + (pz - 15.5) ** 2)
    assert np.abs(r - 4.0).max() < 1e-9
    # every link starts in fluid and ends in solid
    assert not g.solid.reshape(-1)[cell].any()
    nb = ((z + c[dr, 2]) * 32 + (y + c[dr, 1])) * 64 + (x + c[dr, 0])
    assert g.solid.reshape(-1)[nb].all()


def test_random_obstacle_reproducible_and_placed():
    g1 = random_obstacle((128, 64, 64), 5)
    g2 = random_obstacle((128, 64, 64), 5)
    assert np.array_equal(g1.solid, g2.solid)
    assert g1.n_solid > 0
    zz, yy, xx = np.nonzero(g1.solid)
    assert abs(xx.mean() - 0.3 * 128) < 12
    assert 1000 <= g1.params["re"] <= 10000 and -15 <= g1.params["aoa"] <= 15


def test_spanwise_cylinder_links():
    g = spanwise_cylinder((128, 64, 16), center=(38.4, 31.5), diameter=16.0)
    assert g.solid[:, 31, 38] .all()
    cell, dr, q = g.links
    c = directions()
    x, y = cell % 128, (cell // 128) % 64
    px, py = x + q * c[dr, 0], y + q * c[dr, 1]
    assert np.abs(np.hypot(px - 38.4, py - 31.5) - 8.0).max() < 1e-9


def test_turned_obstacle_is_the_turned_mask():
    from oracle import dataset as ods
    shape = (64, 32, 32)
    for seed in (3, 8):
        g0 = random_obstacle(shape, seed)
        for q in (1, 2, 3):
            gq = random_obstacle(shape, seed, turns=q)
            assert np.array_equal(gq.solid, ods.turn_mask(g0.solid, q))


def test_coarse_inputs_channels():
    from inputs import coarse_inputs, to_bf16_bits
    shape = (128, 64, 64)
    x, obj = coarse_inputs(shape, 5)
    assert x.shape == (4, 64, 32, 32) and x.dtype == np.float32
    assert -1.0 <= x[0].min() and x[0].max() <= 1.0
    assert np.array_equal(x[1] > 0, x[0] <= 0)
    assert x[1].sum() > 0
    assert np.all(x[2] == np.float32(obj["re"] / 1e4)) and np.all(x[3] == np.float32(obj["aoa"] / 15.0))
    # the obstacle sits near x = 0.3 nx
    xs = np.nonzero(x[1])[0]
    assert abs(xs.mean() * 2 + 0.5 - 0.3 * 128) < 6
    # bf16 rounding: exact for representable values, ties to even
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5], np.float32)
    assert list(to_bf16_bits(v)) == [0x3F80, 0x3F80, 0x3F82, 0xC020]


def test_reynolds_and_angle_overrides():
    """re and aoa replace the seeded values in the description, the input
    channels and the geometry (the angle turns the obstacle)."""
    from inputs import coarse_inputs, random_obstacle
    shape = (64, 32, 32)
    base, obj = coarse_inputs(shape, 7)
    feats, obj2 = coarse_inputs(shape, 7, re=2500.0, aoa=-12.0)
    assert obj2["re"] == 2500.0 and obj2["aoa"] == -12.0
    assert np.all(feats[2] == np.float32(0.25)) and np.all(feats[3] == np.float32(-0.8))
    same, _ = coarse_inputs(shape, 7, re=obj["re"], aoa=obj["aoa"])
    assert np.array_equal(same, base)
    g0 = random_obstacle(shape, 7)
    g1 = random_obstacle(shape, 7, aoa=obj["aoa"] + 10.0)
    assert g1.params["aoa"] == obj["aoa"] + 10.0 and not np.array_equal(g0.solid, g1.solid)
