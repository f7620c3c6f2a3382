"""Pins of the data-curation oracle (block-mean downsampling, quarter turns
about x, per-field min-max scaling; paper Sec. 2 and App. A.2) against
library routines, invariants and the solver's own symmetry."""
import numpy as np
import pytest

from oracle import dataset as ods
from oracle import lbm as olbm

RNG = np.random.default_rng(7)


def test_pool_mean_equals_reshape_mean_and_keeps_the_sum():
    m = RNG.standard_normal((4, 6, 8, 10))  # natural [c][z][y][x]
    out = ods.pool_mean(m, 2)
    a = np.transpose(m, (0, 3, 2, 1)).reshape(4, 5, 2, 4, 2, 3, 2).mean(axis=(2, 4, 6))
    assert out.shape == (4, 5, 4, 3)
    assert np.abs(out - a).max() < 1e-15
    assert abs(out.sum() * 8 - m.sum()) < 1e-12
    const = np.kron(RNG.standard_normal((4, 3, 4, 5)), np.ones((1, 2, 2, 2)))  # constant per block
    assert np.abs(ods.pool_mean(const, 2) - np.transpose(const[:, ::2, ::2, ::2], (0, 3, 2, 1))).max() < 1e-15


@pytest.mark.parametrize("q", [1, 2, 3])
def test_quarter_turn_scalar_part_is_rot90(q):
    f = RNG.standard_normal((4, 3, 6, 6))
    t = ods.quarter_turn(f, q)
    assert np.array_equal(t[3], np.rot90(f[3], q, axes=(1, 2)))


def test_quarter_turn_vectors_and_group_laws():
    n = 6
    f = RNG.standard_normal((4, 3, n, n))
    assert np.array_equal(ods.quarter_turn(f, 4), f)
    assert np.abs(ods.quarter_turn(ods.quarter_turn(f, 1), 3) - f).max() == 0.0
    # uniform +y flow turns into uniform +z flow, +z into -y
    e = np.zeros((4, 2, n, n))
    e[1] = 1.0
    t = ods.quarter_turn(e, 1)
    assert np.all(t[2] == 1.0) and np.all(t[1] == 0.0)
    e = np.zeros((4, 2, n, n))
    e[2] = 1.0
    t = ods.quarter_turn(e, 1)
    assert np.all(t[1] == -1.0) and np.all(t[2] == 0.0)
    # a solid-body rotation about the x axis is invariant
    c = (n - 1) / 2
    y, z = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r = np.zeros((4, 2, n, n))
    r[1] = -z
    r[2] = y
    assert np.abs(ods.quarter_turn(r, 1) - r).max() < 1e-15


def test_turn_mask_matches_scalar_turn():
    s = (RNG.random((6, 6, 5)) > 0.5).astype(np.uint8)  # natural [z][y][x]
    f = np.zeros((4, 5, 6, 6))
    f[3] = np.transpose(s, (2, 1, 0))
    for q in range(4):
        assert np.array_equal(np.transpose(ods.turn_mask(s, q), (2, 1, 0)), ods.quarter_turn(f, q)[3])


def test_minmax_and_scale_round_trip():
    x = RNG.standard_normal((5, 3, 4, 4)) * np.array([1.0, 10.0, 0.1])[None, :, None, None]
    lo, hi = ods.minmax(x)
    for c in range(3):
        assert lo[c] == x[:, c].min() and hi[c] == x[:, c].max()
    y = ods.scale(x, lo, hi)
    assert np.allclose(y.min(axis=(0, 2, 3)), 0.0, atol=0) and np.allclose(y.max(axis=(0, 2, 3)), 1.0, atol=1e-15)
    assert np.abs(ods.scale(y, lo, hi, inverse=True) - x).max() < 1e-13
    const = np.ones((2, 1, 3))
    assert np.array_equal(ods.scale(const, *ods.minmax(const)), np.zeros((2, 1, 3)))


@pytest.mark.skipif(not olbm.available(), reason="oracle library not built")
def test_solver_is_equivariant_under_quarter_turns():
    """The square channel (ny == nz, walls on four sides, inlet and outlet
    along x) is symmetric under turns about x: the mean fields of the turned
    obstacle are the turned mean fields, up to rounding."""
    shape = (24, 8, 8)
    solid = np.zeros((8, 8, 24), np.uint8)
    solid[2:5, 1:4, 6:9] = 1   # an off-centre block, no symmetry of its own
    solid[3, 5, 7] = 1
    p = olbm.make_params(shape, nu=0.02, u_in=0.05, mode=0, avg_start=0)
    r0 = olbm.Run(p, solid=solid)
    r0.step(60)
    r1 = olbm.Run(p, solid=ods.turn_mask(solid, 1))
    r1.step(60)
    a = ods.quarter_turn(ods.pool_mean(r0.mean_fields(), 1), 1)
    b = ods.pool_mean(r1.mean_fields(), 1)
    assert np.abs(a).max() > 1e-3
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max() + 1e-15
