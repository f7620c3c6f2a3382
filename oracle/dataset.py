"""FP64/numpy oracle of the surrogate's data curation.

TEST INFRASTRUCTURE ONLY: the product library never imports this module.

Paper Sec. 2 stores the fields at a reduced resolution. App. A.2 trains on
128x64x64 fields with min-max scaling per field and adds three 90-degree
turns about the x axis per geometry. The readings used here:

* the reduced field is the mean over f x f x f blocks of the mean fields,
  with solid cells counting as zero;
* a quarter turn about +x takes +y to +z and +z to -y. The turned field at
  a point is R applied to the original field at R^-1 of that point;
* scaling maps each channel to (x - min) / (max - min), where min and max
  are taken over all samples and points.
"""
import numpy as np


def pool_mean(means, f):
    """means: natural-layout [4][nz][ny][nx] (solid cells already zero).
    Returns [4][nx/f][ny/f][nz/f] in the surrogate layout (z fastest): the
    plain mean over each f^3 block."""
    c, nz, ny, nx = means.shape
    a = np.transpose(np.asarray(means, np.float64), (0, 3, 2, 1))  # [c][x][y][z]
    X, Y, Z = nx // f, ny // f, nz // f
    out = np.zeros((c, X, Y, Z))
    for dx in range(f):
        for dy in range(f):
            for dz in range(f):
                out += a[:, dx::f, dy::f, dz::f][:, :X, :Y, :Z]
    return out / f ** 3


def quarter_turn(fields, q):
    """fields [4][X][Y][Z] = (u, v, w, p), Y == Z. q quarter turns about +x.
    One turn: out[x, y, z] = R field[x, z, Y-1-y], R (u, v, w) = (u, -w, v)."""
    out = np.asarray(fields, np.float64).copy()
    n = out.shape[2]
    assert out.shape[2] == out.shape[3]
    for _ in range(q % 4):
        src = out
        out = np.empty_like(src)
        for y in range(n):
            for z in range(n):
                u, v, w, p = src[:, :, z, n - 1 - y]
                out[0, :, y, z] = u
                out[1, :, y, z] = -w
                out[2, :, y, z] = v
                out[3, :, y, z] = p
    return out


def turn_mask(solid, q):
    """Natural-layout mask [nz][ny][nx] turned like a scalar field."""
    a = np.asarray(solid)
    n = a.shape[0]
    assert a.shape[0] == a.shape[1]
    for _ in range(q % 4):
        src = a
        a = np.empty_like(src)
        for y in range(n):
            for z in range(n):
                a[z, y, :] = src[n - 1 - y, z, :]
    return a


def minmax(x):
    """Per-channel minimum and maximum of x [S][C][...]."""
    x = np.asarray(x)
    C = x.shape[1]
    flat = np.moveaxis(x, 1, 0).reshape(C, -1)
    return flat.min(1), flat.max(1)


def scale(x, lo, hi, inverse=False):
    x = np.asarray(x, np.float64)
    shp = (1, -1) + (1,) * (x.ndim - 2)
    lo = np.asarray(lo, np.float64).reshape(shp)
    hi = np.asarray(hi, np.float64).reshape(shp)
    r = hi - lo
    if inverse:
        return x * r + lo
    return np.where(r > 0, (x - lo) / np.where(r > 0, r, 1.0), 0.0)


__all__ = ["pool_mean", "quarter_turn", "turn_mask", "minmax", "scale"]
