"""Input channels of the surrogate (paper Sec. 4 and App. A.2: geometry and
Reynolds number in, mean fields out), evaluated on the coarse grid of the
pooled fields.

Channels, each [X][Y][Z] with Z fastest, at the centres of the factor^3
blocks of the fine channel (fine coordinate factor*i + (factor-1)/2):
  0  signed distance / 16, clipped to [-1, 1]
  1  obstacle mask (1 where the signed distance at the centre is <= 0)
  2  Re / 10^4 (constant)
  3  angle of attack / 15 degrees (constant)
"""
import numpy as np

from .geometry import obstacle_sdf


def coarse_inputs(shape, seed, factor=2, turns=0, re=None, aoa=None):
    """float32 [4][X][Y][Z] for the seeded random obstacle in a channel of
    the given fine shape, and the object description (re and aoa override
    the seeded values)."""
    nx, ny, nz = shape
    X, Y, Z = nx // factor, ny // factor, nz // factor
    obj, sdf, _, _ = obstacle_sdf(shape, seed, turns=turns, re=re, aoa=aoa)
    off = (factor - 1) / 2.0
    x, y, z = np.meshgrid(np.arange(X) * factor + off, np.arange(Y) * factor + off, np.arange(Z) * factor + off,
                          indexing="ij")
    d = sdf(np.stack([x, y, z], -1))
    out = np.empty((4, X, Y, Z), np.float32)
    out[0] = np.clip(d / 16.0, -1.0, 1.0)
    out[1] = (d <= 0.0)
    out[2] = obj["re"] / 1.0e4
    out[3] = obj["aoa"] / 15.0
    return out, obj


def to_bf16_bits(a):
    """Round float32 to bfloat16 (nearest, ties to even); returns uint16."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    nan = np.isnan(np.ascontiguousarray(a, np.float32))
    r = np.where(nan, 0x7FC0, r)
    return r.astype(np.uint16)
