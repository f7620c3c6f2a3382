"""Obstacle geometries for the obstructed channel (seeded, synthetic).

The paper builds objects as unions of primitives (cylinder, rectangle, sphere,
torus, wedge) with an angle of attack, placed at x/2L = 0.3 and centred in
the y-z plane (Sec. 2, Sec. 3.1), and uses wall distances for its
interpolated bounce-back (Sec. 3.2).  Here:

* nodes sit at integer coordinates 0..N-1; the lateral walls are at -1/2 and
  N-1/2;
* a node is solid iff the signed distance at the node is <= 0;
* for every fluid node x and lattice direction c with x + c solid, the wall
  distance fraction q in (0, 1] is the zero of sdf(x + t c) on t in [0, 1],
  found by bisection to 1e-13.

Directions use the index i = 9(cz+1) + 3(cy+1) + (cx+1).
"""
from dataclasses import dataclass
import math

import numpy as np

from .rng import uniform_pm1


def directions():
    c = np.zeros((27, 3), dtype=np.int64)
    for i in range(27):
        c[i] = (i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1)
    return c


@dataclass
class Geometry:
    shape: tuple            # (nx, ny, nz)
    solid: np.ndarray       # uint8 [nz][ny][nx]
    links: tuple            # (cell int64[n], direction uint8[n], q float64[n])
    frontal_area: float     # projected area normal to x (cells^2), for c_d
    name: str = ""
    params: dict = None

    @property
    def n_solid(self):
        return int(self.solid.sum())


# ---------------------------------------------------------------- primitives
def _sd_sphere(p, r):
    return np.sqrt((p ** 2).sum(-1)) - r


def _sd_box(p, b):
    q = np.abs(p) - b
    out = np.sqrt((np.maximum(q, 0.0) ** 2).sum(-1))
    return out + np.minimum(q.max(-1), 0.0)


def _sd_cylinder(p, r, h):
    """Capped cylinder along local z: radius r, half-height h."""
    d = np.stack([np.sqrt(p[..., 0] ** 2 + p[..., 1] ** 2) - r, np.abs(p[..., 2]) - h], -1)
    return np.minimum(d.max(-1), 0.0) + np.sqrt((np.maximum(d, 0.0) ** 2).sum(-1))


def _sd_torus(p, R, r):
    q = np.stack([np.sqrt(p[..., 0] ** 2 + p[..., 1] ** 2) - R, p[..., 2]], -1)
    return np.sqrt((q ** 2).sum(-1)) - r


def _sd_wedge(p, s, h):
    """Triangular prism: cross-section the triangle (-s/2,-s/2), (s/2,-s/2),
    (-s/2, s/2) in local x-y, half-depth h along z.  Intersection of half
    spaces (exact sign; distance exact near the faces)."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    d1 = -s / 2 - x
    d2 = -s / 2 - y
    d3 = (x + y) / math.sqrt(2.0)
    d4 = np.abs(z) - h
    return np.maximum(np.maximum(d1, d2), np.maximum(d3, d4))


def _rotation_from_quaternion(q):
    a, b, c, d = q / np.linalg.norm(q)
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def _rot_z(deg):
    t = math.radians(deg)
    return np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0], [0.0, 0.0, 1.0]])


class _Stream:
    """Sequential uniform variates from the counter-based generator."""

    def __init__(self, seed):
        self.seed, self.k = int(seed), 0

    def u(self, lo=0.0, hi=1.0):
        v = float(uniform_pm1(self.seed, self.k))
        self.k += 1
        return lo + (hi - lo) * 0.5 * (v + 1.0)

    def normal(self):
        # Box-Muller from two uniforms
        u1 = max(self.u(), 1e-300)
        u2 = self.u()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


PRIMITIVES = ("cylinder", "box", "sphere", "torus", "wedge")


def random_object(seed, scale=1.0):
    """Description of a seeded random object: 1-3 primitives, sizes U[8,24]
    cells (times scale), Haar-random rotations, centres offset U[-4,4]^3
    (times scale), angle of attack U[-15,15] deg about z."""
    st = _Stream(seed)
    n = 1 + min(int(st.u() * 3.0), 2)
    prims = []
    for _ in range(n):
        kind = PRIMITIVES[min(int(st.u() * 5.0), 4)]
        size = st.u(8.0, 24.0) * scale
        q = np.array([st.normal() for _ in range(4)])
        R = _rotation_from_quaternion(q)
        off = np.array([st.u(-4.0, 4.0) for _ in range(3)]) * scale
        aspect = st.u(0.5, 1.0)
        prims.append(dict(kind=kind, size=size, rot=R, offset=off, aspect=aspect))
    aoa = st.u(-15.0, 15.0)
    re = st.u(1000.0, 10000.0)
    return dict(prims=prims, aoa=aoa, re=re, seed=seed, scale=scale)


def object_sdf(obj, center):
    """Signed distance function of a described object placed at center."""
    Raoa = _rot_z(obj["aoa"])

    def sdf(p):
        p = np.asarray(p, dtype=np.float64)
        rel = (p - center) @ Raoa  # rotate the point by -aoa
        d = np.full(p.shape[:-1], np.inf)
        for pr in obj["prims"]:
            lp = (rel - pr["offset"]) @ pr["rot"]
            s, a = pr["size"], pr["aspect"]
            if pr["kind"] == "sphere":
                di = _sd_sphere(lp, s / 2)
            elif pr["kind"] == "box":
                di = _sd_box(lp, np.array([s / 2, s / 2 * a, s / 2 * (0.5 + 0.5 * a)]))
            elif pr["kind"] == "cylinder":
                di = _sd_cylinder(lp, s / 2 * a, s / 2)
            elif pr["kind"] == "torus":
                di = _sd_torus(lp, s / 2 * 0.7, s / 2 * 0.3)
            else:
                di = _sd_wedge(lp, s, s / 2 * a)
            d = np.minimum(d, di)
        return d

    return sdf


# ---------------------------------------------------------------- assembly
def _grid_points(shape, z0, z1):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(z0, z1), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x, y, z], -1).astype(np.float64)


def from_sdf(shape, sdf, name="", params=None, bbox=None, zchunk=16, margin=3):
    """Build solid mask and boundary links from a signed distance function.

    bbox = ((x0,x1),(y0,y1),(z0,z1)) limits the evaluation (cells outside are
    fluid); the obstacle must stay `margin` cells clear of inlet and outlet."""
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), np.uint8)
    if bbox is None:
        bbox = ((0, nx), (0, ny), (0, nz))
    (x0, x1), (y0, y1), (z0, z1) = [(max(0, int(a)), min(n, int(b))) for (a, b), n in zip(bbox, (nx, ny, nz))]
    for zs in range(z0, z1, zchunk):
        ze = min(z1, zs + zchunk)
        z, y, x = np.meshgrid(np.arange(zs, ze), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        pts = np.stack([x, y, z], -1).astype(np.float64)
        solid[zs:ze, y0:y1, x0:x1] = (sdf(pts) <= 0.0).astype(np.uint8)
    if solid[:, :, :margin].any() or solid[:, :, nx - margin - 1:].any():
        raise ValueError("obstacle too close to inlet or outlet")
    c = directions()
    cells, dirs, qs = [], [], []
    zi, yi, xi = np.nonzero(solid)
    if zi.size:
        # fluid neighbours of solid cells are the boundary cells
        for i in range(27):
            if i == 13:
                continue
            fx, fy, fz = xi - c[i, 0], yi - c[i, 1], zi - c[i, 2]
            ok = (fx >= 0) & (fx < nx) & (fy >= 0) & (fy < ny) & (fz >= 0) & (fz < nz)
            fx, fy, fz = fx[ok], fy[ok], fz[ok]
            ok2 = solid[fz, fy, fx] == 0
            fx, fy, fz = fx[ok2], fy[ok2], fz[ok2]
            if fx.size == 0:
                continue
            p0 = np.stack([fx, fy, fz], -1).astype(np.float64)
            lo = np.zeros(fx.size)
            hi = np.ones(fx.size)
            for _ in range(48):
                mid = 0.5 * (lo + hi)
                inside = sdf(p0 + mid[:, None] * c[i][None, :].astype(np.float64)) <= 0.0
                hi = np.where(inside, mid, hi)
                lo = np.where(inside, lo, mid)
            cells.append((fz.astype(np.int64) * ny + fy) * nx + fx)
            dirs.append(np.full(fx.size, i, np.uint8))
            qs.append(np.clip(0.5 * (lo + hi), 1e-6, 1.0))
    if cells:
        links = (np.concatenate(cells), np.concatenate(dirs), np.concatenate(qs))
        order = np.lexsort((links[1], links[0]))
        links = tuple(a[order] for a in links)
    else:
        links = (np.zeros(0, np.int64), np.zeros(0, np.uint8), np.zeros(0))
    area = float(solid.any(axis=2).sum())
    return Geometry(shape=tuple(shape), solid=solid, links=links, frontal_area=area, name=name, params=params)


def sphere_channel(shape=(64, 32, 32), center=(16.0, 15.5, 15.5), radius=4.0):
    """Sphere of the given radius in the channel (solid iff distance <= r)."""
    ctr = np.asarray(center, dtype=np.float64)
    r = float(radius)

    def sdf(p):
        return np.sqrt(((p - ctr) ** 2).sum(-1)) - r

    bb = tuple((ctr[d] - r - 2, ctr[d] + r + 3) for d in range(3))
    g = from_sdf(shape, sdf, name="sphere", params=dict(center=center, radius=radius), bbox=bb)
    g.frontal_area = math.pi * r * r
    return g


def spanwise_cylinder(shape=(1024, 512, 512), center=(307.2, 255.5), diameter=64.0):
    """Cylinder spanning z (wall to wall), axis at (x, y) = center."""
    nx, ny, nz = shape
    cx, cy = center
    r = diameter / 2.0

    def sdf(p):
        return np.sqrt((p[..., 0] - cx) ** 2 + (p[..., 1] - cy) ** 2) - r

    # the cross-section is z-independent: evaluate one plane, replicate
    z1 = min(nz, 1)
    plane = from_sdf((nx, ny, z1), sdf, bbox=((cx - r - 2, cx + r + 3), (cy - r - 2, cy + r + 3), (0, z1)))
    solid = np.broadcast_to(plane.solid[0], (nz, ny, nx)).copy()
    c = directions()
    cells, dirs, qs = [], [], []
    pc, pd, pq = plane.links
    pxy = pc % (nx * ny)
    for i in range(27):
        if i == 13:
            continue
        # planar links with any cz: the crossing fraction is set by the x-y motion
        sel_dir = [j for j in range(27) if c[j, 0] == c[i, 0] and c[j, 1] == c[i, 1] and c[j, 2] == 0]
        m = pd == sel_dir[0]
        if not m.any():
            continue
        for z in range(nz):
            if c[i, 2] != 0 and not (0 <= z + c[i, 2] < nz):
                continue
            cells.append(z * nx * ny + pxy[m])
            dirs.append(np.full(int(m.sum()), i, np.uint8))
            qs.append(pq[m])
    links = (np.concatenate(cells), np.concatenate(dirs), np.concatenate(qs))
    order = np.lexsort((links[1], links[0]))
    links = tuple(a[order] for a in links)
    return Geometry(shape=tuple(shape), solid=solid, links=links, frontal_area=diameter * nz, name="cylinder",
                    params=dict(center=center, diameter=diameter))


def obstacle_sdf(shape, seed, scale=None, turns=0, re=None, aoa=None):
    """Description and signed distance function of the seeded random object
    placed at (0.3 nx, (ny-1)/2, (nz-1)/2), turned by `turns` quarter turns
    about the channel axis (+y towards +z; needs ny == nz when turns != 0).
    re and aoa, when given, replace the seeded Reynolds number and angle of
    attack (degrees)."""
    nx, ny, nz = shape
    if scale is None:
        scale = nx / 256.0
    obj = random_object(seed, scale)
    if re is not None:
        obj["re"] = float(re)
    if aoa is not None:
        obj["aoa"] = float(aoa)
    center = np.array([0.3 * nx, (ny - 1) / 2.0, (nz - 1) / 2.0])
    base = object_sdf(obj, center)
    q = int(turns) % 4
    if q == 0:
        return obj, base, center, scale
    if ny != nz:
        raise ValueError("turns about x need ny == nz")
    cy, cz = center[1], center[2]

    def sdf(p):
        p = np.asarray(p, dtype=np.float64)
        y, z = p[..., 1] - cy, p[..., 2] - cz
        for _ in range(q):  # pull back: (y, z) -> (z, -y)
            y, z = z, -y
        return base(np.stack([p[..., 0], y + cy, z + cz], -1))

    return obj, sdf, center, scale


def random_obstacle(shape, seed, scale=None, turns=0, re=None, aoa=None):
    """Seeded union of 1-3 primitives at (0.3 nx, (ny-1)/2, (nz-1)/2); sizes
    refer to a 256x128x128 channel and scale with nx/256 unless given; re and
    aoa override the seeded values."""
    obj, sdf, center, scale = obstacle_sdf(shape, seed, scale, turns, re, aoa)
    ext = 24.0 * scale * 1.5 + 4.0 * scale * 1.8 + 3
    bb = tuple((center[d] - ext, center[d] + ext + 1) for d in range(3))
    g = from_sdf(shape, sdf, name=f"random{seed}" + (f"t{turns}" if turns else ""), params=obj, bbox=bb)
    return g
