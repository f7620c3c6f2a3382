"""Brute-force numpy variant of the lattice Boltzmann oracle (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

It pins ``oracle.lbm`` on small boxes by reaching the same step through
different mathematics:
  * central moments from raw moments by binomial shift (not the direct sum);
  * cumulants and their inverse by the generic set-partition formula
    kappa(X_1..X_n) = sum_pi (|pi|-1)! (-1)^(|pi|-1) prod_B E[prod_{i in B} X_i]
    (moments from cumulants: the same sum with all coefficients +1), with the
    first-order central moments taken as zero inside the products;
  * populations from moments by solving the 27x27 raw-moment system (LU);
  * streaming by explicit neighbour index tables.
The relaxation is the cumulant method's (Sec. 3.2 of the paper; plain mode
and the fourth-order parametrised mode with limiter), transcribed
independently of the C oracle.
"""
import itertools
import math
from functools import lru_cache

import numpy as np

W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}


def lattice():
    c = np.zeros((27, 3), dtype=np.int64)
    w = np.zeros(27)
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                i = 9 * (cz + 1) + 3 * (cy + 1) + (cx + 1)
                c[i] = (cx, cy, cz)
                w[i] = W1[cx] * W1[cy] * W1[cz]
    return c, w


C, WT = lattice()
EXPS = [(a, b, cc) for a in range(3) for b in range(3) for cc in range(3)]  # index 9a+3b+c
RAW = np.array([[C[i, 0] ** a * C[i, 1] ** b * C[i, 2] ** cc for i in range(27)] for (a, b, cc) in EXPS],
               dtype=np.float64)


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        yield [[first]] + part
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]


@lru_cache(maxsize=None)
def _partition_table(a, b, cc):
    """List of (coefficient, [exponent triples of blocks]) for moment index
    (a,b,c), partitions without singleton blocks."""
    var = [0] * a + [1] * b + [2] * cc
    out = []
    for part in _set_partitions(list(range(len(var)))):
        if any(len(B) == 1 for B in part):
            continue
        blocks = []
        for B in part:
            cnt = [0, 0, 0]
            for e in B:
                cnt[var[e]] += 1
            blocks.append(tuple(cnt))
        out.append((len(part), blocks))
    return out


def _idx(t):
    return 9 * t[0] + 3 * t[1] + t[2]


def cumulants_generic(k):
    """k: normalised central moments [27, M] -> cumulants [27, M]."""
    Cm = k.copy()
    for m, (a, b, cc) in enumerate(EXPS):
        if a + b + cc < 4:
            continue
        s = np.zeros_like(k[0])
        for nb, blocks in _partition_table(a, b, cc):
            coef = math.factorial(nb - 1) * (-1) ** (nb - 1)
            prod = np.ones_like(k[0])
            for t in blocks:
                prod = prod * k[_idx(t)]
            s = s + coef * prod
        Cm[m] = s
    return Cm


def moments_generic(Cm):
    """Cumulants [27, M] -> normalised central moments [27, M]."""
    k = Cm.copy()
    for m, (a, b, cc) in enumerate(EXPS):
        if a + b + cc < 4:
            continue
        s = np.zeros_like(Cm[0])
        for nb, blocks in _partition_table(a, b, cc):
            prod = np.ones_like(Cm[0])
            for t in blocks:
                prod = prod * Cm[_idx(t)]
            s = s + prod
        k[m] = s
    return k


def _shift(mom, u, sign):
    """Binomial shift of moments: sign=-1 raw->central, sign=+1 central->raw."""
    out = np.zeros_like(mom)
    for m, (a, b, cc) in enumerate(EXPS):
        s = np.zeros_like(mom[0])
        for p in range(a + 1):
            for q in range(b + 1):
                for r in range(cc + 1):
                    coef = math.comb(a, p) * math.comb(b, q) * math.comb(cc, r)
                    s = s + coef * (sign * u[0]) ** (a - p) * (sign * u[1]) ** (b - q) * (sign * u[2]) ** (cc - r) \
                        * mom[9 * p + 3 * q + r]
        out[m] = s
    return out


def k17_coefficients(w1, w2=1.0):
    w3 = 8 * (w1 - 2) * (w2 * (3 * w1 - 1) - 5 * w1) / (8 * (5 - 2 * w1) * w1 + w2 * (8 + w1 * (9 * w1 - 26)))
    w4 = 8 * (w1 - 2) * (w1 + w2 * (3 * w1 - 7)) / (w2 * (56 - 42 * w1 + 9 * w1 ** 2) - 8 * w1)
    w5 = 24 * (w1 - 2) * (4 * w1 ** 2 + w1 * w2 * (18 - 13 * w1) + w2 ** 2 * (2 + w1 * (6 * w1 - 11))) / (
        16 * w1 ** 2 * (w1 - 6) - 2 * w1 * w2 * (216 + 5 * w1 * (9 * w1 - 46))
        + w2 ** 2 * (w1 * (3 * w1 - 10) * (15 * w1 - 28) - 48))
    A = (4 * w1 ** 2 + 2 * w1 * w2 * (w1 - 6) + w2 ** 2 * (w1 * (10 - 3 * w1) - 4)) / (
        (w1 - w2) * (w2 * (2 + 3 * w1) - 8 * w1))
    B = (4 * w1 * w2 * (9 * w1 - 16) - 4 * w1 ** 2 - 2 * w2 ** 2 * (2 + 9 * w1 * (w1 - 2))) / (
        3 * (w1 - w2) * (w2 * (2 + 3 * w1) - 8 * w1))
    return np.array([w3, w4, w5, A, B])


def collide(fbar, omega1, omega2=1.0, mode=0, galilean=1, lam=0.01, force=(0, 0, 0), k17=None):
    """fbar [27, M] -> post-collision fbar [27, M]."""
    f = fbar + WT[:, None]
    raw = RAW @ f
    rho = raw[0]
    F = np.asarray(force, dtype=np.float64)
    u = [(raw[9] + 0.5 * F[0]) / rho, (raw[3] + 0.5 * F[1]) / rho, (raw[1] + 0.5 * F[2]) / rho]
    K = _shift(raw, u, -1.0)
    k = K / rho
    k1 = k.copy()
    for m in (9, 3, 1):
        k1[m] = 0.0
    Cm = cumulants_generic(k1)
    w1, w2 = omega1, omega2
    Cs = np.zeros_like(Cm)
    c200, c020, c002 = Cm[18], Cm[6], Cm[2]
    Dxu = -0.5 * w1 * (2 * c200 - c020 - c002) - 0.5 * w2 * (c200 + c020 + c002 - 1.0)
    Dyv = Dxu + 1.5 * w1 * (c200 - c020)
    Dzw = Dxu + 1.5 * w1 * (c200 - c002)
    G = float(galilean)
    m1, m2, a = c200 - c020, c200 - c002, c200 + c020 + c002
    ux2, uy2, uz2 = u[0] ** 2, u[1] ** 2, u[2] ** 2
    m1s = (1 - w1) * m1 - G * 3 * (1 - w1 / 2) * (ux2 * Dxu - uy2 * Dyv)
    m2s = (1 - w1) * m2 - G * 3 * (1 - w1 / 2) * (ux2 * Dxu - uz2 * Dzw)
    as_ = a + w2 * (1 - a) - G * 3 * (1 - w2 / 2) * (ux2 * Dxu + uy2 * Dyv + uz2 * Dzw)
    Cs[18] = (m1s + m2s + as_) / 3
    Cs[6] = (as_ - 2 * m1s + m2s) / 3
    Cs[2] = (as_ + m1s - 2 * m2s) / 3
    Cs[12] = (1 - w1) * Cm[12]  # 110
    Cs[10] = (1 - w1) * Cm[10]  # 101
    Cs[4] = (1 - w1) * Cm[4]    # 011
    if mode == 1:
        w3, w4, w5, A, B = k17 if k17 is not None else k17_coefficients(w1, w2)

        def lim(w, c):
            return w + (1 - w) * np.abs(c) / (lam + np.abs(c))

        for p_, q_ in ((_idx((1, 2, 0)), _idx((1, 0, 2))), (_idx((2, 1, 0)), _idx((0, 1, 2))),
                       (_idx((2, 0, 1)), _idx((0, 2, 1)))):
            s = Cm[p_] + Cm[q_]
            d = Cm[p_] - Cm[q_]
            ss = (1 - lim(w3, s)) * s
            ds = (1 - lim(w4, d)) * d
            Cs[p_] = 0.5 * (ss + ds)
            Cs[q_] = 0.5 * (ss - ds)
        c111 = Cm[_idx((1, 1, 1))]
        Cs[_idx((1, 1, 1))] = (1 - lim(w5, c111)) * c111
        t = 1 / w1 - 0.5
        Cs[_idx((2, 2, 0))] = -(2 / 3) * t * A * (Dxu + Dyv)
        Cs[_idx((2, 0, 2))] = -(2 / 3) * t * A * (Dxu + Dzw)
        Cs[_idx((0, 2, 2))] = -(2 / 3) * t * A * (Dyv + Dzw)
        Cs[_idx((2, 1, 1))] = -(1 / 3) * t * B * (-3 * w1 * Cm[4])
        Cs[_idx((1, 2, 1))] = -(1 / 3) * t * B * (-3 * w1 * Cm[10])
        Cs[_idx((1, 1, 2))] = -(1 / 3) * t * B * (-3 * w1 * Cm[12])
    ks = moments_generic(Cs)
    Ks = rho * ks
    Ks[0] = rho
    Ks[9], Ks[3], Ks[1] = -K[9], -K[3], -K[1]
    raws = _shift(Ks, u, +1.0)
    fs = np.linalg.solve(RAW, raws)
    return fs - WT[:, None]


def equilibrium(rho, u):
    """Discrete equilibrium from its central moments: Gaussian moments
    (rho/3 per squared direction, products thereof), all others zero."""
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    M = rho.size
    K = np.zeros((27, M))
    for m, (a, b, cc) in enumerate(EXPS):
        if a % 2 == 0 and b % 2 == 0 and cc % 2 == 0:
            K[m] = rho * (1 / 3) ** ((a + b + cc) // 2)
    u = [np.broadcast_to(np.asarray(u[d], dtype=np.float64), (M,)) for d in range(3)]
    raw = _shift(K, u, +1.0)
    return np.linalg.solve(RAW, raw) - WT[:, None]


def run(shape, nsteps, fbar, omega1, periodic=(1, 1, 1), solid=None, u_in=0.0, mode=0, galilean=1, lam=0.01,
        omega2=1.0, force=(0, 0, 0)):
    """Two-lattice run with halfway bounce-back at walls/obstacle, moving-wall
    inlet at x=-1/2 and zero-gradient outlet.  fbar [27, nz, ny, nx]."""
    nx, ny, nz = shape
    fb = fbar.reshape(27, -1).copy()
    N = nx * ny * nz
    sol = np.zeros(N, bool) if solid is None else np.asarray(solid, bool).reshape(-1)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xx, yy, zz = xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)
    fluid = ~sol
    # source tables: (kind, index) per direction
    tables = []
    for i in range(27):
        sx, sy, sz = xx - C[i, 0], yy - C[i, 1], zz - C[i, 2]
        kind = np.zeros(N, np.int64)  # 0 fluid, 1 bounce, 2 inlet
        if periodic[1]:
            sy = sy % ny
        else:
            kind[(sy < 0) | (sy >= ny)] = 1
        if periodic[2]:
            sz = sz % nz
        else:
            kind[(sz < 0) | (sz >= nz)] = 1
        if periodic[0]:
            sx = sx % nx
        else:
            kind[(kind == 0) & (sx < 0)] = 2
            sx = np.minimum(sx, nx - 1)
        sxc, syc, szc = np.clip(sx, 0, nx - 1), np.clip(sy, 0, ny - 1), np.clip(sz, 0, nz - 1)
        src = (szc * ny + syc) * nx + sxc
        kind[(kind == 0) & sol[src]] = 1
        tables.append((kind, src))
    for _ in range(nsteps):
        post = np.zeros_like(fb)
        post[:, fluid] = collide(fb[:, fluid], omega1, omega2, mode, galilean, lam, force)
        nxt = np.zeros_like(fb)
        for i in range(27):
            kind, src = tables[i]
            o = 26 - i
            v = np.where(kind == 0, post[i, src], post[o])
            v = np.where(kind == 2, post[o] + 6 * WT[i] * C[i, 0] * u_in, v)
            nxt[i] = np.where(fluid, v, 0.0)
        fb = nxt
    return fb.reshape(fbar.shape)


__all__ = ["lattice", "collide", "equilibrium", "run", "cumulants_generic", "moments_generic", "k17_coefficients",
           "RAW", "C", "WT", "EXPS"]

if __name__ == "__main__":
    print(len(_partition_table(2, 2, 2)))
    print(list(itertools.islice(_set_partitions([0, 1, 2]), 10)))
