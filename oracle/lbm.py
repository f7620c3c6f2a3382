"""ctypes wrapper of the FP64 lattice Boltzmann oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Arrays use the natural layout ``[27][nz][ny][nx]`` (x fastest) for shifted
populations ``fbar = f - w_i`` and ``[4][nz][ny][nx]`` for (u, v, w, p) fields.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("omega1", ctypes.c_double), ("omega2", ctypes.c_double),
        ("mode", ctypes.c_int32), ("galilean", ctypes.c_int32),
        ("lam", ctypes.c_double),
        ("k17_given", ctypes.c_int32), ("k17", ctypes.c_double * 5),
        ("u_in", ctypes.c_double), ("force", ctypes.c_double * 3),
        ("obstacle_bc", ctypes.c_int32), ("emulate", ctypes.c_int32),
        ("avg_start", ctypes.c_int32), ("snap_every", ctypes.c_int32), ("snap_start", ctypes.c_int32),
    ]


EMULATE = {None: 0, "none": 0, "f32": 1, "f16": 2, "bf16": 3}


def lib():
    global _LIB
    if _LIB is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.orc_init.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, dp]
        L.orc_collide.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_void_p]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_central_moments.argtypes = [dp, dp, dp]
        L.orc_populations_from_central.argtypes = [dp, dp, dp]
        L.orc_cumulants.argtypes = [dp, dp]
        L.orc_moments_from_cumulants.argtypes = [dp, dp]
        L.orc_k17_coefficients.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), dp]
        L.orc_round.restype = ctypes.c_double
        L.orc_round.argtypes = [ctypes.c_double, ctypes.c_int32]
        L.orc_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def omega_from_nu(nu):
    """omega1 = 1/(3 nu + 1/2): the shear rate that gives lattice viscosity nu."""
    return 1.0 / (3.0 * nu + 0.5)


def make_params(shape, periodic=(0, 0, 0), nu=None, omega1=None, omega2=1.0, mode=0, galilean=1, lam=0.01,
                k17=None, u_in=0.0, force=(0.0, 0.0, 0.0), obstacle_bc=0, emulate=None, avg_start=0,
                snap_every=0, snap_start=0):
    """shape = (nx, ny, nz).  Give either nu or omega1."""
    if omega1 is None:
        omega1 = omega_from_nu(nu)
    p = Params()
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    for d in range(3):
        p.periodic[d] = int(periodic[d])
        p.force[d] = float(force[d])
    p.omega1, p.omega2 = float(omega1), float(omega2)
    p.mode, p.galilean, p.lam = int(mode), int(galilean), float(lam)
    if k17 is not None:
        p.k17_given = 1
        for i in range(5):
            p.k17[i] = float(k17[i])
    p.u_in = float(u_in)
    p.obstacle_bc = int(obstacle_bc)
    p.emulate = EMULATE[emulate]
    p.avg_start, p.snap_every, p.snap_start = int(avg_start), int(snap_every), int(snap_start)
    return p


def lattice():
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    lib().orc_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w))
    return c, w


def equilibrium(rho, u):
    out = np.zeros(27)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def central_moments(f, u):
    """K[9a+3b+c] = sum_i f_i (cx-u)^a (cy-v)^b (cz-w)^c (unshifted f)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    K = np.zeros(27)
    lib().orc_central_moments(_dp(f), _dp(u), _dp(K))
    return K


def populations_from_central(K, u):
    K = np.ascontiguousarray(K, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(27)
    lib().orc_populations_from_central(_dp(K), _dp(u), _dp(f))
    return f


def cumulants(k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    C = np.zeros(27)
    lib().orc_cumulants(_dp(k), _dp(C))
    return C


def moments_from_cumulants(C):
    C = np.ascontiguousarray(C, dtype=np.float64)
    k = np.zeros(27)
    lib().orc_moments_from_cumulants(_dp(C), _dp(k))
    return k


def k17_coefficients(omega1, omega2=1.0):
    out = np.zeros(5)
    lib().orc_k17_coefficients(float(omega1), float(omega2), _dp(out))
    return out


def collide(p, fbar):
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    out = np.zeros(27)
    lib().orc_collide(ctypes.byref(p), _dp(fbar), _dp(out), None)
    return out


def round_storage(v, fmt):
    return lib().orc_round(float(v), EMULATE[fmt])


def threads():
    return lib().orc_threads()


def init(p, solid=None, rho0=None, u0=None):
    """Equilibrium initial state f_eq(rho0, u0) - w (rho0 = 1, u0 = 0 if None)."""
    N = p.nx * p.ny * p.nz
    fbar = np.zeros((27, p.nz, p.ny, p.nx))
    s = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    assert s is None or s.size == N
    assert u is None or u.size == 3 * N
    lib().orc_init(ctypes.byref(p), None if s is None else s.ctypes.data, None if r is None else r.ctypes.data,
                   None if u is None else u.ctypes.data, _dp(fbar))
    return fbar


def dense_q(shape, links):
    """Dense [27][nz][ny][nx] wall-distance array from a sparse link list
    (cell, direction, q); unused entries are 0.5."""
    nx, ny, nz = shape
    q = np.full((27, nz * ny * nx), 0.5)
    if links is not None:
        cell, d, qq = links
        q[np.asarray(d, np.int64), np.asarray(cell, np.int64)] = qq
    return q.reshape(27, nz, ny, nx)


class Run:
    """Stateful oracle run: keeps the populations, the mean accumulators, the
    force series and the snapshots across calls to ``step``."""

    def __init__(self, p, solid=None, links=None, u0=None, rho0=None, fbar=None):
        self.p = p
        self.shape = (p.nx, p.ny, p.nz)
        N = p.nx * p.ny * p.nz
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(p.nz, p.ny, p.nx)
        self.q = dense_q(self.shape, links) if (links is not None and p.obstacle_bc == 1) else None
        self.fbar = init(p, self.solid, rho0, u0) if fbar is None else np.ascontiguousarray(fbar, dtype=np.float64).copy()
        self.acc = np.zeros((4, N))
        self.count = 0
        self.steps = 0
        self.forces = []
        self.snaps = []

    def step(self, n, forces=True, snap_cap=0):
        p = self.p
        N = p.nx * p.ny * p.nz
        cnt = ctypes.c_int64(self.count)
        fo = np.zeros((max(n, 1), 3)) if forces else None
        sn = np.zeros((snap_cap, 4, N)) if snap_cap > 0 else None
        ns = ctypes.c_int32(0)
        rc = lib().orc_run(ctypes.byref(p), None if self.solid is None else self.solid.ctypes.data,
                           None if self.q is None else self.q.ctypes.data, _dp(self.fbar), int(self.steps), int(n),
                           self.acc.ctypes.data, ctypes.byref(cnt), None if fo is None else fo.ctypes.data,
                           None if sn is None else sn.ctypes.data, int(snap_cap), ctypes.byref(ns))
        if rc != 0:
            raise RuntimeError(f"oracle run failed with code {rc}")
        self.count = cnt.value
        self.steps += n
        if forces:
            self.forces.extend(list(fo[:n]))
        if sn is not None:
            self.snaps.extend(list(sn[: ns.value]))
        return self

    def mean_fields(self):
        """(u, v, w, p) means over the sampled steps; zero in solid cells."""
        if self.count == 0:
            return np.zeros((4, self.p.nz, self.p.ny, self.p.nx))
        return (self.acc / self.count).reshape(4, self.p.nz, self.p.ny, self.p.nx)

    def macroscopic(self):
        """Instantaneous (rho, u, v, w) of the current state."""
        c, _ = lattice()
        f = self.fbar.reshape(27, -1)
        d = f.sum(0)
        rho = 1.0 + d
        F = np.array([self.p.force[0], self.p.force[1], self.p.force[2]])
        u = (c.T.astype(np.float64) @ f + 0.5 * F[:, None]) / rho
        shp = (self.p.nz, self.p.ny, self.p.nx)
        return rho.reshape(shp), u.reshape((3,) + shp)


def threads_used():
    return threads()


def available():
    try:
        lib()
        return True
    except (OSError, Exception):
        return False


__all__ = ["Params", "make_params", "Run", "lattice", "equilibrium", "central_moments", "populations_from_central",
           "cumulants", "moments_from_cumulants", "k17_coefficients", "collide", "init", "round_storage",
           "omega_from_nu", "dense_q", "threads", "available"]

if __name__ == "__main__":
    print(os.path.abspath(lib()._name))
