"""Python binding of the lattice Boltzmann part of the C ABI (argument
marshalling only; every step of the path runs in the HIP library).

Fields come back as numpy arrays in the natural layout ([k][nz][ny][nx]), or
land in caller-provided torch CUDA tensors when ``out`` is given.
"""
import ctypes

import numpy as np

from ._lib import LbmParams, check, load

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
MODES = {"auto": -1, "plain": 0, "k17": 1}


def nu_from_re(u_in, length, re):
    """Lattice viscosity for Reynolds number re on a length in cells at
    inlet velocity u_in (paper Sec. 3.1: Re set through the viscosity)."""
    return u_in * length / re


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Lbm:
    """D3Q27 cumulant lattice Boltzmann solver on one GPU."""

    def __init__(self, shape, storage="f32", periodic=(0, 0, 0), u_in=0.05, nu=None, re=None, l_ref=None,
                 omega2=1.0, mode="auto", galilean=1, lam=0.01, obstacle_bc=0, body_force=(0.0, 0.0, 0.0),
                 avg_start=0, snap_every=0, snap_count=20, snap_start=0, force_every=1, xcd_remap=1, solid=None,
                 links=None, u0=None, perturb=None, stream=None, check_every=0, force_capacity=0,
                 workspace=None):
        """shape (nx, ny, nz); give the viscosity nu, or re (and l_ref, in
        cells, default the channel height ny) for the library to derive it.
        workspace: a caller-owned CUDA tensor of at least
        ``Lbm.workspace_size(...)`` bytes that holds all device state (needs
        force_capacity > 0 when forces are on); kept referenced by the
        object."""
        L = load()
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        if nu is None and re is None:
            raise ValueError("give nu or re")
        p = LbmParams()
        L.lbm_default_params(ctypes.byref(p), nx, ny, nz)
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        for d in range(3):
            p.periodic[d] = int(periodic[d])
            p.body_force[d] = float(body_force[d])
        p.u_in, p.omega2 = float(u_in), float(omega2)
        if re is not None:
            p.re, p.l_ref = float(re), float(l_ref or 0.0)
        else:
            p.nu = float(nu)
        p.check_every, p.force_capacity = int(check_every), int(force_capacity)
        p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        p.galilean, p.lam, p.obstacle_bc = int(galilean), float(lam), int(obstacle_bc)
        p.avg_start = -1 if avg_start is None else int(avg_start)
        p.snap_every, p.snap_count, p.snap_start = int(snap_every), int(snap_count), int(snap_start)
        p.force_every, p.xcd_remap = int(force_every), int(xcd_remap)
        if perturb is not None:
            # (seed, amplitude): the library draws the initial velocity itself
            p.perturb_seed, p.perturb_amp = int(perturb[0]), float(perturb[1])
        self.params = p
        self.storage = storage
        keep = []
        sol = None
        if solid is not None:
            sol = np.ascontiguousarray(np.asarray(solid).reshape(-1), dtype=np.uint8)
            assert sol.size == self.N
            keep.append(sol)
        nl, lc, ld, lq = 0, None, None, None
        if links is not None and len(links[0]) > 0:
            lc = np.ascontiguousarray(links[0], dtype=np.int64)
            ld = np.ascontiguousarray(links[1], dtype=np.uint8)
            lq = np.ascontiguousarray(links[2], dtype=np.float64)
            nl = lc.size
            keep += [lc, ld, lq]
        u = None
        if u0 is not None:
            u = np.ascontiguousarray(np.asarray(u0, dtype=np.float64).reshape(3, -1))
            assert u.shape[1] == self.N
            keep.append(u)
        h = ctypes.c_void_p()
        self._L = L
        self._h = None
        self._workspace = workspace
        ws, wsb = None, 0
        if workspace is not None:
            ws = ctypes.c_void_p(workspace.data_ptr())
            wsb = workspace.numel() * workspace.element_size()
        rc = L.lbm_create_in(ctypes.byref(p), None if sol is None else _ptr(sol), nl,
                             None if lc is None else _ptr(lc), None if ld is None else _ptr(ld),
                             None if lq is None else _ptr(lq), None if u is None else _ptr(u), ws, wsb,
                             _stream_handle(stream), ctypes.byref(h))
        check(rc, None, "lbm_create_in" if workspace is not None else "lbm_create")
        self._h = h

    @staticmethod
    def params_struct(shape, **kw):
        """The lbm_params the constructor would pass (for workspace sizing)."""
        L = load()
        nx, ny, nz = (int(v) for v in shape)
        p = LbmParams()
        L.lbm_default_params(ctypes.byref(p), nx, ny, nz)
        for k, v in kw.items():
            if k == "storage":
                v = STORAGE[v] if isinstance(v, str) else int(v)
            elif k == "mode":
                v = MODES[v] if isinstance(v, str) else int(v)
            elif k == "avg_start" and v is None:
                v = -1
            if k in ("periodic", "body_force"):
                for d in range(3):
                    getattr(p, k)[d] = v[d]
            else:
                setattr(p, k, v)
        return p

    @staticmethod
    def workspace_size(shape, solid=None, **kw):
        """Bytes lbm_workspace_size reports for these parameters (keyword
        names of lbm_params) and solid mask; host work only."""
        L = load()
        p = Lbm.params_struct(shape, **kw)
        sol = None
        if solid is not None:
            sol = np.ascontiguousarray(np.asarray(solid).reshape(-1), dtype=np.uint8)
        n = ctypes.c_size_t()
        check(L.lbm_workspace_size(ctypes.byref(p), None if sol is None else _ptr(sol), ctypes.byref(n)), None,
              "lbm_workspace_size")
        return n.value

    # ------------------------------------------------------------------
    def close(self):
        if self._h is not None:
            self._L.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc, what):
        check(rc, self._h, what)

    def _fshape(self, k):
        nx, ny, nz = self.shape
        return (k, nz, ny, nx)

    # ------------------------------------------------------------------
    def step(self, n=1):
        self._chk(self._L.lbm_step(self._h, int(n)), "lbm_step")
        return self

    def info(self):
        s, w, m = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
        self._chk(self._L.lbm_info(self._h, ctypes.byref(s), ctypes.byref(w), ctypes.byref(m)), "lbm_info")
        return dict(steps=s.value, omega1=w.value, mode=m.value)

    def mean_fields(self, out=None):
        """(u, v, w, p) means [4][nz][ny][nx] (double) and the sample count."""
        n = ctypes.c_int64()
        if out is not None:
            self._chk(self._L.lbm_mean_fields(self._h, ctypes.c_void_p(out.data_ptr()), 1, ctypes.byref(n)),
                      "lbm_mean_fields")
            return out, n.value
        a = np.empty(self._fshape(4))
        self._chk(self._L.lbm_mean_fields(self._h, _ptr(a), 0, ctypes.byref(n)), "lbm_mean_fields")
        return a, n.value

    def mean_fields_pooled(self, factor=2, quarter_turns=0, out=None):
        """Means pooled over factor^3 blocks, device float [4][X][Y][Z]
        (Z fastest), optionally turned about +x; asynchronous."""
        import torch
        nx, ny, nz = self.shape
        if out is None:
            out = torch.empty((4, nx // factor, ny // factor, nz // factor), dtype=torch.float32, device="cuda")
        assert out.dtype == torch.float32 and out.is_cuda and out.is_contiguous()
        assert out.numel() == 4 * (nx // factor) * (ny // factor) * (nz // factor)
        self._chk(self._L.lbm_mean_fields_pooled(self._h, factor, quarter_turns, ctypes.c_void_p(out.data_ptr())),
                  "lbm_mean_fields_pooled")
        return out

    def bandwidth_probe(self, passes=20):
        """Average ms of one pass that moves the even step's traffic (27
        slots loaded and stored per cell) without the collision; passes must
        be even and leave the state unchanged."""
        ms = ctypes.c_double()
        self._chk(self._L.lbm_bandwidth_probe(self._h, int(passes), ctypes.byref(ms)), "lbm_bandwidth_probe")
        return ms.value

    def snapshots(self):
        k = ctypes.c_int32()
        self._chk(self._L.lbm_snapshots(self._h, None, 0, ctypes.byref(k), None), "lbm_snapshots")
        out = np.empty((k.value,) + self._fshape(4), np.float32)
        steps = np.empty(k.value, np.int64)
        if k.value:
            self._chk(self._L.lbm_snapshots(self._h, _ptr(out), 0, ctypes.byref(k), _ptr(steps)), "lbm_snapshots")
        return out, steps

    def forces(self):
        n = ctypes.c_int64()
        self._chk(self._L.lbm_forces(self._h, None, 0, ctypes.byref(n), None), "lbm_forces")
        out = np.empty((n.value, 3))
        steps = np.empty(n.value, np.int64)
        if n.value:
            self._chk(self._L.lbm_forces(self._h, _ptr(out), n.value, ctypes.byref(n), _ptr(steps)), "lbm_forces")
        return out, steps

    def moments(self, out=None):
        if out is not None:
            self._chk(self._L.lbm_moments(self._h, ctypes.c_void_p(out.data_ptr()), 1), "lbm_moments")
            return out
        a = np.empty(self._fshape(4), np.float32)
        self._chk(self._L.lbm_moments(self._h, _ptr(a), 0), "lbm_moments")
        return a

    def populations(self):
        a = np.empty(self._fshape(27))
        self._chk(self._L.lbm_get_populations(self._h, _ptr(a)), "lbm_get_populations")
        return a

    def populations_box(self, origin, size):
        """Pre-collision populations of the cells of one box, natural layout,
        double [27][bz][by][bx]; origin (x0, y0, z0), size (bx, by, bz)."""
        (x0, y0, z0), (bx, by, bz) = origin, size
        a = np.empty((27, bz, by, bx))
        self._chk(self._L.lbm_get_populations_box(self._h, x0, y0, z0, bx, by, bz, _ptr(a)),
                  "lbm_get_populations_box")
        return a

    def set_populations(self, fbar):
        a = np.ascontiguousarray(fbar, dtype=np.float64)
        assert a.size == 27 * self.N
        self._chk(self._L.lbm_set_populations(self._h, _ptr(a)), "lbm_set_populations")

    def mass(self):
        m = ctypes.c_double()
        self._chk(self._L.lbm_mass(self._h, ctypes.byref(m)), "lbm_mass")
        return m.value

    def export_state(self):
        n = ctypes.c_size_t()
        self._chk(self._L.lbm_export_state(self._h, None, 0, ctypes.byref(n)), "lbm_export_state")
        buf = np.empty(n.value, np.uint8)
        self._chk(self._L.lbm_export_state(self._h, _ptr(buf), n.value, ctypes.byref(n)), "lbm_export_state")
        return buf

    def import_state(self, blob):
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        self._chk(self._L.lbm_import_state(self._h, _ptr(b), b.size), "lbm_import_state")

    def profile(self, enable=True):
        self._chk(self._L.lbm_profile(self._h, int(bool(enable))), "lbm_profile")

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._chk(self._L.lbm_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)), "lbm_profile_read")
        return ms.value, n.value


def copy_bandwidth(nbytes=4 * 2 ** 30, passes=10, stream=None):
    """GB/s (read + write) of the library's plain streaming copy of nbytes
    between two device buffers: the attainable-bandwidth reference."""
    L = load()
    ms = ctypes.c_double()
    check(L.lbm_copy_bandwidth(int(nbytes), int(passes), _stream_handle(stream), ctypes.byref(ms)), None,
          "lbm_copy_bandwidth")
    return 2.0 * nbytes / (ms.value / 1e3) / 1e9


def bytes_per_cell_update(storage, averaging=False):
    """Algorithmic HBM bytes of one cell update: 27 reads and 27 writes of the
    stored population type, one flag byte, and with averaging a read-modify-
    write of four FP64 accumulators."""
    s = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]
    return 2 * 27 * s + 1 + (64 if averaging else 0)
