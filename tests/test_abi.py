"""C ABI: the library loads and exports every symbol the header declares;
argument validation answers with error codes before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mi355lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*((?:lbm|fno|unet)_[a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_path_entry_points():
    names = header_functions()
    for n in ("lbm_create", "lbm_step", "lbm_mean_fields", "fno_forward", "fno_train_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_16765_amd._lib import load
    L = load()
    missing = [n for n in header_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_invalid_parameters_rejected_without_device_work():
    from paper_2606_16765_amd._lib import LbmParams, load
    L = load()
    p = LbmParams()
    L.lbm_default_params(ctypes.byref(p), 63, 32, 32)
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(p), None, 0, None, None, None, None, None, ctypes.byref(h)) == 1
    assert b"nx % 64" in L.lbm_last_error(None)
    L.lbm_default_params(ctypes.byref(p), 64, 32, 32)
    p.nu = -1.0
    assert L.lbm_create(ctypes.byref(p), None, 0, None, None, None, None, None, ctypes.byref(h)) == 1
    L.lbm_default_params(ctypes.byref(p), 64, 32, 32)
    p.storage = 7
    assert L.lbm_create(ctypes.byref(p), None, 0, None, None, None, None, None, ctypes.byref(h)) == 1
    assert L.lbm_step(None, 1) == 1
    ms = ctypes.c_double()
    assert L.lbm_bandwidth_probe(None, 2, ctypes.byref(ms)) == 1
    assert L.lbm_get_populations_box(None, 0, 0, 0, 1, 1, 1, None) == 1
    assert L.lbm_mean_fields_pooled(None, 2, 0, None) == 1
    lo = (ctypes.c_float * 4)()
    assert L.fno_field_minmax(None, 1, 1, 1, None, lo, lo) == 1
    assert L.fno_field_scale(None, 1, 1, 1, lo, lo, 0, None) == 1
    fp = __import__("paper_2606_16765_amd._lib", fromlist=["FnoParams"]).FnoParams()
    fp.nx, fp.ny, fp.nz, fp.cin, fp.cout, fp.width, fp.layers = 48, 16, 16, 4, 4, 16, 1
    fp.mx = fp.my = fp.mz = 4
    fp.proj_hidden, fp.max_batch = 16, 1
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # 48 is not a power of two
    assert b"powers of two" in L.fno_last_error(None)
    fp.nx = 64
    fp.width = 80
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # wider than the mixing kernels
    assert b"at most 64" in L.fno_last_error(None)
    fp.width, fp.my, fp.mz = 16, 2, 4
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # 2 my mz = 16 < 32
    assert b"2 my mz" in L.fno_last_error(None)
    fp.my = 4
    fp.proj_act = 2
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"proj_act" in L.fno_last_error(None)
    fp.proj_act, fp.proj_w0 = 1, 0.0
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # sine needs w0 > 0
    assert b"sine projection" in L.fno_last_error(None)
    fp.proj_act, fp.proj_w0 = 0, 30.0
    fp.arch = 3
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"arch must be" in L.fno_last_error(None)
    # factorized FNO: nz 16 (< 32), 2 modes, width 48
    fp.arch, fp.ff_hidden = 2, 32
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"factorized FNO needs 4 to 16 modes" in L.fno_last_error(None)
    fp.nz, fp.mz = 32, 2
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"factorized FNO needs 4 to 16 modes" in L.fno_last_error(None)
    fp.mz, fp.width = 4, 48
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"width 16 or 32" in L.fno_last_error(None)
    fp.nz = 16
    fp.arch, fp.ff_hidden, fp.width = 1, 32, 48
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # hybrid width above 32
    assert b"hybrid" in L.fno_last_error(None)
    fp.width, fp.ff_hidden = 16, 160
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # feed-forward wider than 128
    assert b"hybrid" in L.fno_last_error(None)


def test_hybrid_parameter_count_matches_the_oracle_layout():
    """fno_param_count (host only) for the three architectures against the
    oracle's parameter layout."""
    from oracle import fno as ofno
    from paper_2606_16765_amd._lib import FnoParams, load
    L = load()
    for arch, code in (("fno", 0), ("hybrid", 1), ("ffno", 2)):
        fp = FnoParams()
        fp.nx, fp.ny, fp.nz, fp.cin, fp.cout, fp.width, fp.layers = 128, 64, 64, 4, 4, 32, 4
        fp.mx, fp.my, fp.mz, fp.proj_hidden, fp.max_batch = 16, 16, 16, 128, 1
        fp.arch, fp.ff_hidden = code, 96
        assert L.fno_param_count(ctypes.byref(fp)) == ofno.param_count(ofno.Shape(arch=arch, ff_hidden=96))


def test_binding_raises_on_error():
    import paper_2606_16765_amd as P
    from paper_2606_16765_amd._lib import HipError
    with pytest.raises(HipError):
        P.Lbm((63, 8, 8), nu=0.01)


def _params(shape, **kw):
    from paper_2606_16765_amd._lib import LbmParams, load
    L = load()
    p = LbmParams()
    L.lbm_default_params(ctypes.byref(p), *shape)
    for k, v in kw.items():
        setattr(p, k, v)
    return L, p


def test_fourth_order_mode_rejected_where_its_rates_are_undefined():
    """A and B of the fourth-order mode carry 1/(omega1 - omega2): at
    nu = 1/6 (omega1 = 1 = omega2) lbm_create answers LBM_EINVAL before any
    device work, and so it does where a third-order rate leaves (0, 2)
    (omega1 = 1.5 gives omega4 = 3.2).  Plain mode at the same viscosity is
    not rejected by this rule (lbm_workspace_size, host only, accepts it)."""
    h = ctypes.c_void_p()
    for nu in (1.0 / 6.0, (1 / 1.5 - 0.5) / 3):
        L, p = _params((64, 8, 8), nu=nu, mode=1)
        assert L.lbm_create(ctypes.byref(p), None, 0, None, None, None, None, None, ctypes.byref(h)) == 1
        assert b"fourth-order mode undefined" in L.lbm_last_error(None)
        n = ctypes.c_size_t()
        assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 1
        p.mode = 0
        assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 0
    # the production range (omega1 near 2) is accepted
    L, p = _params((64, 8, 8), nu=0.05 * 8 / 3900, mode=1)
    n = ctypes.c_size_t()
    assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 0


def test_reynolds_number_maps_to_viscosity_in_the_library():
    """re > 0 makes the library derive nu = u_in l_ref / re, and that nu
    decides the automatic switch at Re_c = u_in ny / nu = 3000.  With
    l_ref = ny and u_in = re / 48 on ny = 8 the derived nu is 1/6, where the
    fourth-order mode has a pole (omega1 = 1 = omega2): re = 3000 resolves
    to that mode and is rejected, re = 2990 resolves to the plain mode and
    is accepted (host-only checks through lbm_workspace_size)."""
    n = ctypes.c_size_t()
    for re_, rc in ((3000.0, 1), (2990.0, 0)):
        L, p = _params((64, 8, 8), re=re_, l_ref=8.0, u_in=re_ / 48.0, nu=0.01)  # nu ignored when re > 0
        assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == rc, re_
    # l_ref <= 0 means the channel height
    L, p = _params((64, 8, 8), re=3000.0, l_ref=0.0, u_in=3000.0 / 48.0)
    assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 1
    L, p = _params((64, 8, 8), re=1000.0, u_in=0.0)
    assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 1
    assert b"re needs u_in" in L.lbm_last_error(None)


def test_workspace_size_counts_every_region():
    """lbm_workspace_size: two population lattices in the padded layout
    (27 slots of nx + 64 per padded row, ny + 2 rows, nz + 2 planes),
    each behind a 256-byte guard, flags, rows, tables, accumulators (32 B
    per cell), snapshot ring (16 B per cell per snapshot), each region
    rounded up to 256 bytes."""
    import numpy as np
    shape = (128, 16, 8)
    nx, ny, nz = shape
    N = nx * ny * nz
    r256 = lambda b: (b + 255) // 256 * 256  # noqa: E731
    base = lambda es, nb: (2 * (256 + r256(27 * (nx + 64) * (ny + 2) * (nz + 2) * es)) + r256(N) + r256(4 * N)  # noqa: E731
                           + r256(4 * max(nb, 1)) + r256(216 * max(nb, 1)) + 256)
    n = ctypes.c_size_t()
    L, p = _params(shape, avg_start=-1, force_every=0)
    assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 0
    assert n.value == base(4, 0)
    L, p = _params(shape, storage=0, avg_start=0, snap_every=25, snap_count=3, force_every=0)
    assert L.lbm_workspace_size(ctypes.byref(p), None, ctypes.byref(n)) == 0
    assert n.value == base(8, 0) + r256(32 * N) + r256(3 * 16 * N)
    # one solid cell far from the faces: 26 fluid neighbours, all in one
    # x tile and 2 y tiles (3 z planes) -> slots in 6 tiles
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[4, 8, 40] = 1
    L, p = _params(shape, avg_start=-1, force_every=1, force_capacity=10)
    assert L.lbm_workspace_size(ctypes.byref(p), solid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)) == 0
    tiles = (nx // 64) * (ny // 2) * nz
    assert n.value == base(4, 26) + r256(4 * tiles) + r256(24 * 6) + r256(24 * 10)


def test_product_package_does_not_load_the_oracle():
    """The product package never imports, loads or runs anything under
    oracle/: only the tests, the smoke check and the benchmark's CPU
    baseline do."""
    pkg = os.path.join(ROOT, "paper_2606_16765_amd")
    bad = []
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                if re.search(r"^\s*(from\s+oracle\b|import\s+oracle\b)|lbm_oracle|_lbm_oracle", txt, flags=re.M):
                    bad.append(f)
    assert not bad, bad
