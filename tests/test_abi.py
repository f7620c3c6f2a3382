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
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*((?:lbm|fno)_[a-z_0-9]+)\s*\(", txt, flags=re.M)
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
    fp.arch = 2
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1
    assert b"arch must be" in L.fno_last_error(None)
    fp.arch, fp.ff_hidden, fp.width = 1, 32, 48
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # hybrid width above 32
    assert b"hybrid" in L.fno_last_error(None)
    fp.width, fp.ff_hidden = 16, 160
    assert L.fno_create(ctypes.byref(fp), 0, None, ctypes.byref(h)) == 1  # feed-forward wider than 128
    assert b"hybrid" in L.fno_last_error(None)


def test_hybrid_parameter_count_matches_the_oracle_layout():
    """fno_param_count (host only) for both architectures against the
    oracle's parameter layout."""
    from oracle import fno as ofno
    from paper_2606_16765_amd._lib import FnoParams, load
    L = load()
    for arch, code in (("fno", 0), ("hybrid", 1)):
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
