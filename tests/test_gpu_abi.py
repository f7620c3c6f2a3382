"""GPU checks of the C ABI's run-time services: the stability check
(check_every -> sticky LBM_EUNSTABLE), the caller workspace
(lbm_workspace_size / lbm_create_in), the force ring and the Reynolds
number mapped to the viscosity in the library."""
import numpy as np
import pytest

from inputs import perturbation, sphere_channel

pytestmark = pytest.mark.gpu


def _P():
    import paper_2606_16765_amd as P
    return P


def test_check_every_flags_an_injected_nan_within_the_period():
    """A NaN written into one fluid cell through lbm_set_populations is
    found by the next check step (steps 5, 10, ... for check_every = 5):
    once the stream has drained, lbm_step(0) and every readout return the
    sticky LBM_EUNSTABLE.  The same run without the NaN passes many
    checks."""
    import torch
    P = _P()
    from paper_2606_16765_amd._lib import HipError
    shape = (64, 8, 8)
    u0 = perturbation(shape, 5, 5e-4)
    ok = P.Lbm(shape, storage="f32", nu=0.02, u0=u0, check_every=5, avg_start=None)
    ok.step(50)
    torch.cuda.synchronize()
    ok.step(0)
    ok.mass()
    bad = P.Lbm(shape, storage="f32", nu=0.02, u0=u0, check_every=5, avg_start=None)
    bad.step(3)
    f = bad.populations()
    f[4, 3, 4, 20] = np.nan
    bad.set_populations(f)
    bad.step(5)          # steps 3..7: the check runs on step index 4
    torch.cuda.synchronize()
    with pytest.raises(HipError) as e:
        bad.step(0)
    assert e.value.code == 4 and "check step" in str(e.value)
    with pytest.raises(HipError) as e:
        bad.forces()
    assert e.value.code == 4


def test_check_every_flags_a_runaway_velocity():
    """A finite state moving at the lattice sound speed is flagged too."""
    import torch
    P = _P()
    from paper_2606_16765_amd._lib import HipError
    shape = (64, 8, 8)
    g = P.Lbm(shape, storage="f64", nu=0.02, periodic=(1, 1, 1), u_in=0.0, check_every=1, avg_start=None)
    f = g.populations()
    f[14, 1, 1, 5] += 0.35     # +x population
    f[12, 1, 1, 5] -= 0.35     # -x population: rho = 1, u = 0.7 > 1/sqrt(3)
    g.set_populations(f)
    g.step(1)
    torch.cuda.synchronize()
    with pytest.raises(HipError) as e:
        g.step(0)
    assert e.value.code == 4


def test_caller_workspace_is_bitwise_the_library_allocation():
    """lbm_create_in with a torch-allocated workspace of exactly
    lbm_workspace_size bytes runs the same computation bit for bit as the
    library's own allocation; with force_capacity = 8 the force series is
    a ring holding the last 8 samples of the full series, with their
    steps; a checkpoint of the ring resumes bitwise."""
    import torch
    P = _P()
    shape = (64, 16, 16)
    geo = sphere_channel(shape, center=(20.0, 7.5, 7.5), radius=3.0)
    u0 = perturbation(shape, 9, 5e-4, geo.solid)
    kw = dict(storage="f32", nu=0.005, obstacle_bc=1, avg_start=3, snap_every=7, snap_count=2)
    ref = P.Lbm(shape, solid=geo.solid, links=geo.links, u0=u0, **kw).step(29)
    nbytes = P.Lbm.workspace_size(shape, solid=geo.solid, force_capacity=8, **kw)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    g = P.Lbm(shape, solid=geo.solid, links=geo.links, u0=u0, force_capacity=8, workspace=ws, **kw).step(29)
    assert np.array_equal(g.populations(), ref.populations())
    assert np.array_equal(g.mean_fields()[0], ref.mean_fields()[0])
    assert np.array_equal(g.snapshots()[0], ref.snapshots()[0])
    fr, sr = ref.forces()
    fg, sg = g.forces()
    assert len(fg) == 8 and np.array_equal(sg, sr[-8:]) and np.array_equal(fg, fr[-8:])
    blob = g.export_state()
    g.step(11)
    ref.step(11)
    h = P.Lbm(shape, solid=geo.solid, links=geo.links, u0=u0, force_capacity=8, **kw)
    h.import_state(blob)
    h.step(11)
    assert np.array_equal(h.populations(), g.populations())
    fh, sh = h.forces()
    fr, sr = ref.forces()
    assert np.array_equal(sh, sr[-8:]) and np.array_equal(fh, fr[-8:])


def test_caller_workspace_checks():
    """A workspace smaller than lbm_workspace_size, or forces on with a
    growing series, is rejected before any device work."""
    import torch
    P = _P()
    from paper_2606_16765_amd._lib import HipError
    shape = (64, 8, 8)
    geo = sphere_channel(shape, center=(20.0, 3.5, 3.5), radius=2.0)
    n = P.Lbm.workspace_size(shape, solid=geo.solid, nu=0.02, force_capacity=4)
    ws = torch.empty(n - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(HipError, match="smaller than lbm_workspace_size"):
        P.Lbm(shape, nu=0.02, solid=geo.solid, force_capacity=4, workspace=ws)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(HipError, match="force_capacity"):
        P.Lbm(shape, nu=0.02, solid=geo.solid, workspace=ws)


def test_reynolds_number_sets_the_viscosity():
    """re and l_ref give omega1 = 1/(3 u_in l_ref / re + 1/2) and the
    automatic mode switch at Re_c = u_in ny / nu = 3000."""
    P = _P()
    shape = (64, 32, 8)
    for re, l_ref, mode in ((1000.0, None, 0), (3000.0, 32.0, 1), (900.0, 8.0, 1)):
        g = P.Lbm(shape, storage="f32", u_in=0.05, re=re, l_ref=l_ref, avg_start=None)
        nu = 0.05 * (l_ref or 32.0) / re
        info = g.info()
        assert abs(info["omega1"] - 1.0 / (3.0 * nu + 0.5)) < 1e-15
        assert info["mode"] == mode, (re, l_ref)
        g.close()
