"""GPU lattice Boltzmann path (HIP library through the C ABI) against the
FP64 CPU oracle, element by element on the same seeded inputs.

Tolerances: FP64 storage and arithmetic 1e-11 relative (only the summation
order differs between the two sides); FP32 1e-5 relative L2 on the mean
fields (the target of the FP32 path); FP16/BF16 shifted storage against the
storage-emulating oracle with the bounds stated in each test.
"""
import numpy as np
import pytest

from inputs import perturbation, sphere_channel
from oracle import lbm as olbm

pytestmark = pytest.mark.gpu


def _gpu():
    import paper_2606_16765_amd as P
    return P


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def f64_err(a, b):
    """Populations: max |a - b| against 1e-11 max|b| + 1e-14.  The absolute
    floor is the oracle's own rounding: it works on unshifted f (up to 8/27),
    so a few hundred operations leave ~1e-14 absolute noise even where the
    shifted populations are tiny."""
    return float(np.abs(a - b).max() / (1e-11 * np.abs(b).max() + 1e-14)) * 1e-11


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def pair(shape, steps, storage="f64", solid=None, links=None, u0=None, periodic=(0, 0, 0), nu=0.02, u_in=0.05,
         mode="plain", obstacle_bc=0, body_force=(0, 0, 0), avg_start=0, snap_every=0, snap_count=20, emulate=None,
         xcd_remap=1, force_every=1):
    P = _gpu()
    g = P.Lbm(shape, storage=storage, periodic=periodic, u_in=u_in, nu=nu, mode=mode, obstacle_bc=obstacle_bc,
              body_force=body_force, avg_start=avg_start, snap_every=snap_every, snap_count=snap_count,
              solid=solid, links=links, u0=u0, xcd_remap=xcd_remap, force_every=force_every)
    g.step(steps)
    p = olbm.make_params(shape, periodic=periodic, nu=nu, u_in=u_in, mode={"plain": 0, "k17": 1}[mode],
                         obstacle_bc=obstacle_bc, force=body_force, avg_start=avg_start, snap_every=snap_every,
                         emulate=emulate)
    o = olbm.Run(p, solid=solid, links=links, u0=u0)
    o.step(steps, snap_cap=(steps // snap_every + 1) if snap_every else 0)
    return g, o


# ------------------------------------------------------------------ small
@pytest.mark.parametrize("steps", [20, 21])
def test_periodic_box_f64_populations(steps):
    shape = (64, 8, 4)
    u0 = perturbation(shape, 11, 0.02)
    g, o = pair(shape, steps, periodic=(1, 1, 1), nu=0.05, u0=u0, u_in=0.0)
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err


@pytest.mark.parametrize("steps", [30, 31])
def test_walled_channel_f64_populations(steps):
    shape = (64, 8, 8)
    u0 = perturbation(shape, 3, 5e-4)
    g, o = pair(shape, steps, u0=u0)
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err
    m, n = g.mean_fields()
    assert n == steps
    assert rel_max(m, o.mean_fields()) < 1e-11


@pytest.mark.parametrize("mode", ["plain", "k17"])
def test_periodic_sides_obstacle_channel_f64(mode):
    """Inlet and outlet in x with periodic y and z, the lateral setting of
    the sphere-drag validation runs, with interpolated bounce-back."""
    shape = (64, 16, 16)
    geo = sphere_channel(shape, center=(20.3, 7.6, 7.4), radius=3.3)
    u0 = perturbation(shape, 6, 5e-4, geo.solid)
    nu = 0.05 * 16 / 5000 if mode == "k17" else 0.01
    g, o = pair(shape, 33, solid=geo.solid, links=geo.links, u0=u0, nu=nu, mode=mode, obstacle_bc=1,
                periodic=(0, 1, 1))
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err
    fg, _ = g.forces()
    fo = np.array(o.forces)
    assert np.abs(fg - fo).max() < 1e-11 * np.abs(fo).max()


def test_periodic_z_wrap_beyond_int32_elements():
    """Periodic z on a grid whose wrap offset, nz - 1 padded planes, exceeds
    2^31 elements (64 x 4 x 103584, FP64 storage, inlet and outlet in x,
    periodic y and z).  The initial velocity repeats every 16 planes, so the
    state stays 16-periodic in z and every 16-plane box must equal the
    oracle on a 16-plane periodic domain, the boxes at both periodic faces
    included; their cells pull across the wrap on odd steps."""
    P = _gpu()
    nx, ny, per = 64, 4, 16
    plane = 27 * (nx + 64) * (ny + 2)
    nz = per * ((1 << 31) // (plane * per) + 2)
    assert (nz - 1) * plane >= (1 << 31)
    small = (nx, ny, per)
    u0s = perturbation(small, 21, 5e-3)
    nu, steps = 0.01, 11
    g = P.Lbm((nx, ny, nz), storage="f64", periodic=(0, 1, 1), u_in=0.05, nu=nu, mode="k17",
              u0=np.tile(u0s, (1, nz // per, 1, 1)))
    g.step(steps)
    p = olbm.make_params(small, periodic=(0, 1, 1), nu=nu, u_in=0.05, mode=1)
    o = olbm.Run(p, u0=u0s)
    o.step(steps)
    for z0 in (0, (nz // 2 // per) * per, nz - per):
        err = f64_err(g.populations_box((0, 0, z0), small), o.fbar)
        print("z0", z0, "err", err)
        assert err < 1e-11, (z0, err)
    g.close()


@pytest.mark.parametrize("mode", ["plain", "k17"])
@pytest.mark.parametrize("obstacle_bc", [0, 1])
def test_obstacle_channel_f64(mode, obstacle_bc):
    shape = (64, 16, 16)
    geo = sphere_channel(shape, center=(20.3, 7.6, 7.4), radius=3.3)
    u0 = perturbation(shape, 5, 5e-4, geo.solid)
    nu = 0.05 * 16 / 5000 if mode == "k17" else 0.01
    g, o = pair(shape, 41, solid=geo.solid, links=geo.links, u0=u0, nu=nu, mode=mode, obstacle_bc=obstacle_bc)
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err
    fg, steps = g.forces()
    fo = np.array(o.forces)
    assert np.array_equal(steps, np.arange(41))
    assert np.abs(fg - fo).max() < 1e-11 * np.abs(fo).max()


def test_precision_study_reference_f64_at_128x64x64():
    """The FP64 storage path that serves as the reference of the FP32/FP16/
    BF16 error study agrees with the oracle at the study's size: the seeded
    random obstacle at 128x64x64, interpolated bounce-back, K17 (Re 10000 on
    the channel height), 60 steps."""
    from inputs import random_obstacle
    shape = (128, 64, 64)
    geo = random_obstacle(shape, 0)
    u0 = perturbation(shape, 0, 5e-4, geo.solid)
    nu = 0.05 * 64 / 10000.0
    g, o = pair(shape, 60, solid=geo.solid, links=geo.links, u0=u0, nu=nu, mode="k17", obstacle_bc=1)
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err
    m, n = g.mean_fields()
    assert rel_max(m, o.mean_fields()) < 1e-11


def test_bandwidth_probe_leaves_state_unchanged():
    """The probe swaps every cell's opposite slots; an even number of passes
    must restore the populations bitwise, at any AA parity."""
    shape = (64, 8, 8)
    geo = sphere_channel(shape, center=(20.3, 3.6, 3.4), radius=2.3)
    P = _gpu()
    g = P.Lbm(shape, storage="f32", nu=0.02, solid=geo.solid, perturb=(4, 5e-4))
    for steps in (3, 4):
        g.step(steps)
        before = g.populations()
        ms = g.bandwidth_probe(4)
        assert ms > 0
        assert np.array_equal(g.populations(), before)
    with pytest.raises(Exception):
        g.bandwidth_probe(3)
    g.close()


def test_poiseuille_body_force_f64():
    shape = (64, 16, 1)
    g, o = pair(shape, 300, periodic=(1, 0, 1), nu=0.1, u_in=0.0, body_force=(1e-6, 0, 0))
    err = f64_err(g.populations(), o.fbar)
    assert err < 1e-11, err


def test_snapshots_match_oracle():
    shape = (64, 8, 8)
    u0 = perturbation(shape, 9, 5e-4)
    g, o = pair(shape, 60, storage="f64", u0=u0, snap_every=25, snap_count=2)
    snaps, steps = g.snapshots()
    assert list(steps) == [25, 50]
    so = np.array(o.snaps).reshape((-1, 4) + shape[::-1])
    # oracle keeps every snapshot (0, 25, 50); the ring keeps the last two
    assert rel_max(snaps.astype(np.float64), so[1:3]) < 1e-6


# ------------------------------------------------------------------ C0
C0 = dict(shape=(64, 32, 32), steps=500, nu=0.05 * 8 / 1000, u_in=0.05)


@pytest.fixture(scope="module")
def c0_oracle():
    geo = sphere_channel()
    u0 = perturbation(geo.shape, 0, 0.01 * C0["u_in"], geo.solid)
    p = olbm.make_params(geo.shape, nu=C0["nu"], u_in=C0["u_in"], mode=0, avg_start=0)
    o = olbm.Run(p, solid=geo.solid, u0=u0)
    o.step(C0["steps"])
    return geo, u0, o


def _c0_gpu(geo, u0, storage, xcd_remap=1):
    P = _gpu()
    g = P.Lbm(geo.shape, storage=storage, u_in=C0["u_in"], nu=C0["nu"], mode="plain", solid=geo.solid, u0=u0,
              avg_start=0, xcd_remap=xcd_remap)
    g.step(C0["steps"])
    return g


def test_c0_f64_mean_fields_and_drag(c0_oracle):
    geo, u0, o = c0_oracle
    g = _c0_gpu(geo, u0, "f64")
    m, n = g.mean_fields()
    assert n == C0["steps"]
    mo = o.mean_fields()
    assert rel_max(m, mo) < 1e-11
    fg, _ = g.forces()
    fo = np.array(o.forces)
    assert np.abs(fg - fo).max() < 1e-11 * np.abs(fo).max()


def test_c0_f32_mean_fields_within_1e5(c0_oracle):
    geo, u0, o = c0_oracle
    g = _c0_gpu(geo, u0, "f32")
    m, _ = g.mean_fields()
    mo = o.mean_fields()
    vel = rel_l2(m[:3], mo[:3])
    per = [rel_l2(m[k], mo[k]) for k in range(4)]
    print("C0 FP32 mean fields: e_vel", vel, "u v w p", per, flush=True)
    assert vel < 1e-5, vel
    for k in range(4):
        assert per[k] < 1e-5, (k, per[k])
    fg, _ = g.forces()
    fo = np.array(o.forces)
    assert rel_l2(fg[:, 0], fo[:, 0]) < 1e-5


def test_c0_f32_xcd_remap_is_bitwise_neutral(c0_oracle):
    """Different workgroup-to-tile orders give bitwise identical results: the
    in-place AA update has no cross-cell read-after-write hazard."""
    geo, u0, _ = c0_oracle
    a = _c0_gpu(geo, u0, "f32", xcd_remap=1)
    b = _c0_gpu(geo, u0, "f32", xcd_remap=0)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.mean_fields()[0], b.mean_fields()[0])


# ------------------------------------------------------------------ precision
@pytest.mark.parametrize("storage,bound", [("f16", 3e-3), ("bf16", 3e-2)])
def test_shifted_low_precision_storage(storage, bound):
    """FP16/BF16 storage of f - w_i with FP32 arithmetic against the oracle
    that rounds the stored populations the same way (and against the plain
    FP64 oracle): the relative L2 error of the mean velocity after 200
    steps stays below a bound set by the storage precision."""
    shape = (64, 16, 16)
    geo = sphere_channel(shape, center=(20.0, 7.5, 7.5), radius=3.0)
    u0 = perturbation(shape, 2, 5e-4, geo.solid)
    g, o = pair(shape, 200, storage=storage, solid=geo.solid, u0=u0, nu=0.005, emulate=storage)
    m, _ = g.mean_fields()
    e_emul = rel_l2(m[:3], o.mean_fields()[:3])
    p = olbm.make_params(shape, nu=0.005, u_in=0.05, mode=0)
    o64 = olbm.Run(p, solid=geo.solid, u0=u0).step(200, forces=False)
    e64 = rel_l2(m[:3], o64.mean_fields()[:3])
    assert e_emul < bound and e64 < bound, (e_emul, e64)


def test_f32_mass_conserved_periodic():
    P = _gpu()
    shape = (64, 16, 8)
    u0 = perturbation(shape, 4, 0.02)
    g = P.Lbm(shape, storage="f32", periodic=(1, 1, 1), nu=0.01, u_in=0.0, u0=u0, avg_start=None)
    m0 = g.mass()
    g.step(100)
    m1 = g.mass()
    assert abs(m1 - m0) < 1e-4 * 0.02 * shape[0] * shape[1] * shape[2] * 1e-2


def test_checkpoint_resume_bitwise():
    P = _gpu()
    shape = (64, 16, 16)
    geo = sphere_channel(shape, center=(20.0, 7.5, 7.5), radius=3.0)
    u0 = perturbation(shape, 8, 5e-4, geo.solid)
    kw = dict(storage="f32", nu=0.005, solid=geo.solid, u0=u0, snap_every=10, snap_count=3)
    a = P.Lbm(shape, **kw).step(37)
    blob = a.export_state()
    a.step(40)
    b = P.Lbm(shape, **kw)
    b.import_state(blob)
    b.step(40)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.mean_fields()[0], b.mean_fields()[0])
    assert np.array_equal(a.forces()[0], b.forces()[0])
    assert np.array_equal(a.snapshots()[0], b.snapshots()[0])


def test_set_populations_round_trip():
    P = _gpu()
    shape = (64, 8, 8)
    g = P.Lbm(shape, storage="f64", nu=0.02, u0=perturbation(shape, 1, 5e-4))
    g.step(7)
    f = g.populations()
    g.set_populations(f)
    assert np.array_equal(g.populations(), f)


def test_moments_match_populations():
    P = _gpu()
    shape = (64, 8, 8)
    g = P.Lbm(shape, storage="f64", nu=0.02, u0=perturbation(shape, 1, 5e-4)).step(9)
    f = g.populations().reshape(27, -1)
    c, _ = olbm.lattice()
    d = f.sum(0)
    u = (c.T.astype(float) @ f) / (1 + d)
    m = g.moments().reshape(4, -1)
    assert np.abs(m[:3] - u).max() < 1e-7
    assert np.abs(m[3] - d / 3).max() < 1e-7


def test_device_perturbation_matches_host_generator():
    """The library's on-device SplitMix64 perturbation equals the host
    input generator's, so both initial states are identical."""
    P = _gpu()
    shape = (64, 8, 8)
    geo = sphere_channel(shape, center=(20.0, 3.5, 3.5), radius=2.0)
    u0 = perturbation(shape, 77, 5e-4, geo.solid)
    a = P.Lbm(shape, storage="f64", nu=0.02, solid=geo.solid, u0=u0)
    b = P.Lbm(shape, storage="f64", nu=0.02, solid=geo.solid, perturb=(77, 5e-4))
    assert np.array_equal(a.populations(), b.populations())


# ------------------------------------------------------ full size (boxes)
def _box_links(geo, shape, o, s):
    cell, d, q = geo.links
    nx, ny, _ = shape
    lx, ly, lz = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    (x0, y0, z0), (bx, by, bz) = o, s
    inb = (lx >= x0) & (lx < x0 + bx) & (ly >= y0) & (ly < y0 + by) & (lz >= z0) & (lz < z0 + bz)
    lc = ((lz[inb] - z0) * by + (ly[inb] - y0)) * bx + (lx[inb] - x0)
    return (lc, d[inb], q[inb])


def _valid(shape, o, s):
    """Cells of the box whose whole neighbourhood is in the box or beyond a
    real domain boundary, as slices (z, y, x)."""
    sl = []
    for org, size, n in zip(o[::-1], s[::-1], shape[::-1]):
        sl.append(slice(0 if org == 0 else 1, size if org + size == n else size - 1))
    return tuple(sl)


def _check_boxes(sim, geo, shape, boxes, params, bound, first_step):
    """Step the GPU twice; after each step compare every box with one FP64
    oracle step of the box's previous state.  Returns the worst error."""
    worst = 0.0
    for k in range(2):
        pres = [sim.populations_box(o, s) for o, s in boxes]
        sim.step(1)
        for (o, s), pre in zip(boxes, pres):
            post = sim.populations_box(o, s)
            (x0, y0, z0), (bx, by, bz) = o, s
            solid = np.ascontiguousarray(geo.solid[z0:z0 + bz, y0:y0 + by, x0:x0 + bx])
            links = _box_links(geo, shape, o, s)
            run = olbm.Run(params(s), solid=solid, links=links, fbar=pre)
            run.step(1, forces=False)
            ref = run.fbar.reshape(27, bz, by, bx)
            v = (slice(None),) + _valid(shape, o, s)
            err = float(np.abs(post[v] - ref[v]).max() / np.abs(ref[v]).max())
            print(f"step {first_step + k} box {o} {s}: {len(links[0])} links, max rel err {err:.2e}")
            assert np.abs(ref[v]).max() > 0
            assert err < bound, (o, s, k, err)
            worst = max(worst, err)
    return worst


def test_full_size_c2_step_on_sampled_boxes():
    """The benchmark configuration itself: 1024 x 512 x 512, FP32 storage,
    spanwise cylinder D = 64 at (307.2, 255.5), Re_D 3900 (K17), interpolated
    bounce-back, forces every step.  After 40 steps, boxes of cells are cut
    out of the GPU state (natural layout) and stepped once by the FP64 oracle
    as stand-alone domains; the GPU's next step must agree on every cell
    whose neighbourhood lies in the box or beyond a real domain boundary.
    Two consecutive steps cover both AA parities.  The boxes hold the
    cylinder surface (interpolated links, general path), open interior
    (flag-free tiles), the inlet with two walls and the outlet with the two
    other walls.  Bound: 1e-5 of the largest |fbar| in the box (FP32 storage
    and arithmetic against FP64 from the same FP32 inputs)."""
    P = _gpu()
    from inputs import spanwise_cylinder
    shape = (1024, 512, 512)
    geo = spanwise_cylinder(shape, center=(307.2, 255.5), diameter=64.0)
    nu = P.nu_from_re(0.05, 64.0, 3900.0)
    sim = P.Lbm(shape, storage="f32", u_in=0.05, nu=nu, mode="auto", solid=geo.solid, links=geo.links,
                obstacle_bc=1, perturb=(0, 0.01 * 0.05), avg_start=None, force_every=1)
    assert sim.info()["mode"] == 1
    sim.step(40)
    boxes = [((260, 236, 100), (96, 40, 12)),   # cylinder front and flank
             ((600, 300, 200), (64, 16, 16)),   # open interior
             ((0, 0, 0), (32, 16, 16)),          # inlet corner with walls y = 0, z = 0
             ((992, 496, 496), (32, 16, 16))]    # outlet corner with walls y = ny - 1, z = nz - 1
    worst = _check_boxes(sim, geo, shape, boxes,
                         lambda s: olbm.make_params(s, nu=nu, u_in=0.05, mode=1, obstacle_bc=1), 1e-5, 41)
    print("worst", worst)
    sim.close()


@pytest.mark.parametrize("storage,bound", [("f16", 2.0 ** -10), ("bf16", 2.0 ** -7)])
def test_full_size_c3_low_precision_step_on_sampled_boxes(storage, bound):
    """The storage study's throughput configuration at full size: 512 x 256 x
    256, seeded random obstacle (seed 0), Re_c 5500 (K17), shifted FP16 or
    BF16 storage.  Sampled boxes are stepped by the oracle in its storage
    emulation mode (FP64 arithmetic, the result rounded to the storage type
    with RNE).  The GPU rounds an FP32 result, so a value can land one
    storage ulp away where the two straddle a rounding boundary: bound one
    ulp at the top of the range, 2^-10 (FP16) and 2^-7 (BF16) of max |fbar|."""
    P = _gpu()
    from inputs import random_obstacle
    shape = (512, 256, 256)
    geo = random_obstacle(shape, 0)
    nu = P.nu_from_re(0.05, shape[1], 5500.0)
    sim = P.Lbm(shape, storage=storage, u_in=0.05, nu=nu, mode="auto", solid=geo.solid, links=geo.links,
                obstacle_bc=1, perturb=(0, 0.0005), avg_start=None, force_every=1)
    assert sim.info()["mode"] == 1
    sim.step(30)
    zi, yi, xi = np.nonzero(geo.solid)
    yc, zc = (int(yi.min()) + int(yi.max())) // 2, (int(zi.min()) + int(zi.max())) // 2
    boxes = [((int(xi.min()) - 4, yc - 16, zc - 8), (40, 32, 16)),   # obstacle front
             ((400, 40, 200), (32, 16, 16)),                          # interior
             ((0, 240, 0), (16, 16, 16))]                             # inlet corner
    worst = _check_boxes(sim, geo, shape, boxes,
                         lambda s: olbm.make_params(s, nu=nu, u_in=0.05, mode=1, obstacle_bc=1, emulate=storage),
                         bound, 31)
    print(storage, "worst", worst)
    sim.close()


def test_full_size_c1_running_mean_on_a_sampled_box():
    """The dataset configuration at full size (256 x 128 x 128, FP32, seeded
    obstacle, Re_c 5500, running mean from step 0, snapshots every 25 steps):
    the FP64 means on a box around the obstacle equal the mean over the
    steps of the oracle's moments of the exported pre-collision states (the
    sample of step n is the state that step reads)."""
    P = _gpu()
    from inputs import random_obstacle
    shape = (256, 128, 128)
    geo = random_obstacle(shape, 0)
    nu = P.nu_from_re(0.05, shape[1], 5500.0)
    sim = P.Lbm(shape, storage="f32", u_in=0.05, nu=nu, mode="auto", solid=geo.solid, links=geo.links,
                obstacle_bc=1, perturb=(0, 0.0005), avg_start=0, snap_every=25, snap_count=20, force_every=1)
    zi, yi, xi = np.nonzero(geo.solid)
    o = (int(xi.min()) - 4, (int(yi.min()) + int(yi.max())) // 2 - 16, (int(zi.min()) + int(zi.max())) // 2 - 8)
    s = (40, 32, 16)
    p = olbm.make_params(s, nu=nu, u_in=0.05, mode=1, obstacle_bc=1)
    K = 30
    acc = np.zeros((4, s[2], s[1], s[0]))
    for _ in range(K):
        rho, u = olbm.Run(p, fbar=sim.populations_box(o, s)).macroscopic()
        acc[:3] += u
        acc[3] += (rho - 1.0) / 3.0
        sim.step(1)
    means, n = sim.mean_fields()
    assert n == K
    (x0, y0, z0) = o
    got = means[:, z0:z0 + s[2], y0:y0 + s[1], x0:x0 + s[0]]
    fluid = geo.solid[z0:z0 + s[2], y0:y0 + s[1], x0:x0 + s[0]] == 0
    ref = acc / K
    err = float(np.abs(got[:, fluid] - ref[:, fluid]).max() / np.abs(ref[:, fluid]).max())
    print("running mean max rel err", err, "solid cells in the box", int((~fluid).sum()))
    assert (~fluid).sum() > 0
    assert np.all(got[:, ~fluid] == 0.0)
    assert err < 1e-5
    sim.close()


def test_populations_box_matches_full_export():
    """The box export returns the full export's values for its cells, at
    both AA parities, and rejects boxes that leave the grid."""
    P = _gpu()
    shape = (64, 32, 32)
    geo = sphere_channel(shape, (20.0, 15.5, 15.5), 5.0)
    g = P.Lbm(shape, storage="f32", nu=0.01, u_in=0.05, mode="k17", solid=geo.solid, links=geo.links,
              obstacle_bc=1, perturb=(3, 5e-4))
    for n in (7, 1):
        g.step(n)
        full = g.populations()
        b = g.populations_box((5, 9, 2), (40, 13, 21))
        assert np.array_equal(b, full[:, 2:23, 9:22, 5:45])
    from paper_2606_16765_amd._lib import HipError
    with pytest.raises(HipError, match="box outside"):
        g.populations_box((30, 0, 0), (40, 8, 8))
    g.close()
