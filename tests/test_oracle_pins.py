"""Pins of the FP64 lattice Boltzmann oracle against what the mathematics and
the physics fix, independent of the oracle's own formulas.

Each test names what it pins; together they are chosen so that a dropped
term, a wrong sign or index, or a transposed operand anywhere in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import brute, lbm

RNG = np.random.default_rng(1234)


# ------------------------------------------------------------------ lattice
def test_lattice_isotropy_closed_forms():
    """D3Q27 weights: sum w = 1, sum w c = 0, sum w c_a c_b = delta_ab/3,
    sum w c_a^2 c_b^2 = 1/9 (a != b), sum w cx^2 cy^2 cz^2 = 1/27; opposite
    of direction i is 26 - i."""
    c, w = lbm.lattice()
    c = c.astype(np.float64)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-16)
    assert abs((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum() - 1 / 9) < 1e-16
    assert abs((w * c[:, 0] ** 4).sum() - 1 / 3) < 1e-16
    assert abs((w * c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2).sum() - 1 / 27) < 1e-16
    for i in range(27):
        assert np.array_equal(c[26 - i], -c[i])
    assert sorted(np.round(w * 216).astype(int).tolist()) == sorted([64] + [16] * 6 + [4] * 12 + [1] * 8)


# ------------------------------------------------------------ equilibrium
@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.07, (0.05, -0.03, 0.02)), (0.93, (-0.1, 0.08, 0.12))])
def test_equilibrium_central_moments(rho, u):
    """Central moments of the discrete equilibrium are the Gaussian ones:
    K000 = rho, K200 = rho/3, K220 = rho/9, K222 = rho/27, all others 0."""
    _, w = lbm.lattice()
    f = lbm.equilibrium(rho, np.array(u)) + w
    K = lbm.central_moments(f, np.array(u))
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                m = 9 * a + 3 * b + cc
                if a % 2 or b % 2 or cc % 2:
                    expect = 0.0
                else:
                    expect = rho * (1 / 3) ** ((a + b + cc) // 2)
                assert abs(K[m] - expect) < 1e-15, (a, b, cc, K[m], expect)


def test_equilibrium_matches_gaussian_moment_solve():
    """Product-form equilibrium equals the one solved from its central
    moments through the 27x27 raw-moment system (brute variant)."""
    for _ in range(5):
        rho = 1 + 0.1 * RNG.standard_normal()
        u = 0.1 * RNG.standard_normal(3)
        a = lbm.equilibrium(rho, u)
        b = brute.equilibrium(rho, u)[:, 0]
        assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("galilean", [0, 1])
@pytest.mark.parametrize("omega1", [0.7, 1.3, 1.85, 1.99])
def test_equilibrium_is_fixed_point(mode, galilean, omega1):
    """The collision leaves any equilibrium unchanged (to rounding)."""
    for omega2 in (1.0, 1.4):
        p = lbm.make_params((1, 1, 1), omega1=omega1, omega2=omega2, mode=mode, galilean=galilean)
        for _ in range(3):
            rho = 1 + 0.05 * RNG.standard_normal()
            u = 0.08 * RNG.standard_normal(3)
            fe = lbm.equilibrium(rho, u)
            assert np.abs(lbm.collide(p, fe) - fe).max() < 1e-13


# ------------------------------------------------------------ conservation
@pytest.mark.parametrize("mode", [0, 1])
def test_collision_conserves_mass_and_momentum(mode):
    """sum f and sum f c are invariant under the collision; with a body force
    the momentum changes by exactly F."""
    c, w = lbm.lattice()
    for force in ((0.0, 0.0, 0.0), (1e-4, -2e-4, 3e-5)):
        p = lbm.make_params((1, 1, 1), omega1=1.93, mode=mode, force=force)
        for _ in range(5):
            f = lbm.equilibrium(1.0, 0.05 * RNG.standard_normal(3)) + 1e-3 * RNG.standard_normal(27)
            g = lbm.collide(p, f)
            assert abs(g.sum() - f.sum()) < 1e-16 * 30
            dj = c.T.astype(float) @ (g - f)
            assert np.abs(dj - np.array(force)).max() < 1e-16 * 30


def test_force_free_collision_without_relaxation_is_identity():
    """omega1 = omega2 = 0 (no relaxation) with orders >= 3 kept would be the
    identity; in plain mode orders >= 3 are dropped, so only states whose
    higher cumulants vanish (equilibria with non-equilibrium second order)
    are preserved."""
    p = lbm.make_params((1, 1, 1), omega1=1e-12, omega2=1e-12, galilean=0)
    # build a state with arbitrary second-order cumulants and zero higher ones
    u = np.array([0.03, -0.01, 0.02])
    C = np.zeros(27)
    C[0] = 1.0
    C[18], C[6], C[2] = 0.34, 0.32, 0.335
    C[12], C[10], C[4] = 0.004, -0.002, 0.001
    k = lbm.moments_from_cumulants(C)
    K = 1.02 * k
    K[0] = 1.02
    f = lbm.populations_from_central(K, u)
    _, w = lbm.lattice()
    fb = f - w
    assert np.abs(lbm.collide(p, fb) - fb).max() < 1e-14


# ------------------------------------------------------------ transforms
def test_central_moments_match_binomial_shift_of_raw_moments():
    for _ in range(5):
        f = 1 / 27 + 0.01 * RNG.standard_normal(27)
        u = 0.1 * RNG.standard_normal(3)
        K = lbm.central_moments(f, u)
        raw = brute.RAW @ f
        Kb = brute._shift(raw[:, None], [np.array([u[0]]), np.array([u[1]]), np.array([u[2]])], -1.0)[:, 0]
        assert np.abs(K - Kb).max() < 1e-15


def test_central_moment_map_round_trip():
    for _ in range(5):
        f = 1 / 27 + 0.01 * RNG.standard_normal(27)
        u = 0.1 * RNG.standard_normal(3)
        g = lbm.populations_from_central(lbm.central_moments(f, u), u)
        assert np.abs(g - f).max() < 1e-15
        # and the other way round, from arbitrary moments
        K = RNG.standard_normal(27)
        K2 = lbm.central_moments(lbm.populations_from_central(K, u), u)
        assert np.abs(K2 - K).max() < 1e-13


def test_cumulant_closed_forms_match_set_partition_sums():
    """Orders 4-6 written out equal the generic partition formula, both
    directions, on random moments (first order zero)."""
    for _ in range(6):
        k = RNG.standard_normal(27) * 0.3
        k[9] = k[3] = k[1] = 0.0
        Cc = lbm.cumulants(k)
        Cg = brute.cumulants_generic(k[:, None])[:, 0]
        assert np.abs(Cc - Cg).max() < 1e-14
        kk = lbm.moments_from_cumulants(Cc)
        kg = brute.moments_generic(Cc[:, None])[:, 0]
        assert np.abs(kk - kg).max() < 1e-14
        assert np.abs(kk - k).max() < 1e-14


def test_cumulants_of_product_distribution_factorise():
    """For a distribution that is a product of independent 1D
    distributions, every mixed cumulant vanishes (independence), whatever
    the marginals."""
    _, w = lbm.lattice()
    px = np.array([0.2, 0.5, 0.3])
    py = np.array([0.25, 0.45, 0.3])
    pz = np.array([0.1, 0.7, 0.2])
    f = np.zeros(27)
    for i in range(27):
        f[i] = px[i % 3] * py[(i // 3) % 3] * pz[i // 9]
    c, _ = lbm.lattice()
    u = c.T.astype(float) @ f
    K = lbm.central_moments(f, u)
    Cm = lbm.cumulants(K)
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                if sum(x > 0 for x in (a, b, cc)) >= 2 and a + b + cc >= 2:
                    assert abs(Cm[9 * a + 3 * b + cc]) < 1e-15, (a, b, cc)


# ------------------------------------------------------------ operator
@pytest.mark.parametrize("mode", [0, 1])
def test_collide_matches_brute_variant(mode):
    for _ in range(4):
        u = 0.06 * RNG.standard_normal(3)
        f = lbm.equilibrium(1 + 0.02 * RNG.standard_normal(), u) + 2e-3 * RNG.standard_normal(27)
        for G in (0, 1):
            p = lbm.make_params((1, 1, 1), omega1=1.95, mode=mode, galilean=G, lam=0.01)
            a = lbm.collide(p, f)
            b = brute.collide(f[:, None], 1.95, mode=mode, galilean=G, lam=0.01)[:, 0]
            assert np.abs(a - b).max() < 1e-15


def test_k17_with_neutral_coefficients_is_plain():
    """w3 = w4 = w5 = 1 and A = B = 0 make the parametrised operator the plain
    one (third order relaxed fully, fourth order zero)."""
    f = lbm.equilibrium(1.01, np.array([0.04, 0.01, -0.02])) + 2e-3 * RNG.standard_normal(27)
    p0 = lbm.make_params((1, 1, 1), omega1=1.97, mode=0)
    p1 = lbm.make_params((1, 1, 1), omega1=1.97, mode=1, k17=(1, 1, 1, 0, 0))
    assert np.abs(lbm.collide(p0, f) - lbm.collide(p1, f)).max() < 1e-17


def test_k17_rates_limits():
    """Rates vanish as omega1 -> 2 (the factor omega1 - 2) and are small
    positive relaxation rates at omega1 = 1.99; the closed forms agree with
    the brute variant's transcription.  (The limiter is pinned by
    test_limiter_effective_rate_closed_form.)"""
    co = lbm.k17_coefficients(2.0 - 1e-9)
    assert np.abs(co[:3]).max() < 1e-7
    co99 = lbm.k17_coefficients(1.99)
    assert 0 < co99[0] < 0.1 and 0 < co99[1] < 0.1 and 0 < co99[2] < 0.1
    assert np.allclose(lbm.k17_coefficients(1.9), brute.k17_coefficients(1.9), rtol=1e-14)


def _state_from_cumulants(C, rho=1.0, u=(0.0, 0.0, 0.0)):
    """Shifted populations whose normalised cumulants are C (index 9a+3b+c)
    at density rho and velocity u."""
    u = np.asarray(u, float)
    k = lbm.moments_from_cumulants(C)
    K = rho * k
    K[0] = rho
    K[9] = K[3] = K[1] = 0.0
    _, w = lbm.lattice()
    return lbm.populations_from_central(K, u) - w


def _post_cumulants(p, fbar, u=(0.0, 0.0, 0.0)):
    _, w = lbm.lattice()
    g = lbm.collide(p, fbar) + w
    rho = g.sum()
    return lbm.cumulants(lbm.central_moments(g, np.asarray(u, float)) / rho)


@pytest.mark.parametrize("which", ["sum", "diff", "c111"])
def test_limiter_effective_rate_closed_form(which):
    """Third-order limiter of the fourth-order mode (Sec. 3.2, limiter of
    the parametrised operator; reading R4).  At rest with second-order
    cumulants at equilibrium, one third-order combination c is relaxed to
    (1 - w_eff) c and nothing else changes.  The limiter's defining
    properties fix w_eff without the formula: w_eff -> w (the unlimited
    rate) for |c| << lambda, w_eff -> 1 (full relaxation) for |c| >> lambda,
    w_eff = (w + 1)/2 at |c| = lambda (lambda is the half-way scale), even
    in c and monotone in |c|.  Given rates w3 = 0.2 (pair sums),
    w4 = 0.5 (pair differences) and w5 = 0.8 (c111) are distinct, so a rate
    applied to the wrong combination fails too, and so does a limiter
    weighted by lambda/(lambda + |c|) or with (1 + w)."""
    lam = 1e-3
    rates = {"sum": 0.2, "diff": 0.5, "c111": 0.8}
    w = rates[which]
    p = lbm.make_params((1, 1, 1), omega1=1.9, mode=1, lam=lam, k17=(0.2, 0.5, 0.8, 0.0, 0.0))

    def w_eff(c):
        C = np.zeros(27)
        C[0] = 1.0
        C[18] = C[6] = C[2] = 1.0 / 3.0
        if which == "c111":
            C[13] = c
        else:
            # c120 = IX(1,2,0) = 15, c102 = IX(1,0,2) = 11
            C[15], C[11] = (c / 2, c / 2) if which == "sum" else (c / 2, -c / 2)
        Cs = _post_cumulants(p, _state_from_cumulants(C))
        if which == "c111":
            out = Cs[13]
            other = 0.0
            touched = [13]
        else:
            out = Cs[15] + Cs[11] if which == "sum" else Cs[15] - Cs[11]
            other = Cs[15] - Cs[11] if which == "sum" else Cs[15] + Cs[11]
            touched = [15, 11]
        # everything else keeps its equilibrium value (rest, second order 1/3)
        rest = np.zeros(27)
        rest[0] = 1.0
        rest[18] = rest[6] = rest[2] = 1.0 / 3.0
        mask = np.ones(27, bool)
        mask[touched] = False
        assert np.abs(Cs[mask] - rest[mask]).max() < 1e-13 and abs(other) < 1e-13 * max(abs(c), 1.0)
        return 1.0 - out / c

    small = w_eff(lam * 1e-6)
    assert abs(small - w) < 1e-5
    large = w_eff(lam * 1e6)
    assert abs(large - 1.0) < 1e-5
    assert abs(w_eff(lam) - 0.5 * (w + 1.0)) < 1e-9
    assert abs(w_eff(-lam) - w_eff(lam)) < 1e-12
    grid = [w_eff(lam * t) for t in (0.01, 0.1, 0.5, 1.0, 2.0, 10.0, 100.0)]
    assert all(b > a for a, b in zip(grid, grid[1:]))


def test_collision_relaxes_shear_at_omega1():
    """Off-diagonal second-order cumulants relax at omega1 (the rate that
    sets nu = (1/omega1 - 1/2)/3): at rest, c110* = (1 - omega1) c110, and
    a traceless diagonal deviation relaxes the same way."""
    for om in (0.8, 1.6, 1.99):
        p = lbm.make_params((1, 1, 1), omega1=om, mode=0)
        C = np.zeros(27)
        C[0] = 1.0
        C[18] = C[6] = C[2] = 1.0 / 3.0
        C[12] = 2e-3                               # c110
        C[18] += 1e-3
        C[6] -= 1e-3                               # c200 - c020 = 2e-3, trace unchanged
        Cs = _post_cumulants(p, _state_from_cumulants(C))
        assert abs(Cs[12] - (1 - om) * 2e-3) < 1e-15
        assert abs((Cs[18] - Cs[6]) - (1 - om) * 2e-3) < 1e-15
        assert abs(Cs[18] + Cs[6] + Cs[2] - 1.0) < 1e-15


def _tgv_error(N, omega, mode=0, U=(0.0, 0.0), G=1, U0=1e-3, frac=0.5):
    """Relative error of the Taylor-Green decay rate against 2 nu k^2, with
    nu = (1/omega1 - 1/2)/3; amplitude from the (+-1,+-1) Fourier modes."""
    p = lbm.make_params((N, N, 1), periodic=(1, 1, 1), omega1=omega, mode=mode, galilean=G, lam=1e10)
    k = 2 * np.pi / N
    x = np.arange(N)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((3, 1, N, N))
    u[0, 0] = U[0] + U0 * np.sin(k * X) * np.cos(k * Y)
    u[1, 0] = U[1] - U0 * np.cos(k * X) * np.sin(k * Y)
    nu = (1 / omega - 0.5) / 3
    T = max(int(frac / (2 * nu * k * k)), 4)
    r = lbm.Run(p, u0=u)

    def amp():
        _, uu = r.macroscopic()
        e = 0.0
        for d in range(2):
            F = np.fft.fft2(uu[d, 0] - U[d])
            e += sum(abs(F[i, j]) ** 2 for i in (1, -1) for j in (1, -1))
        return math.sqrt(e)

    r.step(T // 4, forces=False)
    a1 = amp()
    r.step(T, forces=False)
    a2 = amp()
    return math.log(a1 / a2) / T / (2 * nu * k * k) - 1


def test_taylor_green_decay_at_lattice_viscosity():
    """Plain operator: decay rate 2 nu k^2 within 1% and second-order
    convergence (error ratio ~4 per doubling)."""
    e16 = _tgv_error(16, 1.6)
    e32 = _tgv_error(32, 1.6)
    assert abs(e32) < 1e-2 and abs(e16) < 1e-2
    assert 3.0 < e16 / e32 < 6.0


def test_galilean_correction_removes_velocity_dependence():
    """Under a superposed uniform velocity the decay rate error is small with
    the correction, larger without it, larger still with its sign flipped."""
    e1 = abs(_tgv_error(32, 1.6, U=(0.1, 0.0), G=1, U0=0.01, frac=0.25))
    e0 = abs(_tgv_error(32, 1.6, U=(0.1, 0.0), G=0, U0=0.01, frac=0.25))
    em = abs(_tgv_error(32, 1.6, U=(0.1, 0.0), G=-1, U0=0.01, frac=0.25))
    assert e1 < 3e-3
    assert e0 > 5 * e1
    assert em > 1.5 * e0


def test_k17_diffusion_converges_faster_than_plain():
    """The parametrised operator's Taylor-Green decay error falls much faster
    than second order between N = 24 and 48 (plain: ~4x)."""
    om = 1.9
    p24, p48 = _tgv_error(24, om, 0), _tgv_error(48, om, 0)
    k24, k48 = _tgv_error(24, om, 1), _tgv_error(48, om, 1)
    assert 3.5 < p24 / p48 < 4.8
    assert abs(k24 / k48) > 10
    assert abs(k48) < 0.3 * abs(p48)


# ------------------------------------------------------------ boundaries
def _poiseuille(ny, omega, g=1e-6, steps=None, plates=False, q=None):
    """Body-force driven channel, walls in y.  plates=True models the walls
    as obstacle rows (y = 0 and y = ny-1) with wall distance q."""
    nu = (1 / omega - 0.5) / 3
    if steps is None:
        steps = int(12 * ny * ny / nu)
    if plates:
        solid = np.zeros((1, ny, 1), np.uint8)
        solid[0, 0, 0] = solid[0, ny - 1, 0] = 1
        p = lbm.make_params((1, ny, 1), periodic=(1, 1, 1), omega1=omega, force=(g, 0, 0),
                            obstacle_bc=0 if q is None else 1)
        links = None
        if q is not None:
            c, _ = lbm.lattice()
            cells, dirs, qs = [], [], []
            for i in range(27):
                if c[i, 1] == -1:
                    cells.append(1), dirs.append(i), qs.append(q)
                if c[i, 1] == 1:
                    cells.append(ny - 2), dirs.append(i), qs.append(q)
            links = (np.array(cells), np.array(dirs), np.array(qs))
        r = lbm.Run(p, solid=solid, links=links)
    else:
        p = lbm.make_params((1, ny, 1), periodic=(1, 0, 1), omega1=omega, force=(g, 0, 0))
        r = lbm.Run(p)
    r.step(steps, forces=plates)
    _, u = r.macroscopic()
    return r, u[0, 0, :, 0], nu


def test_poiseuille_profile_walls():
    """Halfway walls at y = -1/2 and ny - 1/2: u = g/(2 nu) (y+1/2)(ny-1/2-y),
    error O(dx^2)."""
    errs = []
    for ny in (8, 16):
        _, u, nu = _poiseuille(ny, 1.3)
        y = np.arange(ny)
        ua = 1e-6 / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
        errs.append(np.linalg.norm(u - ua) / np.linalg.norm(ua))
    assert errs[1] < 5e-3
    assert errs[0] / max(errs[1], 1e-16) > 3.0 or errs[1] < 1e-6


def test_wall_force_balances_body_force():
    """Walls as obstacle rows: in steady state the momentum-exchange force
    on the obstacle equals g times the number of fluid cells."""
    r, _, _ = _poiseuille(12, 1.3, plates=True)
    F = np.array(r.forces[-1])
    assert abs(F[0] - 1e-6 * 10) < 1e-6 * 10 * 1e-6
    assert abs(F[1]) < 1e-15 and abs(F[2]) < 1e-15


def test_interpolated_bounce_back_half_equals_halfway():
    """q = 1/2 in the interpolated scheme reproduces halfway bounce-back
    bitwise."""
    from inputs import sphere_channel, perturbation
    g = sphere_channel((24, 12, 12), center=(8.0, 5.5, 5.5), radius=2.5)
    u0 = perturbation(g.shape, 0, 5e-4, g.solid)
    cell, d, _ = g.links
    half = (cell, d, np.full(cell.size, 0.5))
    runs = []
    for bc, links in ((0, None), (1, half)):
        p = lbm.make_params(g.shape, nu=0.01, u_in=0.05, obstacle_bc=bc)
        r = lbm.Run(p, solid=g.solid, links=links, u0=u0).step(10)
        runs.append(r)
    assert np.array_equal(runs[0].fbar, runs[1].fbar)
    assert np.array_equal(np.array(runs[0].forces), np.array(runs[1].forces))


def test_interpolated_bounce_back_stable_where_obstacle_meets_wall():
    """A spanwise cylinder touching the z walls with small wall distances
    (q = 0.1): links with no fluid node behind them fall back to halfway
    bounce-back, and the flow stays bounded (the q >= 1/2 formula applied at
    q < 1/2 would amplify by 1/(2q))."""
    from inputs import spanwise_cylinder
    geo = spanwise_cylinder((64, 32, 16), center=(19.2, 15.5), diameter=8.0)
    cell, d, q = geo.links
    for qq in (0.1, 0.3):
        p = lbm.make_params(geo.shape, nu=0.0008, u_in=0.05, obstacle_bc=1)
        r = lbm.Run(p, solid=geo.solid, links=(cell, d, np.full_like(q, qq))).step(150, forces=False)
        _, u = r.macroscopic()
        assert np.abs(u).max() < 0.2


def test_interpolated_poiseuille_second_order():
    """Plates at y = 1 - q and ny - 2 + q (off-lattice): the linear
    interpolated bounce-back converges at second order."""
    for q in (0.25, 0.75):
        errs = []
        for ny in (10, 18):
            _, u, nu = _poiseuille(ny, 1.3, plates=True, q=q)
            y = np.arange(ny)
            ylo, yhi = 1 - q, ny - 2 + q
            ua = 1e-6 / (2 * nu) * (y - ylo) * (yhi - y)
            ua[0] = ua[-1] = 0.0
            errs.append(np.linalg.norm(u[1:-1] - ua[1:-1]) / np.linalg.norm(ua[1:-1]))
        assert errs[1] < 2e-2
        assert errs[0] / errs[1] > 3.0, (q, errs)


def test_uniform_flow_with_inlet_and_outlet_is_fixed_point():
    """Uniform u_in between a velocity inlet and a zero-gradient outlet
    (periodic in y, z) stays exactly uniform: 6 w_i u_in c_ix equals
    f_eq_i - f_eq_ibar at rho = 1."""
    p = lbm.make_params((12, 4, 4), periodic=(0, 1, 1), nu=0.02, u_in=0.05)
    u0 = np.zeros((3, 4, 4, 12))
    u0[0] = 0.05
    r = lbm.Run(p, u0=u0)
    f0 = r.fbar.copy()
    r.step(40, forces=False)
    assert np.abs(r.fbar - f0).max() < 1e-15


def test_walled_channel_develops_no_slip():
    """Inlet-driven channel with walls: the mean velocity near the walls
    falls below the centre-line velocity, mass stays bounded."""
    p = lbm.make_params((16, 8, 8), nu=0.02, u_in=0.05)
    r = lbm.Run(p).step(200, forces=False)
    rho, u = r.macroscopic()
    prof = u[0, :, :, 8]
    assert prof[4, 4] > prof[0, 4] and prof[4, 4] > prof[4, 0]
    assert np.all(np.isfinite(r.fbar))


def _fields_of(fbar, force=(0.0, 0.0, 0.0)):
    """(u, v, w, p) of a pre-collision state by the definitions of the
    macroscopic quantities: rho = sum f, u = (sum f c + F/2)/rho,
    p = (rho - 1)/3."""
    c, _ = lbm.lattice()
    f = fbar.reshape(27, -1)
    d = f.sum(0)
    u = (c.T.astype(np.float64) @ f + 0.5 * np.asarray(force, float)[:, None]) / (1.0 + d)
    return np.concatenate([u, (d / 3.0)[None]], 0).reshape((4,) + fbar.shape[1:])


def test_mean_fields_sample_the_pre_collision_state():
    """Averaging (Sec. 2; reading R11): the sample of step n is the
    pre-collision state of step n, p = (rho - 1)/3.  One step from an
    equilibrium of known rho0, u0 must give means u0 + F/(2 rho0) and
    (rho0 - 1)/3 exactly: a post-collision sample would carry F/rho0 more
    velocity (the collision adds the body force F), a post-streaming one
    the streamed fields, and p = rho - 1 three times the pressure.  Two
    steps average the initial and the once-stepped state."""
    shape = (8, 6, 5)
    rng = np.random.default_rng(11)
    rho0 = 1.0 + 0.02 * rng.standard_normal((5, 6, 8))
    u0 = 0.03 * rng.standard_normal((3, 5, 6, 8))
    F = (2e-4, -1e-4, 3e-4)
    p = lbm.make_params(shape, periodic=(1, 1, 1), nu=0.02, force=F, avg_start=0)
    r = lbm.Run(p, rho0=rho0, u0=u0)
    f0 = r.fbar.copy()
    r.step(1, forces=False)
    m = r.mean_fields()
    expect_u = u0 + np.asarray(F)[:, None, None, None] / (2.0 * rho0)
    assert np.abs(m[:3] - expect_u).max() < 1e-15
    assert np.abs(m[3] - (rho0 - 1.0) / 3.0).max() < 1e-15
    assert np.abs(_fields_of(f0, F) - m).max() < 1e-15
    f1 = r.fbar.copy()
    r.step(1, forces=False)
    m2 = r.mean_fields()
    assert r.count == 2
    assert np.abs(m2 - 0.5 * (_fields_of(f0, F) + _fields_of(f1, F))).max() < 1e-15
    # a window starting at step 1 holds only the second state
    p1 = lbm.make_params(shape, periodic=(1, 1, 1), nu=0.02, force=F, avg_start=1)
    r1 = lbm.Run(p1, rho0=rho0, u0=u0).step(2, forces=False)
    assert r1.count == 1
    assert np.abs(r1.mean_fields() - _fields_of(f1, F)).max() < 1e-15


def test_snapshots_are_taken_at_snap_start_plus_multiples_of_the_period():
    """Snapshots (Sec. 2, 25 steps apart; reading R12): the FP64 fields of
    the pre-collision states of steps snap_start + k snap_every, here
    2, 5, 8 of a 10-step run, equal to the states stepped one by one."""
    shape = (8, 6, 5)
    rng = np.random.default_rng(12)
    u0 = 0.03 * rng.standard_normal((3, 5, 6, 8))
    p = lbm.make_params(shape, periodic=(1, 1, 1), nu=0.02, avg_start=10 ** 6, snap_every=3, snap_start=2)
    r = lbm.Run(p, u0=u0).step(10, forces=False, snap_cap=10)
    assert len(r.snaps) == 3
    ref = lbm.Run(p, u0=u0)
    states = []
    for _ in range(10):
        states.append(_fields_of(ref.fbar))
        ref.step(1, forces=False)
    for k, n in enumerate((2, 5, 8)):
        assert np.abs(r.snaps[k].reshape(4, 5, 6, 8) - states[n]).max() < 1e-15, n


def _one_step_with_post(p, fbar, solid=None):
    """The oracle's state after one step, and every cell's post-collision
    populations computed cell by cell with lbm.collide."""
    r = lbm.Run(p, solid=solid, fbar=fbar).step(1, forces=False)
    post = np.zeros_like(fbar)
    nz, ny, nx = fbar.shape[1:]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid is None or not solid[z, y, x]:
                    post[:, z, y, x] = lbm.collide(p, fbar[:, z, y, x])
    return r.fbar, post


def test_outlet_inlet_and_walls_at_the_population_level():
    """Boundary rules of the channel (Sec. 3.1; readings R6-R8), checked on
    every boundary population after one step of a state that varies along
    x, y and z (so that copying the wrong column, bouncing the wrong
    population or dropping the inlet term fails):
      outlet, zero gradient: a population entering the last column from
        outside (c_x = -1) equals what the last column itself emits in that
        direction from the cell behind it, post(nx - 1, y - c_y, z - c_z);
      inlet at x = -1/2, moving-wall bounce-back with rho_w = 1: a
        population entering column 0 (c_x = +1) is the cell's own opposite
        post-collision population plus 6 w_i c_ix u_in;
      walls at y = -1/2, ny - 1/2 (halfway): the cell's own opposite
        population, taking precedence over inlet and outlet."""
    shape = (10, 6, 4)
    nx, ny, nz = shape
    rng = np.random.default_rng(13)
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = 0.05 + 0.02 * rng.standard_normal((nz, ny, nx))
    u0[1:] = 0.02 * rng.standard_normal((2, nz, ny, nx))
    rho0 = 1.0 + 0.01 * rng.standard_normal((nz, ny, nx))
    p = lbm.make_params(shape, periodic=(0, 0, 1), nu=0.02, u_in=0.05)
    f0 = lbm.init(p, rho0=rho0, u0=u0)
    f1, post = _one_step_with_post(p, f0)
    c, w = lbm.lattice()
    checked = {"outlet": 0, "inlet": 0, "wall": 0}
    for z in range(nz):
        for y in range(ny):
            for x in (0, nx - 1):
                for i in range(27):
                    cx_, cy_, cz_ = c[i]
                    sy, sz = y - cy_, (z - cz_) % nz
                    if sy < 0 or sy >= ny:
                        expect = post[26 - i, z, y, x]
                        checked["wall"] += 1
                    elif x == 0 and cx_ == 1:
                        expect = post[26 - i, z, y, x] + 6.0 * w[i] * cx_ * 0.05
                        checked["inlet"] += 1
                    elif x == nx - 1 and cx_ == -1:
                        expect = post[i, sz, sy, nx - 1]
                        checked["outlet"] += 1
                    else:
                        continue
                    assert abs(f1[i, z, y, x] - expect) < 1e-16, (x, y, z, i)
    assert min(checked.values()) > 50
    # the outlet copy is not the interior pull: column nx - 2 differs
    assert np.abs(post[:, :, :, nx - 1] - post[:, :, :, nx - 2]).max() > 1e-4


# ------------------------------------------------------------ whole oracle
def _box_cases():
    rng = np.random.default_rng(7)
    cases = []
    shape = (8, 8, 8)
    u0 = 0.02 * rng.standard_normal((3, 8, 8, 8))
    cases.append(("periodic", dict(periodic=(1, 1, 1)), None, u0, 0.0))
    cases.append(("channel", dict(periodic=(0, 0, 0)), None, 0.1 * u0, 0.05))
    solid = np.zeros((8, 8, 8), np.uint8)
    solid[3:5, 3:5, 3:5] = 1
    u1 = 0.1 * u0.copy()
    u1[:, solid.astype(bool)] = 0
    cases.append(("obstacle", dict(periodic=(0, 0, 0)), solid, u1, 0.05))
    cases.append(("obstacle-periodic", dict(periodic=(1, 1, 1)), solid, u1 + np.array([0.03, 0, 0])[:, None, None, None] * (1 - solid), 0.0))
    return shape, cases


@pytest.mark.parametrize("mode", [0, 1])
def test_brute_force_agreement_8cube(mode):
    """Two independent implementations (C: direct sums, closed-form
    cumulants, per-axis inverse; numpy: binomial shifts, partition sums,
    27x27 solve, index-table streaming) agree over 40 steps."""
    shape, cases = _box_cases()
    omega = 1.95 if mode == 1 else 1.7
    for name, kw, solid, u0, u_in in cases:
        p = lbm.make_params(shape, nu=(1 / omega - 0.5) / 3, u_in=u_in, mode=mode, **kw)
        r = lbm.Run(p, solid=solid, u0=u0)
        f0 = r.fbar.copy()
        r.step(40, forces=False)
        fb = brute.run(shape, 40, f0, omega, periodic=kw["periodic"], solid=solid, u_in=u_in, mode=mode)
        scale = np.abs(fb).max()
        err = np.abs(r.fbar - fb).max() / scale
        assert err < 1e-12, (name, err)


def test_storage_rounding_is_round_to_nearest_even():
    assert lbm.round_storage(1.0 + 2 ** -11, "f16") == 1.0          # tie -> even
    assert lbm.round_storage(1.0 + 3 * 2 ** -11, "f16") == 1.0 + 2 ** -9
    assert lbm.round_storage(1.0 + 2 ** -8, "bf16") == 1.0
    assert lbm.round_storage(1.0 + 3 * 2 ** -8, "bf16") == 1.0 + 2 ** -6
    assert lbm.round_storage(3 * 2 ** -25, "f16") == 2 ** -23        # subnormal tie -> even
    assert lbm.round_storage(70000.0, "f16") == math.inf
    x = np.float64(0.1)
    assert lbm.round_storage(x, "f32") == float(np.float32(x))
    # compare with numpy's float16 conversion on random values
    v = RNG.standard_normal(2000) * 10.0 ** RNG.uniform(-7, 4, 2000)
    for a in v:
        assert lbm.round_storage(a, "f16") == float(np.float16(a))
