"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element, on the same seeded inputs.  Bar: max |GPU - oracle| <= 1e-12 on
the FP64 state after the stated number of steps."""
import functools
import math
import sys

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08216_amd.solver import Solver
    return Solver


@functools.lru_cache(maxsize=None)
def oracle_run(key):
    from oracle.orc import Oracle
    prob, steps = CASES[key]()
    o = Oracle(prob)
    o.step(steps)
    return o, prob, steps


def _wall_field(n, seed=3, amp=0.02):
    """Smooth velocity field vanishing on the walls of [0,1]^2 (sine modes)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((n, n))
    v = np.zeros((n, n))
    for _ in range(6):
        kx, ky = rng.integers(1, 5, size=2)
        a, b = rng.normal(size=2) * amp / 3
        u += a * np.sin(math.pi * kx * X) * np.sin(math.pi * ky * Y)
        v += b * np.sin(math.pi * ky * X) * np.sin(math.pi * kx * Y)
    return u, v, np.zeros((n, n))


def _wall_problem(n, pl_n=1.0, beta=None):
    prob = P.cavity(n, re=1000.0) if pl_n == 1.0 else P.powerlaw_cavity(n, pl_n=pl_n)
    if beta is None and pl_n != 1.0:
        prob.inv_dx_x = prob.inv_dx_y = None
        prob.dx_min = 0.0
    u, v, p = _wall_field(n)
    prob.u0, prob.v0, prob.p0 = u, v, p
    return prob


def _ragged():
    u, v, p = P.random_vortex_fields(96, seed=11, kmax=6, urms=0.03)
    u, v, p = u[:52, :80].copy(), v[:52, :80].copy(), p[:52, :80].copy()
    return P.Problem(nx=80, ny=52, lx=2 * math.pi * 80 / 96, ly=2 * math.pi * 52 / 96, nu=0.004, u0=u, v0=v, p0=p)


def _wallx():
    prob = P.poiseuille(40, nu=0.01, force=1e-4)
    prob.bc_x, prob.bc_y = P.WALL, P.PERIODIC
    prob.fx, prob.fy = 0.0, 1e-4
    u, v, _ = _wall_field(40, seed=5)
    prob.u0, prob.v0 = v.T.copy(), u.T.copy()
    return prob


def _mapped():
    n = 64
    prob = P.taylor_green(n, nu=0.005)
    pos, g, dxm = P.sine_mapping(n, 0.2)
    X, Y = np.meshgrid(pos, pos, indexing="xy")
    prob.u0 = 0.01 * np.sin(X) * np.cos(Y)
    prob.v0 = -0.01 * np.cos(X) * np.sin(Y)
    prob.p0 = 0.25e-4 * (np.cos(2 * X) + np.cos(2 * Y))
    prob.inv_dx_x, prob.inv_dx_y, prob.dx_min = g, g.copy(), dxm
    return prob


def _plcav(pl_n):
    prob = P.powerlaw_cavity(64, pl_n=pl_n)
    u, v, p = _wall_field(64, seed=9, amp=0.05 if pl_n < 1 else 0.02)
    prob.u0, prob.v0 = u, v
    assert pl_n < 1 or prob.nu_max == 0.004   # the shear-thickening ceiling of 4 nu_ref
    return prob


def _stretched_cavity(n, pl_n):
    """Cavity on the tanh-stretched grid, wide enough for segments that touch
    no wall (the kernels run those through their wall-free march)."""
    if pl_n == 1.0:
        prob = P.cavity(n, re=1000.0)
        _, g, dxm = P.tanh_mapping(n, 1.5)
        prob.inv_dx_x, prob.inv_dx_y, prob.dx_min = g, g.copy(), dxm
    else:
        prob = P.powerlaw_cavity(n, pl_n=pl_n)
    u, v, p = _wall_field(n, seed=13, amp=0.03)
    prob.u0, prob.v0, prob.p0 = u, v, p
    return prob


CASES = {
    "tg64": lambda: (P.taylor_green(64, u0=0.01, nu=0.01), 1000),
    "ragged": lambda: (_ragged(), 200),
    "cavity128": lambda: (P.cavity(128, re=1000.0), 1000),
    "cavity_field48": lambda: (_wall_problem(48), 300),
    "cavity_field520": lambda: (_wall_problem(520), 30),
    "poiseuille32": lambda: (P.poiseuille(32, nu=0.01, force=1e-4), 500),
    "wallx40": lambda: (_wallx(), 300),
    "mapped64": lambda: (_mapped(), 200),
    "plcav_n0.5": lambda: (_plcav(0.5), 200),
    "plcav_n1.5": lambda: (_plcav(1.5), 200),
    "stretched144": lambda: (_stretched_cavity(144, 1.0), 100),
    "plstretched144": lambda: (_stretched_cavity(144, 0.5), 100),
}


def _run_gpu(Solver, prob, steps, variant, shape=(0, 0)):
    s = Solver(prob, device="cuda:0")
    s.set_kernel(variant, *shape)
    s.step(steps)
    f = s.save().cpu().numpy()
    u, v, p = (t.cpu().numpy() for t in s.moments())
    s.close()
    return f, u, v, p


def _compare(key, Solver, variant, shape=(0, 0)):
    o, prob, steps = oracle_run(key)
    say(f"[gpu parity] case={key} nx={prob.nx} ny={prob.ny} steps={steps} variant={variant} shape={shape}")
    f, u, v, p = _run_gpu(Solver, prob, steps, variant, shape)
    fo = o.f()
    uo, vo, po = o.moments()
    err = np.abs(f - fo).max()
    say(f"    max|df|={err:.3e} max|f|={np.abs(fo).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL, (key, err)
    assert np.abs(u - uo).max() <= TOL and np.abs(v - vo).max() <= TOL and np.abs(p - po).max() <= TOL
    return o


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 8, 2)), (1, (128, 5, 3)), (1, (128, -1, 2)), (1, (256, -1, 2)), (1, (256, -1, 3)), (2, (0, 0)), (2, (0, 64, 2)),
                                           (2, (0, 3, 3))])
def test_taylor_green_64_1000_steps(gpu, variant, shape):
    """The 64^2 Taylor-Green configuration: 1000 FP64 steps agree with the oracle to 1e-12."""
    _compare("tg64", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 7)), (1, (128, 3)), (2, (0, 1)), (2, (0, 7, 3))])
def test_ragged_periodic(gpu, variant, shape):
    """80 x 52 periodic grid: several strips, a ragged last strip, segments of 1-7 rows."""
    _compare("ragged", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 9)), (1, (128, 9, 3)), (1, (128, -1, 2)), (1, (256, 9, 2)), (1, (64, -2, 3)), (2, (0, 0)),
                                           (2, (0, 9, 3)), (2, (0, -2))])
def test_cavity_128_1000_steps(gpu, variant, shape):
    """Lid-driven cavity (the 1024^2 configuration at 128^2): walls on all sides, lid 0.1."""
    _compare("cavity128", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 5)), (2, (0, 5)), (2, (0, 48, 3))])
def test_cavity_with_interior_field(gpu, variant, shape):
    _compare("cavity_field48", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(1, (64, -1, 2)), (1, (128, -1, 3)), (1, (256, -1, 2)), (1, (256, 40, 2)), (1, (256, -1, 3)),
                                           (2, (0, -1))])
def test_wide_cavity_every_tile_width(gpu, variant, shape):
    """520^2 cavity with an interior field: several strips at every tile width
    (wall strips and a strip between them), balanced and fixed segments."""
    _compare("cavity_field520", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 6)), (2, (0, 6)), (2, (0, 32, 3))])
def test_poiseuille_walls_in_y(gpu, variant, shape):
    _compare("poiseuille32", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 6)), (2, (0, 6)), (2, (0, 13, 3))])
def test_walls_in_x_periodic_y(gpu, variant, shape):
    _compare("wallx40", gpu, variant, shape)


@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 10)), (2, (0, 10)), (2, (0, 4, 3))])
def test_mapped_periodic_grid(gpu, variant, shape):
    _compare("mapped64", gpu, variant, shape)


@pytest.mark.parametrize("pl_n", [0.5, 1.5])
@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 8)), (1, (64, 8, 3)), (2, (0, 8)), (2, (0, 5, 3))])
def test_powerlaw_stretched_cavity(gpu, pl_n, variant, shape):
    """Power-law cavity on the tanh-stretched grid (the 2048^2 configuration at 64^2)."""
    _compare(f"plcav_n{pl_n}", gpu, variant, shape)


@pytest.mark.parametrize("key", ["stretched144", "plstretched144"])
@pytest.mark.parametrize("variant,shape", [(1, (64, 10)), (1, (128, 10, 3)), (1, (256, 10, 2)), (1, (256, 10, 3)), (2, (0, 10)),
                                           (2, (0, 17, 3))])
def test_stretched_cavity_interior_segments(gpu, key, variant, shape):
    """Mapped-grid cavities (Newtonian and power law) with segments away from
    every wall next to segments that meet the walls."""
    _compare(key, gpu, variant, shape)


@pytest.mark.parametrize("key", ["tg64", "cavity128", "plcav_n0.5", "plcav_n1.5", "smallest_cavity5x5",
                                 "smallest_periodic5x7", "smallest_wally9x5", "extent_wide32768x6"])
def test_derived_and_diagnostics(gpu, key):
    """mdf_derived (eqs. 2.4.1-2.4.5, all 14 planes) and mdf_diagnostics against the oracle."""
    o, prob, steps = oracle_run(key)
    say(f"[gpu derived] case={key}")
    s = gpu(prob, device="cuda:0")
    s.step(steps)
    d = s.derived().cpu().numpy()
    do = o.derived()
    bound = derived_bounds(prob, o, do)
    for k in range(14):
        err = np.abs(d[k] - do[k]).max()
        assert err <= bound[k], (k, err, bound[k])
    # a subset in mask order
    mask = (1 << 1) | (1 << 6) | (1 << 12)
    sub = s.derived(mask).cpu().numpy()
    for i, k in enumerate((1, 6, 12)):
        assert np.abs(sub[i] - do[k]).max() <= bound[k]
    diag, status = s.diagnostics()
    dio = o.diagnostics()
    assert status == 0
    # bounds propagated from the state tolerance: a moment sums five
    # components (error <= 5 TOL); KE moves by at most sum |u| |du| dA <=
    # 10 TOL sqrt(2 KE area) (Cauchy-Schwarz); enstrophy by max|omega| times the
    # vorticity bound times the area; the central-difference divergence by
    # 10 TOL times the largest 1/dx
    area = dio[7]
    sum_rel = prob.nodes * 2.0 ** -52         # sums over n nodes in different orders: up to n ulps
    assert abs(diag[2] - dio[2]) <= 10 * TOL * np.sqrt(2 * dio[2] * area) + sum_rel * dio[2] + 1e-30
    assert abs(diag[4] - dio[4]) <= 10 * TOL
    assert diag[7] == pytest.approx(dio[7], rel=sum_rel)
    assert abs(diag[3] - dio[3]) <= 2 * np.abs(do[12]).max() * bound[12] * area + sum_rel * dio[3] + 1e-30
    gmax = prob.cfl / (prob.c * o.dt)          # largest 1/dx, since dt = cfl dx_min / c
    assert abs(diag[5] - dio[5]) <= 10 * TOL * gmax
    assert abs(diag[0] - dio[0]) <= 1e-12 * max(1.0, np.abs(o.moments()[0]).sum())
    assert abs(diag[1] - dio[1]) <= 1e-12 * max(1.0, np.abs(o.moments()[1]).sum())
    assert diag[6] == 0.0
    s.close()


def derived_bounds(prob, o, do):
    """Largest admissible |GPU - oracle| per derived plane, propagated from the
    state tolerance: every plane is a sum of two differences of f_hat - f^eq
    (|c_j| = c), each within 2 TOL, divided by nu + c_s^2 dt/2 (eq. 2.4.1 from
    the stored state); the stress planes carry the factor 2 nu (eq. 2.4.4),
    the viscosity plane is compared relatively (its root is solved to
    rounding).  The division by nu + theta amplifies the state's rounding, by
    up to 1e3 in the low-viscosity runs here, which is why these planes are
    not held to the state's 1e-12."""
    nu_plane = do[13]
    theta = 0.2 * prob.c ** 2 * o.dt
    amp = 1.0 / (nu_plane.min() + theta)
    base = 8 * TOL * prob.c * amp
    b = [base] * 14
    for k in (4,):
        b[k] = 2 * base                         # div u: four differences
    for k in (8, 9, 10):
        b[k] = base * 2 * nu_plane.max()
    b[13] = 1e-12 * nu_plane.max()
    # a power-law viscosity agrees to ~1e-13 relative, which moves every plane
    # relatively by as much
    return [bk + 1e-12 * np.abs(do[k]).max() for k, bk in enumerate(b)]


def test_save_load_resume_and_determinism(gpu):
    """n steps + save/load + n steps equals 2n steps bit for bit; two runs are bitwise equal."""
    import torch
    prob = P.cavity(96, re=400.0)
    say("[gpu resume] cavity96")
    a = gpu(prob, device="cuda:0")
    a.step(100)
    snap = a.save().clone()
    a.step(100)
    fa = a.save().cpu().numpy()
    b = gpu(prob, device="cuda:0")
    b.load(snap)
    b.step(100)
    fb = b.save().cpu().numpy()
    c = gpu(prob, device="cuda:0")
    c.step(200)
    fc = c.save().cpu().numpy()
    assert np.array_equal(fa, fc)
    assert np.array_equal(fb, fc)
    assert c.steps == 200 and b.steps == 100
    for s in (a, b, c):
        s.close()
    del torch


def test_diagnostics_flags_non_finite_state(gpu):
    """A non-finite value injected into the loaded state trips MDF_EUNSTABLE."""
    import torch
    prob = P.taylor_green(32)
    s = gpu(prob, device="cuda:0")
    f = s.save()
    f[3, 5, 7] = float("nan")
    s.load(f.contiguous())
    diag, status = s.diagnostics()
    assert status == -4 and diag[6] >= 1
    s.close()
    del torch


def test_full_size_cavity_1024_default_launch(gpu):
    """The 1024^2 cavity at full size in the default (benchmarked) launch
    configuration: 3 steps from a smooth interior field, every node against
    the oracle."""
    from oracle.orc import Oracle
    prob = _wall_problem(1024)
    say("[gpu full-size] cavity 1024^2, 3 steps, default launch")
    s = gpu(prob, device="cuda:0")
    s.step(3)
    f = s.save().cpu().numpy()
    s.close()
    o = Oracle(prob)
    o.step(3)
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e}")
    assert err <= TOL


def test_full_size_powerlaw_2048_sampled(gpu):
    """The 2048^2 power-law stretched cavity at full size (n = 0.5): 1 step in the
    default launch configuration, every node against the oracle."""
    from oracle.orc import Oracle
    prob = P.powerlaw_cavity(2048, pl_n=0.5)
    u, v, p = _wall_field(2048, seed=13, amp=0.05)
    prob.u0, prob.v0 = u, v
    say("[gpu full-size] power-law cavity 2048^2 n=0.5, 1 step, default launch")
    s = gpu(prob, device="cuda:0")
    s.step(1)
    f = s.save().cpu().numpy()
    s.close()
    o = Oracle(prob)
    o.step(1)
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e}")
    assert err <= TOL


def test_autotune_restores_state_and_keeps_parity(gpu):
    """The single-run autotuner tries every kernel and partition scaling on the
    run itself; afterwards the state, step count and results are unchanged."""
    prob, steps = CASES["cavity128"]()
    say(f"[gpu parity] autotune on cavity128, then {steps} steps")
    s = gpu(prob, device="cuda:0")
    s.step(3)
    before = s.save().cpu().numpy()
    choice = s.autotune(4)
    assert int(choice[0]) in (1, 2) and int(choice[1]) in (2, 3) and choice[4] > 0 and int(choice[5]) in (64, 128)
    assert s.steps == 3 and np.array_equal(s.save().cpu().numpy(), before)
    s.step(steps - 3)
    o, _, _ = oracle_run("cavity128")
    err = np.abs(s.save().cpu().numpy() - o.f()).max()
    say(f"    choice={choice} max|df|={err:.3e}")
    assert err <= TOL
    s.close()


def test_tuning_cache_round_trip(gpu, tmp_path):
    """Solver.tuned: the first call tunes and stores the choice under the run's
    signature, the second reuses it; the state is untouched and parity holds."""
    import json
    prob, steps = CASES["cavity128"]()
    say("[gpu parity] tuning cache on cavity128")
    cache = str(tmp_path / "tuning.json")
    s = gpu(prob, device="cuda:0")
    before = s.save().cpu().numpy()
    choice, cached = s.tuned(cache, steps=3)
    assert not cached and int(choice[0]) in (1, 2) and int(choice[1]) in (64, 128, 256)
    assert np.array_equal(s.save().cpu().numpy(), before) and s.steps == 0
    assert json.load(open(cache))[s.signature()]["choice"] == list(choice)
    s2 = gpu(prob, device="cuda:0")
    choice2, cached2 = s2.tuned(cache)
    assert cached2 and tuple(choice2) == tuple(choice)
    s2.step(steps)
    o, _, _ = oracle_run("cavity128")
    err = np.abs(s2.save().cpu().numpy() - o.f()).max()
    say(f"    choice={choice} max|df|={err:.3e}")
    assert err <= TOL
    s.close()
    s2.close()


@pytest.mark.parametrize("pl_n", [0.5, 1.5])
def test_powerlaw_viscosity_over_many_decades(gpu, pl_n):
    """The local power-law viscosity (derived plane 13) of a state whose
    non-equilibrium parts span twelve decades, against the oracle's root of
    nu = K (g/(nu + theta))^(n-1) at every node.  The clamp is widened to
    [1e-12, 1] so that mostly the solve itself is compared, with nu on both
    sides of theta (the two regimes of the n = 3/2 cubic)."""
    import torch
    from oracle.orc import Oracle

    n = 64
    prob = P.powerlaw_cavity(n, pl_n=pl_n)
    prob.nu_min, prob.nu_max = 1e-12, 1.0
    say(f"[gpu powerlaw nu] pl_n={pl_n} n={n}")
    rng = np.random.default_rng(17)
    mag = 10.0 ** rng.uniform(-10.0, 2.0, (1, n, n))
    f = rng.standard_normal((10, n, n)) * mag
    o = Oracle(prob)
    o.set_f(f)
    nu_o = o.derived()[13]
    s = gpu(prob, device="cuda:0")
    s.load(torch.from_numpy(f).to("cuda:0"))
    nu = s.derived(1 << 13).cpu().numpy()[0]
    s.close()
    inside = (nu_o > prob.nu_min) & (nu_o < prob.nu_max)
    assert inside.mean() > 0.75                        # mostly the solve, not the clamp
    assert nu_o[inside].max() / nu_o[inside].min() > 1e4
    theta = 0.2 * prob.c ** 2 * o.dt                   # c_s^2 dt / 2 with c_s^2 = 2c^2/5
    assert 0.2 < (nu_o[inside] < theta).mean() < 0.8   # both regimes of the cubic
    rel = np.abs(nu - nu_o) / nu_o
    assert rel.max() <= 1e-13, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))


def _smallest(nx, ny, bc_x, bc_y, seed, lid=0.0, fx=0.0, fy=0.0):
    """A grid at the smallest size the boundary accepts (5 nodes on an axis):
    one strip whose halo lanes wrap (periodic) or clamp (walls) many times over,
    and segments whose row halos reach both y walls or wrap past both ends."""
    rng = np.random.default_rng(seed)
    u, v, p = (a * rng.standard_normal((ny, nx)) for a in (0.01, 0.01, 1e-4))
    for w, axis in ((bc_x, 1), (bc_y, 0)):
        if w == P.WALL:
            for a in (u, v):
                np.moveaxis(a, axis, 0)[[0, -1]] = 0.0
    dx = 0.25
    lx = dx * (nx - 1 if bc_x == P.WALL else nx)
    ly = dx * (ny - 1 if bc_y == P.WALL else ny)
    return P.Problem(nx=nx, ny=ny, lx=lx, ly=ly, nu=0.02, u0=u, v0=v, p0=p, bc_x=bc_x, bc_y=bc_y,
                     lid_u=lid, fx=fx, fy=fy, name=f"smallest_{nx}x{ny}")


SMALLEST = {
    "cavity5x5": lambda: (_smallest(5, 5, P.WALL, P.WALL, 21, lid=0.05), 60),
    "cavity7x6": lambda: (_smallest(7, 6, P.WALL, P.WALL, 22, lid=0.05), 60),
    "periodic5x7": lambda: (_smallest(5, 7, P.PERIODIC, P.PERIODIC, 23), 60),
    "periodic6x5": lambda: (_smallest(6, 5, P.PERIODIC, P.PERIODIC, 24), 60),
    "wallx5x9": lambda: (_smallest(5, 9, P.WALL, P.PERIODIC, 25, fy=1e-4), 60),
    "wally9x5": lambda: (_smallest(9, 5, P.PERIODIC, P.WALL, 26, fx=1e-4), 60),
}
CASES.update({"smallest_" + k: f for k, f in SMALLEST.items()})


@pytest.mark.parametrize("key", sorted(SMALLEST))
@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, 2, 2)), (1, (128, -1, 3)), (1, (256, -1, 2)), (1, (256, -1, 3)),
                                           (2, (0, 0)), (2, (0, 3, 3))])
def test_smallest_grids(gpu, key, variant, shape):
    """Degenerate sizes: 5 to 9 nodes per axis, every boundary combination,
    every kernel variant and tile width, element by element against the oracle."""
    _compare("smallest_" + key, gpu, variant, shape)


EXTENT = {
    "wide32768x6": lambda: (_smallest(32768, 6, P.PERIODIC, P.PERIODIC, 31), 12),
    "widecavity32768x5": lambda: (_smallest(32768, 5, P.WALL, P.WALL, 32, lid=0.05), 12),
    "tall6x32768": lambda: (_smallest(6, 32768, P.WALL, P.PERIODIC, 33, fy=1e-4), 12),
}
CASES.update({"extent_" + k: f for k, f in EXTENT.items()})


@pytest.mark.parametrize("key", sorted(EXTENT))
@pytest.mark.parametrize("variant,shape", [(0, (0, 0)), (1, (64, -1, 2)), (1, (256, -1, 2)), (2, (0, 0))])
def test_maximum_extent(gpu, key, variant, shape):
    """The largest extent the boundary accepts on one axis (32768 nodes) with
    the smallest on the other: hundreds of strips across one row, or one strip
    down thousands of rows, element by element against the oracle."""
    _compare("extent_" + key, gpu, variant, shape)


@pytest.mark.parametrize("key", ["ragged", "cavity_field48", "plcav_n0.5", "smallest_cavity5x5"])
def test_zero_steps_keep_the_initial_state(gpu, key):
    """Stepping by zero is the empty case: the state stays the initial
    equilibrium the oracle builds from (u0, v0, p0), and the step count stays 0."""
    from oracle.orc import Oracle
    prob, _ = CASES[key]()
    say(f"[gpu parity] zero steps case={key} nx={prob.nx} ny={prob.ny}")
    o = Oracle(prob)
    s = gpu(prob, device="cuda:0")
    s.step(0)
    from paper_2306_08216_amd._lib import MdfError
    with pytest.raises(MdfError):
        s.step(-1)            # rejected before any launch
    f = s.save().cpu().numpy()
    assert s.steps == 0
    s.close()
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e}")
    assert err <= TOL
