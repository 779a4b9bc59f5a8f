"""Von Neumann screen (Sec. 3.1) of the step: the library's analytic growth
matrix against the oracle's, the oracle's growth matrix against closed forms
(momentum conservation, viscous decay of a shear wave), and the screen's
verdict against the method itself run from small noise (no GPU; the screen
is host code behind the C ABI)."""
import math

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P


@pytest.fixture(scope="module")
def L():
    from paper_2306_08216_amd import _lib
    return _lib


def _screen(L, prob, u0, v0, nk):
    from paper_2306_08216_amd.solver import params_of
    keep = []
    return L.mdf_stability(params_of(prob, keep), u0, v0, nk)


@pytest.mark.parametrize("u0,v0,nu,cfl", [(0.0, 0.0, 0.01, 0.5), (0.05, -0.03, 0.002, 0.5),
                                          (0.1, 0.1, 0.0005, 0.9), (-0.2, 0.05, 0.02, 0.3)])
def test_screen_matches_oracle_growth_matrix(L, u0, v0, nu, cfl):
    """Spectral radius of every mode of an 8 x 8 periodic grid: the library's
    closed-form growth matrix equals the oracle's measured one."""
    from oracle import orc_stability as S
    prob = P.taylor_green(8, u0=0.0, nu=nu, cfl=cfl)
    rho, worst = _screen(L, prob, u0, v0, 8)
    for mx in range(-3, 5):
        for my in range(-3, 5):
            ro = S.spectral_radius(S.growth_matrix(prob, u0, v0, mx, my))
            assert rho[my + 3, mx + 3] == pytest.approx(ro, abs=1e-9), (mx, my)
    assert worst[0] == pytest.approx(rho.max(), abs=0.0)


def test_oracle_growth_matrix_conserves_momentum(orc):
    """At theta = 0 the step keeps u = sum_j f_j and v = sum_j g_j (eq. 2.3.4 and
    the telescoping transport): both sums are left eigenvectors with eigenvalue 1."""
    from oracle import orc_stability as S
    prob = P.taylor_green(8, nu=0.003)
    M = S.growth_matrix(prob, 0.04, -0.02, 0, 0)
    eu = np.r_[np.ones(5), np.zeros(5)]
    ev = np.r_[np.zeros(5), np.ones(5)]
    np.testing.assert_allclose(eu @ M, eu, atol=1e-10)
    np.testing.assert_allclose(ev @ M, ev, atol=1e-10)
    assert S.spectral_radius(M) == pytest.approx(1.0, abs=1e-10)


def test_oracle_growth_matrix_shear_wave_decay(orc):
    """A shear wave of wavenumber k decays as exp(-nu k^2 t) (the momentum
    equation recovered in Sec. 2.3 with nu = c_s^2/s): on the 64^2 grid of
    [0, 2 pi]^2 the mode k = 1 has an eigenvalue exp(-nu dt) to 1e-6."""
    from oracle import orc_stability as S
    nu = 0.01
    prob = P.taylor_green(64, nu=nu)
    dt = orc.Oracle(prob).dt
    lam = np.linalg.eigvals(S.growth_matrix(prob, 0.0, 0.0, 1, 0))
    assert np.min(np.abs(lam - math.exp(-nu * dt))) < 1e-6
    assert np.max(np.abs(lam)) < 1.0


def _noise_growth_rate(orc, u0, v0, nu, cfl, n=16, seed=3, t0=400, t1=800):
    """Per-step growth of the state's deviation from its mean between steps t0
    and t1, for the uniform flow (u0, v0) plus 1e-9 noise."""
    rng = np.random.default_rng(seed)
    prob = P.Problem(nx=n, ny=n, lx=2 * math.pi, ly=2 * math.pi, nu=nu, cfl=cfl,
                     u0=u0 + 1e-9 * rng.standard_normal((n, n)), v0=v0 + 1e-9 * rng.standard_normal((n, n)),
                     p0=1e-9 * rng.standard_normal((n, n)))
    o = orc.Oracle(prob)

    def dev():
        f = o.f()
        return np.abs(f - f.mean(axis=(1, 2), keepdims=True)).max()
    o.step(t0)
    d0 = dev()
    o.step(t1 - t0)
    return (dev() / d0) ** (1.0 / (t1 - t0))


def test_screen_verdict_matches_the_method(orc, L):
    """Where the screen finds modes with radius above 1 the method itself,
    started from the uniform flow plus 1e-9 noise, amplifies the deviation by
    the largest radius per step (measured over steps 400-800 once the other
    modes have died out); where every radius is at most 1 it decays."""
    n = 16
    unstable = (0.1, 0.1, 0.0005, 0.9)
    stable = (0.05, -0.03, 0.002, 0.5)
    prob = P.taylor_green(n, nu=unstable[2], cfl=unstable[3])
    _, worst_u = _screen(L, prob, unstable[0], unstable[1], n)
    prob = P.taylor_green(n, nu=stable[2], cfl=stable[3])
    _, worst_s = _screen(L, prob, stable[0], stable[1], n)
    assert worst_u[0] > 1.02 and worst_s[0] <= 1.0 + 1e-12
    assert _noise_growth_rate(orc, *unstable) == pytest.approx(worst_u[0], abs=1e-3)
    assert _noise_growth_rate(orc, *stable) < 1.0


def test_screen_rejects_bad_input(L):
    from paper_2306_08216_amd.solver import params_of
    prob = P.taylor_green(8)
    keep = []
    p = params_of(prob, keep)
    with pytest.raises(L.MdfError):
        L.mdf_stability(p, 0.0, 0.0, 0)
    bad = P.taylor_green(8)
    bad.pl_n, bad.nu_min, bad.nu_max = 0.5, 1e-5, 1e-1
    with pytest.raises(L.MdfError):
        L.mdf_stability(params_of(bad, keep), 0.0, 0.0, 8)
    with pytest.raises(L.MdfError):
        L.mdf_stability(p, float("nan"), 0.0, 8)
