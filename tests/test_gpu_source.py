"""GPU parity of the mass source R (eq. 2.1.1; the pressure of eq. 2.3.23)
through the C ABI against the oracle, element by element, to 1e-12: the
manufactured divergent flows (periodic, walled, ragged, several tiles), a
source on a warped general mapping, a closed cavity with a source/sink pair and
a time-dependent force with a source; moments, derived quantities and
diagnostics; a full-size run; the kernel limits of a run with a source.

The oracle solves the definition of the pressure for P on each stored form
(dense (I + kappa Lambda~)^-1); the kernels add the closed-form offset
R (nu + kappa c_s^2)/2 to the plain sum."""
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


def _warped_source(n=40):
    prob = P.warped_taylor_green(n, shear=1, eps=0.2)
    X, Y = prob.node_xy
    prob.mass_source = 0.01 * np.cos(X) * np.cos(2.0 * Y)
    return prob


def _cavity_source(n=40):
    """A closed cavity (all walls, lid at the top) with a source/sink pair."""
    prob = P.cavity(n, re=100.0)
    X, Y = np.meshgrid(prob.node_x(), prob.node_y(), indexing="xy")
    prob.mass_source = 0.02 * np.cos(math.pi * X) * np.cos(math.pi * Y)
    return prob


def _pulsed_channel(n=40):
    prob = P.divergent_channel(n)
    prob.fx = 1e-4
    prob.force_harmonic, prob.force_omega, prob.force_phase = True, 0.4, 0.2
    return prob


CASES = {
    "divergent32": lambda: (P.divergent_flow(32), 300),
    "divergent_ragged37": lambda: (P.divergent_flow(37), 200),
    "divergent_tiles70": lambda: (P.divergent_flow(70), 60),
    "channel40": lambda: (P.divergent_channel(40), 300),
    "channel_ragged45": lambda: (P.divergent_channel(45), 200),
    "warped_source40": lambda: (_warped_source(40), 200),
    "cavity_source40": lambda: (_cavity_source(40), 300),
    "pulsed_channel40": lambda: (_pulsed_channel(40), 200),
}


@functools.lru_cache(maxsize=None)
def oracle_run(key):
    from oracle.orc import Oracle
    prob, steps = CASES[key]()
    o = Oracle(prob)
    o.step(steps)
    return o, prob, steps


@pytest.mark.parametrize("key", sorted(CASES))
def test_mass_source_parity(gpu, key):
    o, prob, steps = oracle_run(key)
    say(f"[gpu source] case={key} nx={prob.nx} ny={prob.ny} steps={steps}")
    s = gpu(prob, device="cuda:0")
    s.step(steps // 2)
    s.step(steps - steps // 2)
    f = s.save().cpu().numpy()
    u, v, p = (t.cpu().numpy() for t in s.moments())
    d = s.derived().cpu().numpy()
    diag, status = s.diagnostics()
    s.close()
    fo = o.f()
    err = np.abs(f - fo).max()
    say(f"    max|df|={err:.3e} max|f|={np.abs(fo).max():.3e}")
    assert np.all(np.isfinite(f))
    assert err <= TOL, (key, err)
    uo, vo, po = o.moments()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max(), np.abs(p - po).max()) <= TOL
    do = o.derived()
    assert np.abs(d[:13] - do[:13]).max() <= 1e-9 * max(1.0, np.abs(do[:13]).max())
    dio = o.diagnostics()
    assert status == 0
    assert abs(diag[2] - dio[2]) <= 1e-9 * dio[2] + 1e-30
    assert abs(diag[5] - dio[5]) <= 1e-9 * max(dio[5], 1e-12) + 1e-14


def test_source_follows_the_closed_form_on_the_gpu(gpu):
    """The library's own run of the manufactured divergent flow (16^2, nu =
    0.05, c = 4) reaches the closed form as the oracle does (GRE below 1.2e-2,
    the oracle's 8.5e-3 at the steady state)."""
    prob = P.divergent_flow(16, u0=0.01, nu=0.05)
    prob.c = 4.0
    s = gpu(prob, device="cuda:0")
    s.step(int(round(250.0 / s.dt)))
    u, v, _ = (t.cpu().numpy() for t in s.moments())
    s.close()
    ex = P.divergent_flow_exact(prob)
    gre = (np.abs(u - ex["u"]).sum() + np.abs(v - ex["v"]).sum()) / (np.abs(ex["u"]).sum() + np.abs(ex["v"]).sum())
    say(f"[gpu source] divergent16 steady GRE {gre:.3e}")
    assert gre < 1.2e-2


def test_zero_source_matches_the_plain_tiled_step(gpu):
    """R = 0 everywhere through the source kernels gives the plain tiled
    step exactly (the offsets add zero)."""
    prob = P.cavity(40, re=100.0)
    a = gpu(prob, device="cuda:0")
    a.set_kernel(0)
    prob0 = P.cavity(40, re=100.0)
    prob0.mass_source = np.zeros((40, 40))
    b = gpu(prob0, device="cuda:0")
    a.step(50)
    b.step(50)
    fa, fb = a.save().cpu().numpy(), b.save().cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(fa, fb)


def test_mass_source_full_size(gpu):
    """512^2 divergent flow, 3 steps, in the launch configuration of every run
    with a source (the tiled step), against the oracle on every node."""
    from oracle.orc import Oracle
    prob = P.divergent_flow(512)
    say("[gpu source] divergent512 steps=3")
    o = Oracle(prob, threads=8)
    o.step(3)
    s = gpu(prob, device="cuda:0")
    s.step(3)
    f = s.save().cpu().numpy()
    s.close()
    err = np.abs(f - o.f()).max()
    say(f"    max|df|={err:.3e}")
    assert err <= TOL


def test_mass_source_kernel_limits(gpu):
    """A run with a source has the tiled step only: the fused kernels are
    rejected and the autotuner reports variant 0 without changing the state."""
    from paper_2306_08216_amd._lib import MdfError
    o, prob, steps = oracle_run("divergent32")
    s = gpu(prob, device="cuda:0")
    for v in (1, 2):
        with pytest.raises(MdfError):
            s.set_kernel(v)
    choice = s.autotune(2)
    assert int(choice[0]) == 0 and s.steps == 0
    s.step(steps)
    err = np.abs(s.save().cpu().numpy() - o.f()).max()
    s.close()
    assert err <= TOL
