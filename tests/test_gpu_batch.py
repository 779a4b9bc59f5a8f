"""GPU parity of the batched step: one launch per step over many periodic
instances of different size and viscosity, each compared with its own oracle
run; graph replay against eager stepping; the autotuner leaves the state as
it found it.  Bar: max |GPU - oracle| <= 1e-12 (FP64 state)."""
import functools
import json
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
    from paper_2306_08216_amd.batch import BatchSolver
    return BatchSolver


def _mixed(count=10, seed=7):
    """Ragged sizes (strip and tile tails), nu spread over two decades."""
    rng = np.random.default_rng(seed)
    sizes = [40, 57, 64, 96, 113, 130, 64, 88, 150, 71][:count]
    probs = []
    for i, n in enumerate(sizes):
        nu = float(10 ** rng.uniform(-3, -1))
        probs.append(P.random_vortex(n, 500 + i, nu, kmax=6, urms=0.03))
    return probs


@functools.lru_cache(maxsize=None)
def _oracle_f(key, i, steps):
    from oracle.orc import Oracle
    probs = _mixed() if key == "mixed" else None
    o = Oracle(probs[i])
    o.step(steps)
    return o.f()


def test_batch_matches_each_instance_oracle(gpu):
    probs = _mixed()
    steps = 30
    say(f"[gpu batch] mixed count={len(probs)} sizes={[p.nx for p in probs]} steps={steps}")
    b = gpu(probs)
    assert b.workgroups > 0
    for i, p in enumerate(probs):
        assert b.dt(i) == pytest.approx(p.cfl * (p.lx / p.nx) / p.c, rel=1e-15)
    b.step(steps)
    b.synchronize()
    for i, p in enumerate(probs):
        f = b.save(i).cpu().numpy()
        err = np.abs(f - _oracle_f("mixed", i, steps)).max()
        say(f"    instance {i} n={p.nx} nu={p.nu:.3g} max|df|={err:.3e}")
        assert np.all(np.isfinite(f)) and err <= TOL
    b.close()


@pytest.mark.parametrize("variant,prefetch,rounds,tile_w", [(1, 2, 1, 64), (1, 3, 2, 64), (2, 3, 1, 64), (2, 2, 3, 64),
                                                            (1, 3, 1, 128), (1, 2, 2, 256)])
def test_batch_kernel_choices_agree(gpu, variant, prefetch, rounds, tile_w):
    probs = _mixed()
    steps = 30
    say(f"[gpu batch] kernel variant={variant} prefetch={prefetch} rounds={rounds} tile_w={tile_w}")
    b = gpu(probs).set_kernel(variant, prefetch, rounds, tile_w)
    b.step(steps)
    for i in (0, 4, 8):
        err = np.abs(b.save(i).cpu().numpy() - _oracle_f("mixed", i, steps)).max()
        say(f"    instance {i} max|df|={err:.3e}")
        assert err <= TOL
    b.close()


def _wide():
    """Instances wider than one 128- or 256-lane strip, with ragged strip tails."""
    return [P.random_vortex(n, 600 + i, nu, kmax=6, urms=0.03) for i, (n, nu) in enumerate(((300, 2e-3), (64, 1e-2),
                                                                                            (260, 5e-3)))]


@functools.lru_cache(maxsize=None)
def _oracle_wide(i, steps):
    from oracle.orc import Oracle
    o = Oracle(_wide()[i])
    o.step(steps)
    return o.f()


@pytest.mark.parametrize("tile_w,prefetch", [(128, 3), (256, 2)])
def test_batch_wide_strips(gpu, tile_w, prefetch):
    probs = _wide()
    steps = 20
    say(f"[gpu batch] wide instances sizes={[p.nx for p in probs]} tile_w={tile_w} prefetch={prefetch}")
    b = gpu(probs).set_kernel(1, prefetch, 1, tile_w)
    b.step(steps)
    for i in range(len(probs)):
        err = np.abs(b.save(i).cpu().numpy() - _oracle_wide(i, steps)).max()
        say(f"    instance {i} max|df|={err:.3e}")
        assert err <= TOL
    b.close()


def test_graph_replays_match_eager(gpu):
    """Replay the captured n-step graph several times, with eager work of the
    program in between, and check every replay against eager stepping."""
    import torch
    probs = _mixed(6)
    say("[gpu batch] graph replay vs eager, 4 replays of 5 steps (+1 odd replay)")
    eager = gpu(probs)
    graph = gpu(probs)
    for rep in range(4):
        eager.step(5)
        graph.step_graph(5)
        u, _, _ = graph.moments(0)            # eager work between replays
        _ = (u * 2.0).sum().item()
        torch.cuda.synchronize()
        for i in range(len(probs)):
            a = eager.save(i).cpu().numpy()
            g = graph.save(i).cpu().numpy()
            assert np.array_equal(a, g), (rep, i)
    eager.step(3)
    graph.step_graph(3)                        # odd length: starts from the other buffer next time
    graph.step_graph(3)
    eager.step(3)
    for i in range(len(probs)):
        assert np.array_equal(eager.save(i).cpu().numpy(), graph.save(i).cpu().numpy())
    assert graph.steps == eager.steps == 26
    eager.close()
    graph.close()


def test_autotune_restores_state_and_caches(gpu, tmp_path):
    probs = _mixed(6)
    say("[gpu batch] autotune")
    b = gpu(probs)
    b.step(4)
    before = [b.save(i).cpu().numpy() for i in range(len(probs))]
    cache = str(tmp_path / "tune.json")
    choice, cached = b.autotune(cache, steps=3)
    assert not cached and choice[0] in (1, 2) and choice[1] in (2, 3) and 1 <= choice[2] <= 3
    assert choice[3] in (64, 128, 256)
    assert b.steps == 4
    for i in range(len(probs)):
        assert np.array_equal(before[i], b.save(i).cpu().numpy())
    entry = json.load(open(cache))[b.signature()]
    assert tuple(entry["choice"]) == tuple(choice)
    choice2, cached2 = b.autotune(cache)
    assert cached2 and tuple(choice2) == tuple(choice)
    b.step(26)
    for i in (0, 3, 5):
        assert np.abs(b.save(i).cpu().numpy() - _oracle_f("mixed", i, 30)).max() <= TOL
    b.close()


def test_full_batch_config_sampled(gpu):
    """256 instances (sizes 64..512, nu log-uniform in [1e-3, 1e-1], k^-3 fields,
    seed 20230614) in the benchmark's launch configuration (the tuning cache's
    choice, graph replay); 8 sampled instances vs the oracle after 20 steps."""
    import os
    from oracle.orc import Oracle
    inst = P.batch_instances(256, seed=20230614)
    probs = [P.random_vortex(n, sd, nu) for n, nu, sd in inst]
    steps = 20
    say(f"[gpu batch] full config count=256 nodes={sum(p.nx * p.ny for p in probs)} steps={steps}")
    b = gpu(probs)
    tuning = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2306_08216_amd",
                          "tuning_mi355x.json")
    choice, cached = b.autotune(tuning, steps=5)
    say(f"    choice={choice} from_cache={cached}")
    b.step_graph(steps)
    sizes = np.array([p.nx for p in probs])
    picks = []
    for n in (64, 128, 256, 512):
        idx = np.nonzero(sizes == n)[0]
        picks += [int(idx[0]), int(idx[-1])]
    for i in picks:
        o = Oracle(probs[i], threads=8)
        o.step(steps)
        err = np.abs(b.save(i).cpu().numpy() - o.f()).max()
        say(f"    instance {i} n={probs[i].nx} nu={probs[i].nu:.3g} max|df|={err:.3e}")
        assert err <= TOL
    b.close()


def _tiny(nx, ny, seed, nu):
    rng = np.random.default_rng(seed)
    u, v, p = (a * rng.standard_normal((ny, nx)) for a in (0.01, 0.01, 1e-4))
    return P.Problem(nx=nx, ny=ny, lx=0.25 * nx, ly=0.25 * ny, nu=nu, u0=u, v0=v, p0=p, name=f"tiny_{nx}x{ny}")


DEGENERATE = {
    "single": lambda: [P.random_vortex(48, 900, 0.004, kmax=5, urms=0.03)],
    "smallest": lambda: [_tiny(5, 5, 41, 0.02), _tiny(5, 7, 42, 0.01), _tiny(7, 5, 43, 0.05),
                         _tiny(6, 6, 44, 0.02), _tiny(9, 5, 45, 0.03),
                         P.random_vortex(64, 46, 0.005, kmax=5, urms=0.03)],
}


@functools.lru_cache(maxsize=None)
def _degenerate_oracle(key, steps):
    from oracle.orc import Oracle
    out = []
    for p in DEGENERATE[key]():
        o = Oracle(p)
        o.step(steps)
        out.append(o.f())
    return out


@pytest.mark.parametrize("key", sorted(DEGENERATE))
@pytest.mark.parametrize("variant,prefetch,rounds,tile_w", [(1, 2, 1, 64), (1, 3, 2, 128), (1, 2, 1, 256), (2, 2, 1, 64)])
def test_batch_degenerate(gpu, key, variant, prefetch, rounds, tile_w):
    """A batch of one instance, and instances of the smallest size the boundary
    accepts (5 nodes on an axis) beside a larger one, each against its own
    oracle run."""
    probs = DEGENERATE[key]()
    steps = 40
    say(f"[gpu batch] {key} sizes={[(p.nx, p.ny) for p in probs]} steps={steps} "
        f"variant={variant} prefetch={prefetch} rounds={rounds} tile_w={tile_w}")
    want = _degenerate_oracle(key, steps)
    b = gpu(probs)
    b.set_kernel(variant, prefetch, rounds, tile_w)
    b.step(steps)
    b.synchronize()
    for i, p in enumerate(probs):
        f = b.save(i).cpu().numpy()
        err = np.abs(f - want[i]).max()
        say(f"    instance {i} {p.nx}x{p.ny} max|df|={err:.3e}")
        assert np.all(np.isfinite(f)) and err <= TOL
    b.close()


def test_batch_zero_steps_keep_the_initial_state(gpu):
    """Stepping a batch by zero leaves every instance at its initial equilibrium."""
    from oracle.orc import Oracle
    probs = DEGENERATE["smallest"]()
    say(f"[gpu batch] zero steps sizes={[(p.nx, p.ny) for p in probs]}")
    b = gpu(probs)
    b.step(0)
    b.synchronize()
    assert b.steps == 0
    for i, p in enumerate(probs):
        err = np.abs(b.save(i).cpu().numpy() - Oracle(p).f()).max()
        say(f"    instance {i} {p.nx}x{p.ny} max|df|={err:.3e}")
        assert err <= TOL
    b.close()


def test_batch_instance_derived_and_diagnostics(gpu):
    """Per-instance local quantities (Sec. 2.4) and diagnostics of a batch
    against each instance's oracle run (bounds propagated from the state
    tolerance through the division by nu + c_s^2 dt/2, as for single runs)."""
    from oracle.orc import Oracle
    probs = _mixed()
    steps = 30
    say(f"[gpu batch] derived and diagnostics, sizes={[p.nx for p in probs]} steps={steps}")
    b = gpu(probs)
    b.step(steps)
    for i in (0, 4, 8, 9):
        p = probs[i]
        o = Oracle(p)
        o.step(steps)
        do = o.derived()
        d = b.derived(i).cpu().numpy()
        theta = 0.2 * p.c ** 2 * o.dt
        base = 8 * TOL * p.c / (p.nu + theta)
        for k in range(14):
            bound = base * (2 if k == 4 else 1) * (2 * p.nu if k in (8, 9, 10) else 1) + 1e-13 * np.abs(do[k]).max()
            assert np.abs(d[k] - do[k]).max() <= bound, (i, k)
        sub = b.derived(i, (1 << 12) | (1 << 3)).cpu().numpy()
        assert np.abs(sub[0] - do[3]).max() <= base and np.abs(sub[1] - do[12]).max() <= base
        diag, status = b.diagnostics(i)
        dio = o.diagnostics()
        assert status == 0 and diag[6] == 0.0
        # sums over n nodes in different orders differ by up to n ulps
        sum_rel = p.nodes * 2.0 ** -52
        assert abs(diag[2] - dio[2]) <= 10 * TOL * np.sqrt(2 * dio[2] * dio[7]) + sum_rel * dio[2]
        assert abs(diag[4] - dio[4]) <= 10 * TOL and diag[7] == pytest.approx(dio[7], rel=sum_rel)
        assert abs(diag[5] - dio[5]) <= 10 * TOL * p.nx / p.lx
        say(f"    instance {i} n={p.nx}: derived and diagnostics agree")
    b.close()
