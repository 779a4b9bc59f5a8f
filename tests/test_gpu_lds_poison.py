"""Race check of the LDS exchanges (GPU): the checking build libmdf_poison.so
sets every LDS slot to NaN before a kernel publishes in it, so a read of a
slot that no thread wrote for the current row or tile puts a NaN into the
state.  The parity cases below (both fused variants at every tile width,
walls on both axes, the power law, the tiled step on general mappings,
the batch and the diagnostics) must still match the oracle to 1e-12.

The checking build runs in a child process (the environment variable
MDF_LIBRARY selects it), so that this process keeps the released library."""
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
POISON = os.path.join(ROOT, "paper_2306_08216_amd", "libmdf_poison.so")
TOL = 1e-12


def worker():
    sys.path.insert(0, ROOT)
    from oracle.orc import Oracle
    from paper_2306_08216_amd import problems as P
    from paper_2306_08216_amd import _lib as L
    from paper_2306_08216_amd.batch import BatchSolver
    from paper_2306_08216_amd.solver import Solver

    assert os.path.samefile(os.environ["MDF_LIBRARY"], POISON)
    L.lib()

    def pl(n, idx):
        return P.powerlaw_cavity(n, pl_n=idx)

    cases = [
        ("cavity72 variant 1, 64 lanes", P.cavity(72, re=100.0), 120, (1, 64, 0, 2)),
        ("cavity72 variant 1, 128 lanes, prefetch 3", P.cavity(72, re=100.0), 120, (1, 128, 0, 3)),
        ("cavity300 variant 1, 256 lanes", P.cavity(300, re=100.0), 60, (1, 256, 0, 2)),
        ("cavity72 variant 2", P.cavity(72, re=100.0), 120, (2, 0, 0, 0)),
        ("taylor-green 70 variant 2", P.taylor_green(70), 120, (2, 0, 0, 0)),
        ("power law n = 0.5, 64 lanes", pl(48, 0.5), 80, (1, 64, 0, 2)),
        ("power law n = 1.5, 256 lanes", pl(300, 1.5), 30, (1, 256, 0, 2)),
        ("four-roll mill (force field)", P.four_roll_mill(40), 100, (1, 64, 0, 2)),
        ("cavity40 tiled step", P.cavity(40, re=100.0), 100, (0, 0, 0, 0)),
        ("warped Taylor-Green tiled step", P.warped_taylor_green(40, shear=1, eps=0.2), 100, (0, 0, 0, 0)),
        ("trapezoid tiled step", P.trapezoidal_cavity(48), 100, (0, 0, 0, 0)),
        ("divergent channel (mass source)", P.divergent_channel(40), 100, (0, 0, 0, 0)),
    ]
    bad = 0
    for name, prob, steps, (variant, tw, sh, pf) in cases:
        s = Solver(prob)
        s.set_kernel(variant, tw, sh, pf)
        s.step(steps)
        f = s.save().cpu().numpy()
        diag, status = s.diagnostics()
        s.close()
        o = Oracle(prob)
        o.step(steps)
        err = np.abs(f - o.f()).max()
        dio = o.diagnostics()
        derr = abs(diag[2] - dio[2]) / max(dio[2], 1e-300)
        ok = np.isfinite(f).all() and err <= TOL and status == 0 and derr <= 1e-9
        bad += 0 if ok else 1
        print(f"[lds poison] {name}: max|df| = {err:.3e}, KE rel {derr:.1e}, status {status} "
              f"{'ok' if ok else 'FAILED'}", flush=True)
    probs = [P.random_vortex(n, sd, nu) for n, sd, nu in ((64, 1, 1e-2), (96, 2, 3e-3), (128, 3, 1e-3))]
    b = BatchSolver(probs)
    b.step(40)
    for i, prob in enumerate(probs):
        o = Oracle(prob)
        o.step(40)
        err = np.abs(b.save(i).cpu().numpy() - o.f()).max()
        ok = err <= TOL
        bad += 0 if ok else 1
        print(f"[lds poison] batch instance {i} ({prob.nx}^2): max|df| = {err:.3e} {'ok' if ok else 'FAILED'}",
              flush=True)
    b.close()
    sys.exit(1 if bad else 0)


@pytest.mark.gpu
def test_lds_exchanges_read_only_published_slots():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(POISON), "the checking build is missing: run __graft_entry__.build()"
    env = dict(os.environ, MDF_LIBRARY=POISON)
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--worker"], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


if __name__ == "__main__" and "--worker" in sys.argv:
    worker()
