"""Pin of the oracle's walls, corners and moving lid against the vortex
centres of the lid-driven cavity (Sec. 4.4, Table 4, MDF-FDLBM rows): Re = 400
on 128 x 128 nodes, lid speed 0.1, c = 1, CFL 0.5, from rest (no GPU).

The run takes 50 000 steps (t = 197, about 20 lid transits; the primary
centre then moves by less than 2e-4 per 2500 steps) on the OpenMP build of
the oracle, whose results equal the sequential build's."""
import json
import os

import numpy as np
import pytest

from paper_2306_08216_amd import problems as P

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def stream_function(u, y):
    """psi(x, y) = integral of u dy from the bottom wall (trapezoid rule), so
    that u = d psi/dy; the clockwise primary vortex is its minimum."""
    psi = np.zeros_like(u)
    psi[1:] = np.cumsum(0.5 * (u[1:] + u[:-1]) * np.diff(y)[:, None], axis=0)
    return psi


def extremum(psi, x, y, mask, sign):
    """Centre of the extremum of sign * psi inside mask, refined by a parabola
    through the three nodes around it along each axis."""
    ps = np.where(mask, sign * psi, -np.inf)
    j, i = np.unravel_index(np.argmax(ps), ps.shape)

    def vertex(fm, f0, fp):
        d = fm - 2.0 * f0 + fp
        return 0.0 if d == 0.0 else 0.5 * (fm - fp) / d

    return (x[i] + vertex(psi[j, i - 1], psi[j, i], psi[j, i + 1]) * (x[1] - x[0]),
            y[j] + vertex(psi[j - 1, i], psi[j, i], psi[j + 1, i]) * (y[1] - y[0]))


@pytest.mark.slow
def test_cavity_re400_vortex_centres(orc):
    n = 128
    prob = P.cavity(n, re=400.0, lid=0.1)
    o = orc.Oracle(prob, threads=max(1, min(8, os.cpu_count() or 1)))
    o.step(50000)
    u, _, _ = o.moments()
    x, y = prob.node_x(), prob.node_y()
    psi = stream_function(u, y)
    X, Y = np.meshgrid(x, y, indexing="xy")
    inner = (X > 0) & (X < 1) & (Y > 0) & (Y < 1)
    tab = GOLDEN["cavity_vortex_centres_table4"]["Re=400"]
    found = {
        "primary": extremum(psi, x, y, inner, -1.0),
        "lower_left": extremum(psi, x, y, inner & (X < 0.3) & (Y < 0.3), 1.0),
        "lower_right": extremum(psi, x, y, inner & (X > 0.7) & (Y < 0.3), 1.0),
    }
    dx = 1.0 / (n - 1)
    for name, (cx, cy) in found.items():
        tx, ty = tab[name]
        assert abs(cx - tx) < dx and abs(cy - ty) < dx, (name, (cx, cy), (tx, ty))
    # the primary vortex turns clockwise under a lid moving in +x
    assert psi.min() < 0.0
