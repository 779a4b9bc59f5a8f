"""Seeded synthetic problem definitions: grids, parameters and initial fields.

This module describes inputs only -- the flow problems of Sec. 4 (and the
project's synthetic workloads) as parameter sets, initial velocity and
pressure fields and grid metric arrays.  It holds none of the method's
arithmetic, and both the HIP library and the CPU oracle consume exactly the
arrays it produces.

Conventions
-----------
* Fields are float64 arrays of shape (ny, nx), x fastest.
* Periodic axes place nodes at x_i = i L / N; wall axes place nodes on both
  walls, x_i = X(i/(N-1)), so the uniform wall spacing is L/(N-1).
* A mapped axis x = X(xi), xi in [0, 1], is described by the derivative scale
  inv_dx[i] = 1 / (X'(xi_i) * dxi) and by the smallest node spacing dx_min.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

PERIODIC = 0
WALL = 1


@dataclasses.dataclass
class Problem:
    """One MDF-FDLBM run: parameters plus initial fields (u0, v0, p0)."""

    nx: int
    ny: int
    lx: float
    ly: float
    nu: float                       # Newtonian nu, or consistency K if pl_n != 1
    u0: np.ndarray
    v0: np.ndarray
    p0: np.ndarray
    pl_n: float = 1.0
    nu_min: float = 0.0
    nu_max: float = 0.0
    cfl: float = 0.5
    c: float = 1.0
    eta: float = 0.8
    s_ratio: float = 1.5
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    lid_u: float = 0.0
    fx: float = 0.0
    fy: float = 0.0
    inv_dx_x: Optional[np.ndarray] = None
    inv_dx_y: Optional[np.ndarray] = None
    dx_min: float = 0.0
    force_x: Optional[np.ndarray] = None   # (ny, nx) force field added to fx (None: none)
    force_y: Optional[np.ndarray] = None   # (ny, nx) added to fy
    force_harmonic: bool = False           # F(x, t) = F(x) cos(force_omega t + force_phase) (else steady)
    force_omega: float = 0.0
    force_phase: float = 0.0
    metric: Optional[np.ndarray] = None    # (4, ny, nx): d i/dx, d i/dy, d j/dx, d j/dy (general mapping)
    node_xy: Optional[tuple] = None        # physical node positions (X, Y) of a general mapping
    mass_source: Optional[np.ndarray] = None  # (ny, nx) mass source R of eq. 2.1.1 (None: R = 0)
    track_rho0: bool = False               # oracle only: also advance the alpha = 0 equation
    name: str = ""

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def node_x(self) -> np.ndarray:
        return _axis_nodes(self.nx, self.lx, self.bc_x)

    def node_y(self) -> np.ndarray:
        return _axis_nodes(self.ny, self.ly, self.bc_y)


def _axis_nodes(n: int, length: float, bc: int) -> np.ndarray:
    if bc == WALL:
        return np.arange(n, dtype=np.float64) * (length / (n - 1))
    return np.arange(n, dtype=np.float64) * (length / n)


# ---------------------------------------------------------------------------
# analytic set-ups of Sec. 4 and the project's workloads
# ---------------------------------------------------------------------------

def taylor_green(n: int = 64, u0: float = 0.01, nu: float = 0.01, cfl: float = 0.5,
                 eta: float = 0.8, s_ratio: float = 1.5, length: float = 2.0 * math.pi) -> Problem:
    """Decaying Taylor-Green vortex on a periodic [0, L]^2 grid (the unforced
    sibling of the four-roll mill, Sec. 4.1):
    u = u0 sin x cos y, v = -u0 cos x sin y, P = (u0^2/4)(cos 2x + cos 2y)."""
    x = _axis_nodes(n, length, PERIODIC)
    X, Y = np.meshgrid(x, x, indexing="xy")
    k = 2.0 * math.pi / length
    u = u0 * np.sin(k * X) * np.cos(k * Y)
    v = -u0 * np.cos(k * X) * np.sin(k * Y)
    p = 0.25 * u0 * u0 * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    return Problem(nx=n, ny=n, lx=length, ly=length, nu=nu, u0=u, v0=v, p0=p, cfl=cfl,
                   eta=eta, s_ratio=s_ratio, name=f"taylor_green_{n}")


def taylor_green_exact(prob: Problem, t: float, u0: float, nu: float):
    """Analytic decaying Taylor-Green fields at time t (factor exp(-2 nu t))."""
    x, y = prob.node_x(), prob.node_y()
    X, Y = np.meshgrid(x, y, indexing="xy")
    k = 2.0 * math.pi / prob.lx
    dec = math.exp(-2.0 * nu * k * k * t)
    u = u0 * dec * np.sin(k * X) * np.cos(k * Y)
    v = -u0 * dec * np.cos(k * X) * np.sin(k * Y)
    p = 0.25 * u0 * u0 * dec * dec * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    return u, v, p


def four_roll_mill(n: int = 64, u0: float = 1e-4, nu: float = 0.01, cfl: float = 0.5, eta: float = 0.8,
                   s_ratio: float = 1.5, start: str = "exact", printed_sign: bool = False) -> Problem:
    """Four-roll mill (Sec. 4.1): periodic [0, 2pi]^2 driven by the steady force of
    eq. 4.1.1, whose steady solution is eq. 4.1.2, u = U0 sin x cos y,
    v = -U0 sin y cos x, with uniform pressure.  The viscous part of F_2 is
    taken as -2 nu U0 sin y cos x, the sign the Laplacian of v requires (the
    printed + sign, printed_sign=True, does not balance eq. 4.1.2).  start:
    "exact" (f_hat = f^eq of eq. 4.1.2) or "rest"."""
    L = 2.0 * math.pi
    x = _axis_nodes(n, L, PERIODIC)
    X, Y = np.meshgrid(x, x, indexing="xy")
    sgn = 1.0 if printed_sign else -1.0
    fx = u0 * u0 * np.sin(X) * np.cos(X) + 2.0 * nu * u0 * np.sin(X) * np.cos(Y)
    fy = u0 * u0 * np.sin(Y) * np.cos(Y) + sgn * 2.0 * nu * u0 * np.sin(Y) * np.cos(X)
    if start == "exact":
        u, v = u0 * np.sin(X) * np.cos(Y), -u0 * np.sin(Y) * np.cos(X)
    else:
        u, v = np.zeros((n, n)), np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=L, ly=L, nu=nu, u0=u, v0=v, p0=np.zeros((n, n)), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, force_x=fx, force_y=fy, name=f"four_roll_mill_{n}")


def four_roll_mill_exact(prob: Problem, u0: float = 1e-4):
    """Eq. 4.1.2 and eq. 4.1.3 at the nodes: dict of u, v, ux, uy, vx, vy, Sxx,
    Sxy, Syy, omega, Omega_xy."""
    X, Y = np.meshgrid(prob.node_x(), prob.node_y(), indexing="xy")
    c, ss = u0 * np.cos(X) * np.cos(Y), u0 * np.sin(X) * np.sin(Y)
    return {"u": u0 * np.sin(X) * np.cos(Y), "v": -u0 * np.sin(Y) * np.cos(X), "ux": c, "uy": -ss,
            "vx": ss, "vy": -c, "Sxx": c, "Sxy": 0.0 * c, "Syy": -c, "omega": 2.0 * ss, "Omega_xy": -ss}


def divergent_flow(n: int = 32, u0: float = 0.01, nu: float = 0.02, cfl: float = 0.5, eta: float = 0.8,
                   s_ratio: float = 1.5, start: str = "exact") -> Problem:
    """A steady flow with a mass source on the periodic [0, 2pi]^2: u = U0 sin x,
    v = U0 sin y has divergence R = U0 (cos x + cos y) (eq. 2.1.1), and with the
    uniform pressure it is a steady solution of eq. 2.1.2 under the force
        F_x = d(u u)/dx + d(u v)/dy - nu lap u = U0^2 (sin 2x + sin x cos y) + nu U0 sin x,
        F_y = d(v u)/dx + d(v v)/dy - nu lap v = U0^2 (sin 2y + sin y cos x) + nu U0 sin y.
    A manufactured case: the paper gives none with R != 0.  start: "exact" or "rest"."""
    L = 2.0 * math.pi
    x = _axis_nodes(n, L, PERIODIC)
    X, Y = np.meshgrid(x, x, indexing="xy")
    fx = u0 * u0 * (np.sin(2.0 * X) + np.sin(X) * np.cos(Y)) + nu * u0 * np.sin(X)
    fy = u0 * u0 * (np.sin(2.0 * Y) + np.sin(Y) * np.cos(X)) + nu * u0 * np.sin(Y)
    if start == "exact":
        u, v = u0 * np.sin(X), u0 * np.sin(Y)
    else:
        u, v = np.zeros((n, n)), np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=L, ly=L, nu=nu, u0=u, v0=v, p0=np.zeros((n, n)), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, force_x=fx, force_y=fy, mass_source=u0 * (np.cos(X) + np.cos(Y)),
                   name=f"divergent_flow_{n}")


def divergent_flow_exact(prob: Problem, u0: float = 0.01):
    """u, v, du/dx, dv/dy and the divergence of divergent_flow at the nodes."""
    X, Y = np.meshgrid(prob.node_x(), prob.node_y(), indexing="xy")
    return {"u": u0 * np.sin(X), "v": u0 * np.sin(Y), "ux": u0 * np.cos(X), "vy": u0 * np.cos(Y),
            "div": u0 * (np.cos(X) + np.cos(Y))}


def divergent_channel(n: int = 32, v0: float = 0.01, nu: float = 0.02, cfl: float = 0.5, eta: float = 0.8,
                      s_ratio: float = 1.5, start: str = "exact") -> Problem:
    """A channel on [0, 1]^2, periodic in x with walls at y = 0 and 1, fed by a
    mass source: u = 0, v = V0 sin(pi y) vanishes on both walls and has
    divergence R = pi V0 cos(pi y) (eq. 2.1.1); with uniform pressure it is a
    steady solution of eq. 2.1.2 under F_x = 0 and
        F_y = d(v v)/dy - nu d2v/dy2 = pi V0^2 sin(2 pi y) + nu pi^2 V0 sin(pi y).
    A manufactured case with walls.  start: "exact" or "rest"."""
    x = _axis_nodes(n, 1.0, PERIODIC)
    y = _axis_nodes(n, 1.0, WALL)
    X, Y = np.meshgrid(x, y, indexing="xy")
    fy = math.pi * v0 * v0 * np.sin(2.0 * math.pi * Y) + nu * math.pi ** 2 * v0 * np.sin(math.pi * Y)
    z = np.zeros((n, n))
    v = v0 * np.sin(math.pi * Y) if start == "exact" else z.copy()
    return Problem(nx=n, ny=n, lx=1.0, ly=1.0, nu=nu, u0=z, v0=v, p0=z.copy(), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, bc_x=PERIODIC, bc_y=WALL, force_x=z.copy(), force_y=fy,
                   mass_source=math.pi * v0 * np.cos(math.pi * Y), name=f"divergent_channel_{n}")


def divergent_channel_exact(prob: Problem, v0: float = 0.01):
    """u, v of divergent_channel at the nodes."""
    X, Y = np.meshgrid(prob.node_x(), prob.node_y(), indexing="xy")
    return {"u": 0.0 * X, "v": v0 * np.sin(math.pi * Y)}


def swept_vortex(n: int = 32, u0: float = 0.01, nu: float = 0.01, f0: float = 1e-3, omega: float = 0.2,
                 phase: float = 0.0, cfl: float = 0.5, eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    """Taylor-Green vortex (Sec. 4.1 setup) on the periodic [0, 2pi]^2 swept by a
    spatially uniform stream that an oscillating force F = (f0 cos(omega t +
    phase), 0) drives from rest.  By Galilean invariance the solution is the
    decaying vortex carried by the stream (swept_vortex_exact)."""
    prob = taylor_green(n, u0=u0, nu=nu, cfl=cfl, eta=eta, s_ratio=s_ratio)
    prob.fx = f0
    prob.force_harmonic, prob.force_omega, prob.force_phase = True, omega, phase
    prob.name = f"swept_vortex_{n}"
    return prob


def swept_vortex_exact(prob: Problem, t: float, u0: float = 0.01, f0: float = 1e-3):
    """u, v, P of swept_vortex at time t: the stream U(t) = (f0/omega)(sin(omega t
    + phase) - sin phase), its displacement X(t) = integral of U, and the
    vortex u0 e^{-2 nu t} (sin(x - X) cos y, -cos(x - X) sin y) with pressure
    (u0^2 e^{-4 nu t}/4)(cos 2(x - X) + cos 2y)."""
    w, ph = prob.force_omega, prob.force_phase
    U = f0 / w * (math.sin(w * t + ph) - math.sin(ph))
    Xs = f0 / w * ((math.cos(ph) - math.cos(w * t + ph)) / w - t * math.sin(ph))
    X, Y = np.meshgrid(prob.node_x(), prob.node_y(), indexing="xy")
    d = u0 * math.exp(-2.0 * prob.nu * t)
    u = U + d * np.sin(X - Xs) * np.cos(Y)
    v = -d * np.cos(X - Xs) * np.sin(Y)
    p = 0.25 * d * d * (np.cos(2.0 * (X - Xs)) + np.cos(2.0 * Y))
    return {"u": u, "v": v, "p": p, "U": U}


def pulsed_vortex(n: int = 32, a0: float = 0.0, nu: float = 0.01, f0: float = 1e-3, omega: float = 0.2,
                  cfl: float = 0.5, eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    """Cellular flow on the periodic [0, 2pi]^2 driven by the force field
    F(x, t) = f0 cos(omega t) (sin x cos y, -cos x sin y): the velocity stays in
    that mode, u = a(t) (sin x cos y, -cos x sin y), with a' = -2 nu a + f0 cos(omega t)
    (its advection is a pressure gradient), started at amplitude a0."""
    L = 2.0 * math.pi
    x = _axis_nodes(n, L, PERIODIC)
    X, Y = np.meshgrid(x, x, indexing="xy")
    sx, sy = np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y)
    p = 0.25 * a0 * a0 * (np.cos(2.0 * X) + np.cos(2.0 * Y))
    return Problem(nx=n, ny=n, lx=L, ly=L, nu=nu, u0=a0 * sx, v0=a0 * sy, p0=p, cfl=cfl, eta=eta,
                   s_ratio=s_ratio, force_x=f0 * sx, force_y=f0 * sy, force_harmonic=True, force_omega=omega,
                   name=f"pulsed_vortex_{n}")


def pulsed_vortex_amplitude(prob: Problem, t: float, a0: float = 0.0, f0: float = 1e-3) -> float:
    """a(t) of pulsed_vortex: the solution of a' + 2 nu a = f0 cos(omega t), a(0) = a0."""
    k, w = 2.0 * prob.nu, prob.force_omega
    den = k * k + w * w
    return f0 * (k * math.cos(w * t) + w * math.sin(w * t)) / den + (a0 - f0 * k / den) * math.exp(-k * t)


def mapping_metric(x_i, x_j, y_i, y_j):
    """Inverse Jacobian of a mapping of the node indices, (X, Y)(i, j), from its
    derivatives with respect to the indices: returns the planes d i/dx, d i/dy,
    d j/dx, d j/dy and the smallest spacing between neighbouring index lines,
    min(1/|grad i|, 1/|grad j|), the dx_min of the time step."""
    det = x_i * y_j - x_j * y_i
    ix, iy, jx, jy = y_j / det, -x_j / det, -y_i / det, x_i / det
    met = np.stack([ix, iy, jx, jy])
    dxm = float(min((1.0 / np.hypot(ix, iy)).min(), (1.0 / np.hypot(jx, jy)).min()))
    return met, dxm


def warped_taylor_green(n: int = 32, u0: float = 0.01, nu: float = 0.01, shear: int = 1, eps: float = 0.2,
                        cfl: float = 0.5, eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    """Decaying Taylor-Green vortex on a non-orthogonal, non-separable periodic
    grid: node (i, j) sits at x = xi + shear eta + eps sin(eta), y = eta + eps sin(xi)
    with xi = 2 pi i/n, eta = 2 pi j/n.  With an integer shear the map carries the
    index torus onto the [0, 2 pi]^2 torus, so the physical Taylor-Green vortex
    (taylor_green_exact at the node positions) stays the exact solution."""
    L = 2.0 * math.pi
    d = L / n
    xi, et = np.meshgrid(np.arange(n) * d, np.arange(n) * d, indexing="xy")
    X = xi + shear * et + eps * np.sin(et)
    Y = et + eps * np.sin(xi)
    met, dxm = mapping_metric(np.ones_like(xi) * d, (shear + eps * np.cos(et)) * d, eps * np.cos(xi) * d,
                              np.ones_like(xi) * d)
    u = u0 * np.sin(X) * np.cos(Y)
    v = -u0 * np.cos(X) * np.sin(Y)
    p = 0.25 * u0 * u0 * (np.cos(2 * X) + np.cos(2 * Y))
    return Problem(nx=n, ny=n, lx=L, ly=L, nu=nu, u0=u, v0=v, p0=p, cfl=cfl, eta=eta, s_ratio=s_ratio,
                   metric=met, dx_min=dxm, node_xy=(X, Y), name=f"warped_taylor_green_{n}")


def sheared_channel(n: int = 32, nu: float = 0.01, force: float = 1e-4, shear: float = 0.5, cfl: float = 0.5,
                    eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    """Force-driven channel (Sec. 4.3) between walls at y = 0 and y = 1, periodic
    in x with period 1, on a grid whose index lines j = const are the horizontal
    lines y = j/(n-1) and whose lines i = const are slanted: x = i/n + shear y.
    The walls are index lines; the steady solution is the Poiseuille profile."""
    ii, jj = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="xy")
    dx, dy = 1.0 / n, 1.0 / (n - 1)
    Y = jj * dy
    X = ii * dx + shear * Y
    one = np.ones((n, n))
    met, dxm = mapping_metric(one * dx, one * shear * dy, 0.0 * one, one * dy)
    z = np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=1.0, ly=1.0, nu=nu, u0=z, v0=z.copy(), p0=z.copy(), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, bc_x=PERIODIC, bc_y=WALL, fx=force, metric=met, dx_min=dxm, node_xy=(X, Y),
                   name=f"sheared_channel_{n}")


def trapezoidal_cavity(n: int = 64, re: float = 100.0, lid: float = 0.1, taper: float = 0.4, cfl: float = 0.5,
                       eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    """Lid-driven cavity on a trapezoid (the keyword geometry of the paper): the
    bottom wall spans x in [0, 1] at y = 0, the lid spans [taper/2, 1 - taper/2]
    at y = 1, and the side walls are straight; node (i, j) sits at
    y = j/(n-1), x = 1/2 + (i/(n-1) - 1/2)(1 - taper y).  nu = lid/Re (unit
    height)."""
    s = np.arange(n, dtype=np.float64) / (n - 1)
    S, T = np.meshgrid(s, s, indexing="xy")
    h = 1.0 / (n - 1)
    Y = T
    X = 0.5 + (S - 0.5) * (1.0 - taper * T)
    met, dxm = mapping_metric((1.0 - taper * T) * h, -taper * (S - 0.5) * h, 0.0 * S, np.ones_like(S) * h)
    z = np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=1.0, ly=1.0, nu=lid / re, u0=z, v0=z.copy(), p0=z.copy(), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, bc_x=WALL, bc_y=WALL, lid_u=lid, metric=met, dx_min=dxm, node_xy=(X, Y),
                   name=f"trapezoidal_cavity_{n}")


def periodic_flow(nx: int = 32, ny: Optional[int] = None, u0: float = 0.1, nu: float = 0.01, cfl: float = 0.5,
                  eta: float = 0.8, s_ratio: float = 1.5, inv_dx_x: Optional[np.ndarray] = None,
                  x_nodes: Optional[np.ndarray] = None, dx_min: float = 0.0) -> Problem:
    """Steady periodic flow (Sec. 4.2) on [0, 1]^2 with the force of eq. 4.2.1,
    F_x = 8 pi^2 nu u0 sin 2pi x sin 2pi y, F_y = 8 pi^2 nu u0 cos 2pi x cos 2pi y,
    started from its steady solution eq. 4.2.2 (f_hat = f^eq).  ny != nx gives
    the rectangular-cell grid (e.g. 64 x 32); inv_dx_x with its node
    positions x_nodes maps the x axis."""
    ny = nx if ny is None else ny
    x = _axis_nodes(nx, 1.0, PERIODIC) if x_nodes is None else np.asarray(x_nodes, dtype=np.float64)
    y = _axis_nodes(ny, 1.0, PERIODIC)
    X, Y = np.meshgrid(x, y, indexing="xy")
    k = 2.0 * math.pi
    amp = 8.0 * math.pi ** 2 * nu * u0
    fx = amp * np.sin(k * X) * np.sin(k * Y)
    fy = amp * np.cos(k * X) * np.cos(k * Y)
    u = u0 * np.sin(k * X) * np.sin(k * Y)
    v = u0 * np.cos(k * X) * np.cos(k * Y)
    p = 0.25 * u0 * u0 * (np.cos(2 * k * X) - np.cos(2 * k * Y))
    return Problem(nx=nx, ny=ny, lx=1.0, ly=1.0, nu=nu, u0=u, v0=v, p0=p, cfl=cfl, eta=eta, s_ratio=s_ratio,
                   force_x=fx, force_y=fy, inv_dx_x=inv_dx_x, dx_min=dx_min, name=f"periodic_flow_{nx}x{ny}")


def periodic_flow_exact(x: np.ndarray, y: np.ndarray, u0: float = 0.1):
    """Eq. 4.2.2 at nodes x (columns) and y (rows): u, v, p."""
    X, Y = np.meshgrid(x, y, indexing="xy")
    k = 2.0 * math.pi
    return (u0 * np.sin(k * X) * np.sin(k * Y), u0 * np.cos(k * X) * np.cos(k * Y),
            0.25 * u0 * u0 * (np.cos(2 * k * X) - np.cos(2 * k * Y)))


def cavity(n: int = 1024, re: float = 1000.0, lid: float = 0.1, cfl: float = 0.5, eta: float = 0.8,
           s_ratio: float = 1.5, length: float = 1.0) -> Problem:
    """Lid-driven square cavity (Sec. 4.4): fluid at rest, u = 0 and p = 0,
    top wall moving at `lid`, nu = L lid / Re, walls on all four sides."""
    z = np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=length, ly=length, nu=length * lid / re, u0=z, v0=z.copy(), p0=z.copy(),
                   cfl=cfl, eta=eta, s_ratio=s_ratio, bc_x=WALL, bc_y=WALL, lid_u=lid,
                   name=f"cavity_{n}_re{re:g}")


def poiseuille(n: int = 32, nu: float = 0.01, force: float = 1e-6, cfl: float = 0.5, eta: float = 0.8,
               s_ratio: float = 1.5, pl_n: float = 1.0, nu_min: float = 0.0, nu_max: float = 0.0,
               inv_dx_y: Optional[np.ndarray] = None, dx_min: float = 0.0) -> Problem:
    """Force-driven channel (Sec. 4.3): [0,1]^2, periodic in x, walls at
    y = 0 and y = 1, fluid at rest initially."""
    z = np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=1.0, ly=1.0, nu=nu, u0=z, v0=z.copy(), p0=z.copy(), cfl=cfl, eta=eta,
                   s_ratio=s_ratio, bc_x=PERIODIC, bc_y=WALL, fx=force, pl_n=pl_n, nu_min=nu_min,
                   nu_max=nu_max, inv_dx_y=inv_dx_y, dx_min=dx_min, name=f"poiseuille_{n}")


def poiseuille_exact(y: np.ndarray, nu: float, force: float, height: float = 1.0) -> np.ndarray:
    """Newtonian channel profile (eq. 4.3.1): u = F H^2/(2 nu) [y/H - (y/H)^2]."""
    return force * height * height / (2.0 * nu) * (y / height - (y / height) ** 2)


def powerlaw_poiseuille_exact(y: np.ndarray, pl_n: float, K: float, force: float, height: float = 1.0):
    """Steady power-law channel profile for nu = K gdot^(n-1):
    u(y) = n/(n+1) (F/K)^(1/n) [(H/2)^(1+1/n) - |y - H/2|^(1+1/n)]."""
    e = 1.0 + 1.0 / pl_n
    return pl_n / (pl_n + 1.0) * (force / K) ** (1.0 / pl_n) * ((height / 2) ** e - np.abs(y - height / 2) ** e)


def tanh_mapping(n: int, beta: float = 1.5, length: float = 1.0):
    """Wall-clustering map X(xi) = L/2 [1 + tanh(beta (2 xi - 1)) / tanh(beta)]
    on nodes xi_i = i/(n-1).  Returns (node positions, inv_dx, dx_min)."""
    xi = np.arange(n, dtype=np.float64) / (n - 1)
    tb = math.tanh(beta)
    pos = 0.5 * length * (1.0 + np.tanh(beta * (2.0 * xi - 1.0)) / tb)
    dX = length * beta / tb / np.cosh(beta * (2.0 * xi - 1.0)) ** 2   # X'(xi)
    inv_dx = 1.0 / (dX * (1.0 / (n - 1)))
    dx_min = float(np.min(np.diff(pos)))
    return pos, inv_dx, dx_min


def sine_mapping(n: int, amp: float = 0.2, length: float = 2.0 * math.pi):
    """Smooth periodic map X(xi) = xi + amp sin(xi) on xi_i = i L/n (amp < 1).
    Returns (node positions, inv_dx, dx_min)."""
    xi = np.arange(n, dtype=np.float64) * (length / n)
    k = 2.0 * math.pi / length
    pos = xi + amp * np.sin(k * xi) / k
    dX = 1.0 + amp * np.cos(k * xi)
    inv_dx = 1.0 / (dX * (length / n))
    d = np.diff(np.concatenate([pos, [pos[0] + length]]))
    return pos, inv_dx, float(np.min(d))


def powerlaw_cavity(n: int = 2048, pl_n: float = 0.5, beta: float = 1.5, lid: float = 0.1,
                    re: float = 100.0, cfl: float = 0.5, eta: float = 0.8, s_ratio: float = 1.5,
                    ceiling: Optional[float] = None) -> Problem:
    """Power-law lid-driven cavity on a tanh-stretched grid (both axes).
    Re = U^(2-n) L^n / K with L = 1; viscosity clamp [1e-2, ceiling] nu_ref
    with nu_ref = U L / Re.  The ceiling defaults to 100 for a shear-thinning
    fluid (n < 1) and to 4 for a shear-thickening one (n > 1): there the
    viscosity peaks at the singular lid corners, and ceilings of 10 nu_ref and
    more let the corner non-equilibrium parts grow without bound (the run
    diverges at 1024^2 and 2048^2; 100 nu_ref at every size from 64^2)."""
    K = lid ** (2.0 - pl_n) / re
    nu_ref = lid / re
    if ceiling is None:
        ceiling = 100.0 if pl_n <= 1.0 else 4.0
    _, g, dxm = tanh_mapping(n, beta)
    z = np.zeros((n, n))
    return Problem(nx=n, ny=n, lx=1.0, ly=1.0, nu=K, u0=z, v0=z.copy(), p0=z.copy(), pl_n=pl_n,
                   nu_min=1e-2 * nu_ref, nu_max=ceiling * nu_ref, cfl=cfl, eta=eta, s_ratio=s_ratio,
                   bc_x=WALL, bc_y=WALL, lid_u=lid, inv_dx_x=g.copy(), inv_dx_y=g.copy(), dx_min=dxm,
                   name=f"powerlaw_cavity_{n}_n{pl_n:g}")


def random_vortex_fields(n: int, seed: int, kmin: int = 1, kmax: int = 8, urms: float = 0.02,
                         length: float = 2.0 * math.pi):
    """Random-phase periodic velocity field with streamfunction modes
    kmin <= |k| <= kmax, |psi_hat(k)| ~ |k|^-3 (energy spectrum ~ k^-3), scaled
    to the given rms speed.  Fields are direct mode sums evaluated on the node
    positions, so every n samples the same continuous field; the pressure
    solves the Poisson equation lap P = -div(u . grad u) spectrally on the
    mode set (host-side set-up of a consistent initial pressure)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = []
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if ky == 0 and kx <= 0:
                continue
            kk = math.hypot(kx, ky)
            if kk < kmin or kk > kmax:
                continue
            modes.append((kx, ky, kk))
    phases = rng.uniform(0.0, 2.0 * math.pi, size=len(modes))
    k0 = 2.0 * math.pi / length
    # psi = sum amp cos(k0 (kx x + ky y) + ph): u = d psi/dy, v = -d psi/dx, i.e.
    # u = Im sum (-amp k0 ky e^{i ph}) e^{i k0 (kx x + ky y)}.  At the periodic
    # nodes x_i = i L / n that sum is an inverse DFT (all |k| < n/2), so it is
    # evaluated exactly (to rounding) with one inverse FFT per component.
    if 2 * kmax >= n:
        raise ValueError("random_vortex_fields needs n > 2*kmax")
    cu = np.zeros((n, n), dtype=complex)
    cv = np.zeros((n, n), dtype=complex)
    for (kx, ky, kk), ph in zip(modes, phases):
        amp = kk ** -3.0
        e = np.exp(1j * ph) * n * n
        cu[ky % n, kx % n] += -amp * k0 * ky * e
        cv[ky % n, kx % n] += amp * k0 * kx * e
    u = np.ascontiguousarray(np.imag(np.fft.ifft2(cu)))
    v = np.ascontiguousarray(np.imag(np.fft.ifft2(cv)))
    scale = urms / math.sqrt(np.mean(u * u + v * v))
    u *= scale
    v *= scale
    # pressure: lap P = -d_i d_j (u_i u_j), solved with an FFT on the grid
    kvec = np.fft.fftfreq(n, d=1.0 / n) * k0
    KX, KY = np.meshgrid(kvec, kvec, indexing="xy")
    k2 = KX * KX + KY * KY
    k2[0, 0] = 1.0
    uu, uv, vv = np.fft.fft2(u * u), np.fft.fft2(u * v), np.fft.fft2(v * v)
    rhs = -(-(KX * KX) * uu - 2.0 * KX * KY * uv - (KY * KY) * vv)
    ph = rhs / (-k2)
    ph[0, 0] = 0.0
    p = np.real(np.fft.ifft2(ph))
    return u, v, p


def random_vortex(n: int, seed: int, nu: float, kmin: int = 1, kmax: int = 8, urms: float = 0.02,
                  cfl: float = 0.5, eta: float = 0.8, s_ratio: float = 1.5) -> Problem:
    u, v, p = random_vortex_fields(n, seed, kmin, kmax, urms)
    L = 2.0 * math.pi
    return Problem(nx=n, ny=n, lx=L, ly=L, nu=nu, u0=u, v0=v, p0=p, cfl=cfl, eta=eta, s_ratio=s_ratio,
                   name=f"random_vortex_{n}_s{seed}")


def batch_instances(count: int = 256, seed: int = 20230614, sizes: Sequence[int] = (64, 128, 256, 512),
                    log_nu: tuple = (-3.0, -1.0), kmax: int = 8, urms: float = 0.02,
                    field_seed_base: int = 100000):
    """Batched workload: `count` periodic decaying-vortex instances with grid
    sizes uniform over `sizes` and nu log-uniform in 10^log_nu, drawn from a
    PCG64 stream with the given seed.  Returns a list of (n, nu, field_seed);
    fields come from random_vortex(n, field_seed, nu)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.choice(np.asarray(sizes), size=count)
    nus = 10.0 ** rng.uniform(log_nu[0], log_nu[1], size=count)
    return [(int(ns[i]), float(nus[i]), field_seed_base + i) for i in range(count)]


def gre(phi: np.ndarray, exact: np.ndarray) -> float:
    """Global relative error of eq. 4.0: sum |phi - phi*| / sum |phi*|."""
    return float(np.sum(np.abs(phi - exact)) / np.sum(np.abs(exact)))
