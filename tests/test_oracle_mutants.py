"""The oracle's pins catch plausible mistakes (no GPU).

Each case plants one mistake in a copy of the oracle's source -- a dropped
factor, a wrong neighbour, a one-sided difference -- builds that copy on the
CPU, and checks that the pin named for it fails on the copy while it passes on
the oracle itself.  The oracle's own files are never modified."""
import importlib.util
import os
import shutil

import pytest

from oracle import build as orc_build

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.dirname(orc_build.__file__)


def _module(name):
    spec = importlib.util.spec_from_file_location(f"_pins_{name}", os.path.join(HERE, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# (case, text in mdf_oracle.c, replacement, pin module, pin test)
CASES = [
    ("kinetic energy without its 1/2",
     "ke += 0.5 * (u[i] * u[i] + v[i] * v[i]) * dA;", "ke += (u[i] * u[i] + v[i] * v[i]) * dA;",
     "test_oracle_diagnostics", "test_taylor_green_initial_diagnostics"),
    ("enstrophy without its 1/2",
     "ens += 0.5 * om * om * dA;", "ens += om * om * dA;",
     "test_oracle_diagnostics", "test_taylor_green_energy_and_enstrophy_decay"),
    ("node area dA = 1",
     "double dA = 1.0 / (st->gx[x] * st->gy[y]);", "double dA = 1.0;",
     "test_oracle_diagnostics", "test_taylor_green_initial_diagnostics"),
    ("area sum counts nodes",
     "area += dA;", "area += 1.0;",
     "test_oracle_diagnostics", "test_mapped_grid_area_and_energy"),
    ("one-sided divergence",
     "(u[(size_t)y * nx + xp] - u[(size_t)y * nx + xm]) * st->gx[x] / 2.0",
     "(u[(size_t)y * nx + xp] - u[(size_t)y * nx + x]) * st->gx[x]",
     "test_oracle_diagnostics", "test_taylor_green_initial_diagnostics"),
    ("central difference without the 1/2",
     "(u[(size_t)y * nx + xp] - u[(size_t)y * nx + xm]) * st->gx[x] / 2.0",
     "(u[(size_t)y * nx + xp] - u[(size_t)y * nx + xm]) * st->gx[x]",
     "test_oracle_diagnostics", "test_divergence_of_a_compressive_field"),
    ("shear stress without the factor 2 of eq. 2.4.4",
     "2.0 * nu * Sxx, 2.0 * nu * Sxy, 2.0 * nu * Syy,", "nu * Sxx, nu * Sxy, nu * Syy,",
     "test_oracle_diagnostics", "test_stress_and_rotation_of_poiseuille_flow"),
    ("rotation tensor of eq. 2.4.5 transposed",
     "0.5 * (G[0][1] - G[1][0]),", "0.5 * (G[1][0] - G[0][1]),",
     "test_oracle_diagnostics", "test_stress_and_rotation_of_poiseuille_flow"),
    ("velocity gradient of eq. 2.4.1 with the wrong sign",
     "G[a][0] = -(s / st->cs2) * mx;", "G[a][0] = (s / st->cs2) * mx;",
     "test_oracle_flows", "test_taylor_green_decay_64"),
    ("corner extrapolated from its x neighbour",
     "size_t i1 = (size_t)(y + iy) * nx + (x + ix);", "size_t i1 = (size_t)(y + (corner ? 0 : iy)) * nx + (x + ix);",
     "test_oracle_diagnostics", "test_wall_nodes_carry_the_wall_velocity_and_neighbour_pressure"),
    ("lid speed on the top corners",
     "y == ny - 1 && !corner) ? p->lid_u : 0.0;", "y == ny - 1) ? p->lid_u : 0.0;",
     "test_oracle_diagnostics", "test_wall_nodes_carry_the_wall_velocity_and_neighbour_pressure"),
    ("lid on the bottom wall",
     "y == ny - 1 && !corner) ? p->lid_u : 0.0;", "y == 0 && !corner) ? p->lid_u : 0.0;",
     "test_oracle_flows", "test_cavity_sanity_and_lid"),
    ("zeroth-order non-equilibrium extrapolation at walls",
     "out[k] = few[k] + 2.0 * (ph1[k] - fe1[k]) - (ph2[k] - fe2[k]);", "out[k] = few[k] + (ph1[k] - fe1[k]);",
     "test_oracle_flows", "test_poiseuille_against_closed_form_and_table2"),
    ("half step without the force",
     "+ st->h * WJ[j] * Fa[a][i] * m;", ";",
     "test_oracle_flows", "test_half_step_carries_the_force"),
    ("full step with h instead of dt on the force",
     "+ st->dt * WJ[j] * Fa[a][i] * m", "+ st->h * WJ[j] * Fa[a][i] * m",
     "test_oracle_forced", "test_four_roll_mill_steady_solution"),
    ("full step without the (dt^2/2) d_t F term of eq. 2.3.24",
     "+ 0.5 * st->dt * st->dt * WJ[j] * Fa[a][i] * dm;", ";",
     "test_oracle_forced", "test_harmonic_force_mean_momentum"),
    ("d_t F with the wrong sign",
     "const double dm = harmonic ? -st->p.force_omega", "const double dm = harmonic ? st->p.force_omega",
     "test_oracle_forced", "test_harmonic_force_mean_momentum"),
    ("force taken one step late",
     "const double tn = (double)st->steps * st->dt;", "const double tn = (double)(st->steps + 1) * st->dt;",
     "test_oracle_forced", "test_harmonic_force_mean_momentum"),
    ("mapped transport upwinded by the sign of c_j instead of its contravariant component",
     "r += U * mixed_unit(st, pl, x, y, 0, U > 0.0 ? 1 : -1);",
     "r += U * mixed_unit(st, pl, x, y, 0, (CX[j] + CY[j]) > 0.0 ? 1 : -1);",
     "test_oracle_mapping", "test_warped_taylor_green_decay"),
    ("contravariant component U built from d j/dx instead of d i/dy",
     "double U = c * (CX[j] * st->met[i] + CY[j] * st->met[n + i]);",
     "double U = c * (CX[j] * st->met[i] + CY[j] * st->met[2 * n + i]);",
     "test_oracle_mapping", "test_warped_taylor_green_decay"),
    ("mapped node area without the cross terms of the Jacobian",
     "dA = 1.0 / fabs(det);", "dA = 1.0 / fabs(st->met[i] * st->met[3 * n + i]);",
     "test_oracle_mapping", "test_warped_taylor_green_decay"),
    ("mapped divergence without the cross derivatives",
     "div = st->met[i] * ui + st->met[2 * n + i] * uj + st->met[n + i] * vi + st->met[3 * n + i] * vj;",
     "div = st->met[i] * ui + st->met[3 * n + i] * vj;",
     "test_oracle_mapping", "test_divergence_of_a_mapped_field"),
    ("half step with the force not modulated in time",
     "+ st->h * WJ[j] * Fa[a][i] * m;", "+ st->h * WJ[j] * Fa[a][i];",
     "test_oracle_forced", "test_pulsed_vortex_amplitude"),
    ("force field of the x equation read for both",
     "st->Fy[i] = p->fy + (p->force_y ? p->force_y[i] : 0.0);",
     "st->Fy[i] = p->fy + (p->force_x ? p->force_x[i] : 0.0);",
     "test_oracle_forced", "test_four_roll_mill_steady_solution"),
    ("pressure of eq. 2.3.23 without the mass source term",
     "r[k] = Ptry - 0.5 * (T + st->p.nu * R - (u * u + v * v));", "r[k] = Ptry - 0.5 * (T - (u * u + v * v));",
     "test_oracle_source", "test_divergent_flow_converges_to_its_closed_form"),
    ("f_hat taken with the kappa of f_bar in the pressure solve",
     "return form == FORM_HAT ? 0.5 * st->dt :", "return form == FORM_HAT ? 0.5 * st->h :",
     "test_oracle_source", "test_form_pressure_inverts_the_stored_forms"),
    ("alpha = 0 equation without its source in Step (4)",
     "+ st->dt * WJ[q] * source_at(st, i);", ";",
     "test_oracle_source", "test_rho0_equation_stays_uniform"),
    ("source G of eq. 2.2.7 without its 1/c_s^2",
     "*g = WJ[j] * st->c * (CX[j] * d1[0] + CY[j] * d1[1]) / st->cs2;",
     "*g = WJ[j] * st->c * (CX[j] * d1[0] + CY[j] * d1[1]);",
     "test_oracle_source", "test_flux_source_moments_on_a_uniform_flow"),
    ("wall rule taking the neighbour pressures without the mass source",
     "node_state(st, ph1, form, source_at(st, i1), &u1, &v1, &P1);",
     "node_state(st, ph1, form, 0.0, &u1, &v1, &P1);",
     "test_oracle_source", "test_divergent_channel_with_walls"),
]


_PIN_HOLDS = set()


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


@pytest.mark.parametrize("case,old,new,module,pin", CASES, ids=[c[0] for c in CASES])
def test_pin_catches_planted_mistake(orc, mutant_dir, case, old, new, module, pin):
    src = open(os.path.join(ORACLE_DIR, "mdf_oracle.c")).read()
    assert src.count(old) >= 1, f"the text to mutate is gone from the oracle: {old!r}"
    work = mutant_dir / f"m{CASES.index(next(c for c in CASES if c[0] == case))}"
    work.mkdir()
    for f in ("mdf_oracle.h", "cnn_oracle.c", "cnn_oracle.h"):
        shutil.copy(os.path.join(ORACLE_DIR, f), work / f)
    (work / "mdf_oracle.c").write_text(src.replace(old, new))
    lib_path = orc_build.compile_lib(str(work / "libmutant.so"), orc_build.sources(str(work)), openmp=True)
    test = getattr(_module(module), pin)
    if (module, pin) not in _PIN_HOLDS:
        test(orc)                              # the pin holds on the oracle itself (once per pin)
        _PIN_HOLDS.add((module, pin))
    with orc.using_library(lib_path):
        with pytest.raises(AssertionError):
            test(orc)                          # and fails on the planted mistake
