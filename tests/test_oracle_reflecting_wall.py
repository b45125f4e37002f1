"""Pins of the reflecting-wall (RW) variant in the oracle.

The paper benchmarks the faux shock against RW runs (Sec. 3, Table 1 Runs C
and 3D): in the downstream frame a super-Alfvenic flow meets a mirror at
rest, and the shock that forms runs back upstream.  Here the thermal ions
take the SPECULAR wall policy at x = L (the rw1 workload).  Pinned by what
geometry and the shock jump conditions fix, not by the oracle's formulas:
  * a mirror keeps every ion, keeps its speed, and puts it at the mirror
    image of where the straight path would have ended;
  * every ion that meets the mirror comes back, so the ion count changes
    only by injection and by escape at the inflow boundary;
  * the shock obeys conservation of mass across it, n2 v_s = n1 (u0 + v_s)
    with v_s its speed away from the mirror; flux freezing of the
    tangential field, B_y2 / B_y1 = n2 / n1, the ideal-MHD jump of a
    perpendicular shock (at theta_Bn = 80 deg and a shock-frame Alfven Mach
    number of ~30 the oblique correction is below 1e-3); and the
    strong-shock compression of a gas with two degrees of freedom,
    r = (gamma + 1) / (gamma - 1) = 3 for gamma = 2: in 1D with B nearly
    along y the ions are heated only in their gyration plane (x, z), and
    they carry nearly all the downstream pressure (the electron pressure of
    reading R12 stays O(1) against the ~n1 u0^2 ~ 400 ram pressure).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W
from tests.shock import by_of, ion_x, shock_state


def test_specular_wall_mirrors_each_crosser():
    p = W.preset("rw1", precision=64)
    rng = np.random.default_rng(8)
    n = 20000
    v = rng.normal(0.0, 10.0, (n, 3))
    v[:, 0] = np.abs(v[:, 0]) + 1e-3                       # moving into the mirror
    dtdx = p["dt"] / p["dx"]
    delta = v[:, 0] * dtdx * rng.random(n)                 # overshoot past x = L this step, in cells
    out, vnew, xi = O.wall_list(p, 5, 0, np.arange(n, dtype=np.uint64), delta, v.copy())
    assert out.all()
    assert np.array_equal(vnew[:, 0], -v[:, 0]) and np.array_equal(vnew[:, 1:], v[:, 1:])
    assert np.array_equal(np.linalg.norm(vnew, axis=1), np.linalg.norm(v, axis=1))
    # mirror image of x = L + delta about x = L
    assert np.array_equal(xi, p["nx"] - delta)
    assert np.all(xi <= p["nx"]) and np.all(xi > p["nx"] - v[:, 0] * dtdx)


def test_reflecting_wall_run_keeps_every_ion():
    p = W.preset("rw1", precision=64, nx=128)
    o = O.Oracle(p)
    o.init()
    n_prev = o.count(0)
    hits = 0
    for _ in range(400):
        st = o.step()
        assert st["transmitted"] == 0 and st["open_removed"] == 0
        assert st["incident"] == st["reflected"]
        n = o.count(0)
        assert n == n_prev + st["injected_th"] - st["escaped"]
        n_prev = n
        hits += st["incident"]
    assert hits > 0


@pytest.fixture(scope="module")
def rw1_run():
    """The rw1 box in the oracle to t = 12 / Omega_ci, measured at t = 4 and 12."""
    p = W.preset("rw1", precision=64)
    o = O.Oracle(p)
    o.init()
    out = {}
    for s in range(1, 2401):
        o.step()
        if s in (800, 2400):
            out[s * p["dt"]] = shock_state(ion_x(o.particles(0)), by_of(o.B()), p)
    return p, out


def test_reflecting_wall_shock_conserves_mass_across_it(rw1_run):
    p, m = rw1_run
    (t1, (d1, _, _)), (t2, (d2, n2, _)) = sorted(m.items())
    vs = (d2 - d1) / (t2 - t1)
    u0 = p["u_sh"]
    assert vs > 0
    assert abs(n2 * vs / (u0 + vs) - 1.0) < 0.12, (vs, n2)


def test_reflecting_wall_shock_freezes_the_tangential_field(rw1_run):
    p, m = rw1_run
    _, n2, by2 = m[max(m)]
    by1 = np.sin(np.deg2rad(p["theta_deg"]))
    assert abs(by2 / by1 / n2 - 1.0) < 0.04, (n2, by2 / by1)


def test_reflecting_wall_shock_compression_is_the_two_dof_strong_shock(rw1_run):
    p, m = rw1_run
    (t1, (d1, _, _)), (t2, (d2, n2, _)) = sorted(m.items())
    vs = (d2 - d1) / (t2 - t1)
    r_speed = 1.0 + p["u_sh"] / vs                     # from n2 v_s = n1 (u0 + v_s)
    assert 2.6 < n2 < 3.5, n2
    assert 2.6 < r_speed < 3.5, r_speed
