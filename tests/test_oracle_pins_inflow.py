"""Pins of the oracle's injection and box boundaries (Sec. 2: continuous
injection at the far-upstream boundary, cosmic rays injected at the faux
shock; readings R8-R10 of the oracle).

The thermal inflow, the boundary fill of the moments and the inflow node are
pinned by a cold beam (ions and electrons at zero temperature): the uniform
flowing plasma with the motional field E = -u x B0 is an exact steady state
of the continuum equations, so after a full transit of the box the oracle
must hold it at every node.  The cosmic-ray injection is pinned by the
density its flux sets up in the box: with no fields the injected CRs stream
upstream in straight lines, and the steady density they leave in the box
follows from the flux and the speed distribution alone.  Deriving it from an
isotropic population of speed w in the downstream frame (drifting at u2 away
from the wall): crossers into the box have direction cosines mu' > a = u2/w
with weight (w mu' - u2), i.e. a pdf proportional to (mu' - a), and the
density of a flux F of such particles is 2F / (w - u2); the paper's CR
density n_cr at the shock (Table 1: n_cr / n_g = 0.01) thus needs
F = n_cr (w - u2) / 2.  At time T a point at distance X from the wall still
misses the particles slower than X / T, a fraction X / ((w - u2) T) of the
density.

Each test is paired with planted mistakes (built from a patched copy of the
oracle) that it must catch.
"""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W


# --------------------------------------------------------------------------
# cold beam: thermal inflow, moment boundary fill, inflow node
# --------------------------------------------------------------------------
def cold_beam(beta_e=0.0):
    return W.params(dim=1, nx=64, dx=0.5, dt=0.005, u_sh=20.0, beta_i=0.0, beta_e=beta_e,
                    theta_deg=45.0, wall_th="open", n_cr=0.0, ppc=256, n_modes=0, precision=64, seed=5)


def run_beam(p, steps=400):
    # 400 steps: t = 2, 1.25 transits of the 32 d_i box at 20 v_A
    o = O.Oracle(p)
    o.init()
    for _ in range(steps):
        o.step()
    return o


def check_cold_beam(o, p):
    th = math.radians(p["theta_deg"])
    B0 = np.array([math.cos(th), math.sin(th), 0.0])
    motional = -np.cross([p["u_sh"], 0.0, 0.0], B0)
    n, g = o.fluid()
    inner = n[1:-1]                                  # nodes every particle side covers
    assert abs(inner.mean() - 1.0) < 2e-3, inner.mean()
    assert np.max(np.abs(inner - 1.0)) < 0.03, np.max(np.abs(inner - 1.0))
    np.testing.assert_allclose(o.E(), np.broadcast_to(motional, o.E().shape), rtol=0, atol=1e-12)
    np.testing.assert_allclose(o.B(), np.broadcast_to(B0, o.B().shape), rtol=0, atol=1e-12)
    v = o.particles(0)["v"]
    np.testing.assert_allclose(v, np.broadcast_to([p["u_sh"], 0, 0], v.shape), rtol=0, atol=1e-12)


def test_cold_beam_stays_uniform_after_a_transit():
    p = cold_beam()
    o = run_beam(p)
    check_cold_beam(o, p)
    # the end nodes are covered by particles on one side only: the raw
    # moments there hold half the density; Ohm's law sees the filled value
    n, _ = o.fluid()
    assert 0.4 < n[0] < 0.6 and 0.4 < n[-1] < 0.6


def check_boundary_fill(o):
    # warm electrons turn any density step into E_x = -grad p_e / n.  With
    # the boundary fill the end nodes take the density of their covered
    # neighbours and E_x stays at the noise level everywhere; without it the
    # half-covered end nodes make a pressure step of (1 - 0.5^(5/3)) / 2
    Ex = o.E()[:, 0]
    assert np.max(np.abs(Ex)) < 0.05, np.max(np.abs(Ex))


def test_cold_ions_warm_electrons_no_field_at_the_ends():
    o = run_beam(cold_beam(beta_e=1.0))
    check_boundary_fill(o)


def injected_positions_thermal(p, steps=3):
    o = O.Oracle(p)
    for _ in range(steps):
        o.step(O.INJECT)
    pt = o.particles(0)
    x = (pt["cell"][:, 0] + pt["off"][:, 0]) * p["dx"]
    return x, pt["v"]


def test_thermal_injection_distribution():
    # a particle that crossed x = 0 at a uniformly distributed time within
    # the step has travelled v_x U dt; velocities are the drifting Maxwellian
    p = W.params(dim=1, nx=64, dx=0.5, dt=0.005, u_sh=20.0, beta_i=1.0, ppc=2048, precision=64, seed=8)
    x, v = injected_positions_thermal(p)
    sig = math.sqrt(p["beta_i"] / 2)
    assert len(x) > 1000
    assert stats.kstest(x / (v[:, 0] * p["dt"]), "uniform").pvalue > 1e-3
    for comp, mean in ((0, p["u_sh"]), (1, 0.0), (2, 0.0)):
        assert stats.kstest((v[:, comp] - mean) / sig, "norm").pvalue > 1e-3


# planted mistakes of the thermal inflow and the boundary fill
FLUX_X2 = ("fsoracle.c", "double F = (double)c->ppc * c->u_sh * c->dt / c->dx;",
           "double F = 2.0 * (double)c->ppc * c->u_sh * c->dt / c->dx;")
AT_ZERO = ("fsoracle.c", "double xi = v[0] * U[0] * s->c.dt / s->c.dx;",
           "double xi = 0.0 * U[0];")
NO_FILL = ("fsoracle.c", "if (i < s->mclamp) i = s->mclamp;\n        if (i > s->c.nx - s->mclamp) i = s->c.nx - s->mclamp;",
           "")


def test_planted_inflow_flux_fails_the_cold_beam():
    with O.variant([FLUX_X2]):
        p = cold_beam()
        o = run_beam(p)
        with pytest.raises(AssertionError):
            check_cold_beam(o, p)


def test_planted_injection_at_the_boundary_fails_the_distribution():
    with O.variant([AT_ZERO]):
        p = W.params(dim=1, nx=64, dx=0.5, dt=0.005, u_sh=20.0, beta_i=1.0, ppc=2048, precision=64, seed=8)
        x, v = injected_positions_thermal(p)
        assert stats.kstest(x / (v[:, 0] * p["dt"]), "uniform").pvalue < 1e-6


def test_planted_missing_fill_fails_the_warm_electron_beam():
    with O.variant([NO_FILL]):
        o = run_beam(cold_beam(beta_e=1.0))
        with pytest.raises(AssertionError):
            check_boundary_fill(o)


# --------------------------------------------------------------------------
# inflow node (reading R10) through the flux budget
# --------------------------------------------------------------------------
def inflow_flux_budget(steps=15):
    """Largest deviation of the per-step change of the total tangential flux
    from dt u_sh B0_y per row, in a perturbed warm box with a conducting
    wall.  The curl telescopes, so only the end nodes' tangential E enter:
    zero at the conductor, the motional field at the inflow node."""
    p = W.params(dim=1, nx=64, dx=0.5, ppc=16, theta_deg=60.0, u_sh=20.0, wall_th="specular",
                 wall_field=1, seed=77, n_modes=3, mode_amp=0.05, precision=64)
    o = O.Oracle(p)
    o.init()
    want = p["dt"] * p["u_sh"] * math.sin(math.radians(p["theta_deg"]))
    worst = 0.0
    for _ in range(steps):
        b0 = o.B().sum(axis=0) * p["dx"]
        o.step()
        b1 = o.B().sum(axis=0) * p["dx"]
        worst = max(worst, abs((b1[1] - b0[1]) - want), abs(b1[2] - b0[2]))
    return worst


def test_inflow_node_carries_the_motional_field():
    assert inflow_flux_budget() < 1e-11


OHM_AT_INFLOW = ("fsoracle.c", "if (s->c.xbc != ORA_XBC_PERIODIC && i == 0) {", "if (0) {")


def test_planted_ohm_at_the_inflow_node_fails_the_flux_budget():
    with O.variant([OHM_AT_INFLOW]):
        assert inflow_flux_budget() > 1e-6


# --------------------------------------------------------------------------
# cosmic-ray injection at the wall
# --------------------------------------------------------------------------
def cr_box(**kw):
    base = dict(dim=1, nx=32, dx=0.5, dt=0.005, u_sh=20.0, r=4.0, beta_i=0.0, beta_e=0.0, theta_deg=0.0,
                wall_th="open", wall_cr="faux_shock", n_cr=0.01, ppc=0, ppc_cr=256, n_modes=0, precision=64,
                seed=9, alpha_cr=1.5)
    base.update(kw)
    return W.params(**base)


def cr_density_ratio(p, steps=1200, first=800, every=5):
    """Time-averaged CR density in the box (whole-cell bins) over the
    prediction n_cr (1 - X / ((w - u2) T)), with no fields (B0 along x and
    B = 0 make the motional field vanish, and the field update is skipped)."""
    o = O.Oracle(p)
    o.init()
    nx, dx = p["nx"], p["dx"]
    o.set_B(np.zeros((nx, 3)))
    o.compute_E()
    assert np.all(o.E() == 0.0)
    L, u2, w = nx * dx, p["u_sh"] / p["r"], p["cr_w"]
    Xc = L - (np.arange(nx) + 0.5) * dx
    cnt, pred = np.zeros(nx), np.zeros(nx)
    for s in range(steps):
        o.step(O.PUSH | O.BOUNDARY | O.INJECT)
        if s >= first and s % every == 0:
            pt = o.particles(1)
            cnt += np.bincount(pt["cell"][:, 0], minlength=nx)[:nx]
            pred += p["ppc_cr"] * (1.0 - Xc / ((w - u2) * (s + 1) * p["dt"]))
    ratio = cnt.sum() / pred.sum()
    # the macro weight alpha_cr n_cr / ppc_cr turns the count into the density
    o.step(O.DEPOSIT)
    o.compute_E()
    n, _ = o.fluid()
    T = steps * p["dt"]
    Xn = L - np.arange(nx + 1) * dx
    nrat = n[2:-2].sum() / (p["alpha_cr"] * p["n_cr"] * (1.0 - Xn[2:-2] / ((w - u2) * T))).sum()
    return ratio, nrat


def test_cr_injection_sets_the_paper_cr_density():
    ratio, nrat = cr_density_ratio(cr_box())
    assert abs(ratio - 1.0) < 0.02, ratio          # 80 snapshots of 8e3 ions: noise ~0.3%
    assert abs(nrat - 1.0) < 0.05, nrat            # one snapshot: noise ~1.3%


def injected_crs(p, steps=2):
    o = O.Oracle(p)
    for _ in range(steps):
        o.step(O.INJECT)
    pt = o.particles(1)
    x = (pt["cell"][:, 0] + pt["off"][:, 0]) * p["dx"]
    return x, pt["v"]


def test_cr_injection_distribution():
    p = cr_box(ppc_cr=4096)
    x, v = injected_crs(p)
    u2, w = p["u_sh"] / p["r"], p["cr_w"]
    a = u2 / w
    assert len(x) > 3000
    wd = v - np.array([u2, 0.0, 0.0])                # downstream frame
    np.testing.assert_allclose(np.linalg.norm(wd, axis=1), w, rtol=1e-13)
    mu = -wd[:, 0] / w                               # direction cosine into the box
    assert np.all(mu > a)
    assert stats.kstest(mu, lambda m: ((m - a) / (1 - a)) ** 2).pvalue > 1e-3
    assert stats.kstest(np.arctan2(wd[:, 2], wd[:, 1]), "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-3
    L = p["nx"] * p["dx"]
    assert stats.kstest((L - x) / (np.abs(v[:, 0]) * p["dt"]), "uniform").pvalue > 1e-3


CR_FLUX_X2 = ("fsoracle.c", "double Fc = (double)c->ppc_cr * (c->cr_w - u2) * c->dt / (2.0 * c->dx);",
              "double Fc = (double)c->ppc_cr * (c->cr_w - u2) * c->dt / c->dx;")
CR_FLUX_SUM = ("fsoracle.c", "double Fc = (double)c->ppc_cr * (c->cr_w - u2) * c->dt / (2.0 * c->dx);",
               "double Fc = (double)c->ppc_cr * (c->cr_w + u2) * c->dt / (2.0 * c->dx);")
CR_MU_UNIFORM = ("fsoracle.c", "double mu = a + (1.0 - a) * sqrt(U[2]);\n                double stt",
                 "double mu = a + (1.0 - a) * U[2];\n                double stt")


@pytest.mark.parametrize("mistake", [CR_FLUX_X2, CR_FLUX_SUM, CR_MU_UNIFORM],
                         ids=["flux-x2", "w-plus-u2", "uniform-mu"])
def test_planted_cr_injection_mistakes_fail(mistake):
    with O.variant([mistake]):
        ratio, _ = cr_density_ratio(cr_box())
        caught = abs(ratio - 1.0) >= 0.02
        if mistake is CR_MU_UNIFORM:
            p = cr_box(ppc_cr=4096)
            x, v = injected_crs(p)
            a = p["u_sh"] / p["r"] / p["cr_w"]
            mu = (p["u_sh"] / p["r"] - v[:, 0]) / p["cr_w"]
            caught = caught or stats.kstest(mu, lambda m: ((m - a) / (1 - a)) ** 2).pvalue < 1e-6
        assert caught, ratio
