"""Pin of the oracle's SSP-RK3 Faraday update (Scheme H step H6).

With the ions frozen (uniform density 1, no flux, no electron pressure) the
field update is the Hall term alone, E = J x Bbar.  A circularly polarised
mode along the mean field is then an exact solution of the semi-discrete
equations: with the one-cell differences of the staggered grid, J at a node
is parallel to the averaged perturbation there, so J x Bbar = Bmean J x b and
the mode only turns, at the frequency

    omega = Bmean k_h^2,   k_h = (2 / dx) sin(k dx / 2),

the whistler of immobile ions.  For this linear rotation every 3-stage,
third-order Runge-Kutta method multiplies the mode by the degree-3 Taylor
polynomial of exp(i omega h) per (sub)step h.  The tests hold the oracle to

  * that polynomial, to round-off, along each axis of the grid (the x, y and
    z parts of the curl and of the node average all take part), and
  * third order: the error against the exact rotation falls 8x per halving
    of dt;

and show that two plausible mistakes (the 3/4, 1/4 weights of the second
stage swapped, or a plain Euler step) fail them.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

NX = {1: (32, 1, 1), 2: (4, 32, 1), 3: (4, 4, 32)}


def frozen_box(dim, dt, n_sub=1):
    nx, ny, nz = NX[dim]
    return W.params(dim=dim, nx=nx, ny=ny, nz=nz, dx=0.5, dt=dt, xbc="periodic", inject=False,
                    ppc=1, n_modes=0, beta_e=0.0, beta_i=0.0, u_sh=0.0, eta=0.0, j_ext=0.0,
                    n_sub=n_sub, theta_deg=0.0, precision=64)


def mode_field(p, axis, m, amp, phase):
    """Mean field 1 along `axis`, circularly polarised mode of wavenumber
    index m along it: (b_1, b_2) = amp (cos, sin)(k s + phase) for the two
    axes following `axis` cyclically, at cell centres."""
    nx, ny, nz = (p["nx"], p["ny"] if p["dim"] >= 2 else 1, p["nz"] if p["dim"] >= 3 else 1)
    n = (nx, ny, nz)[axis]
    k = 2 * np.pi * m / (n * p["dx"])
    B = np.zeros((nz, ny, nx, 3))
    idx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")[::-1]   # x, y, z
    s = (idx[axis] + 0.5) * p["dx"]
    a1, a2 = (axis + 1) % 3, (axis + 2) % 3
    B[..., axis] = 1.0
    B[..., a1] = amp * np.cos(k * s + phase)
    B[..., a2] = amp * np.sin(k * s + phase)
    return B.reshape(-1, 3), k, s.reshape(-1), (a1, a2)


def run_frozen(p, axis, m, amp, nsteps):
    """Oracle field-only steps from the mode; returns B and the mode data."""
    o = O.Oracle(p)
    nc = p["nx"] * (p["ny"] if p["dim"] >= 2 else 1) * (p["nz"] if p["dim"] >= 3 else 1)
    # one ion at rest at the centre of every cell: density exactly 1 at every
    # node (each node collects one full partition of unity), no flux
    cells = np.array([(i, j, k) for k in range(p["nz"] if p["dim"] >= 3 else 1)
                      for j in range(p["ny"] if p["dim"] >= 2 else 1) for i in range(p["nx"])], dtype=np.int64)
    off = np.full((nc, 3), 0.5)
    off[:, p["dim"]:] = 0.0
    o.set_particles(0, cells, off, np.zeros((nc, 3)), np.arange(nc, dtype=np.uint64))
    B, k, s, comps = mode_field(p, axis, m, amp, 0.3)
    o.set_B(B)
    o.step(O.DEPOSIT)
    o.compute_E()
    n, g = o.fluid()
    assert np.all(n == 1.0) and np.all(g == 0.0)
    for _ in range(nsteps):
        o.step(O.FIELD)
    return o.B(), k, s, comps


def taylor3(z):
    return 1 + z + z * z / 2 + z * z * z / 6


def expected(k, s, dx, amp, t_steps, h, comps, B, rk=True):
    kh = 2.0 / dx * np.sin(k * dx / 2)
    omega = kh * kh
    y0 = amp * np.exp(1j * (k * s + 0.3))
    if rk:
        y = y0 * taylor3(1j * omega * h) ** t_steps
    else:
        y = y0 * np.exp(1j * omega * h * t_steps)
    out = np.zeros_like(B)
    out[:, comps[0]] = y.real
    out[:, comps[1]] = y.imag
    return out


@pytest.mark.parametrize("dim,axis", [(1, 0), (2, 1), (3, 2)])
@pytest.mark.parametrize("n_sub", [1, 2])
def test_rk3_is_the_third_order_taylor_polynomial(dim, axis, n_sub):
    dt, steps, amp, m = 0.1, 12, 0.3, 4
    p = frozen_box(dim, dt, n_sub)
    B, k, s, comps = run_frozen(p, axis, m, amp, steps)
    ref = expected(k, s, p["dx"], amp, steps * n_sub, dt / n_sub, comps, B)
    assert np.max(np.abs(B[:, comps[0]] - ref[:, comps[0]])) < 1e-13
    assert np.max(np.abs(B[:, comps[1]] - ref[:, comps[1]])) < 1e-13
    assert np.all(B[:, axis] == 1.0)
    # the exact rotation is measurably different: the bound above has teeth
    ex = expected(k, s, p["dx"], amp, steps * n_sub, dt / n_sub, comps, B, rk=False)
    assert np.max(np.abs(ex - ref)) > 1e-7


def convergence_ratios(dim=1, axis=0):
    T, amp, m = 1.6, 0.3, 4
    errs = []
    for dt in (0.1, 0.05, 0.025, 0.0125):
        p = frozen_box(dim, dt)
        steps = int(round(T / dt))
        B, k, s, comps = run_frozen(p, axis, m, amp, steps)
        ex = expected(k, s, p["dx"], amp, steps, dt, comps, B, rk=False)
        errs.append(np.max(np.abs(B[:, comps] - ex[:, comps])))
    errs = np.array(errs)
    return errs, errs[:-1] / errs[1:]


def test_rk3_converges_at_third_order():
    errs, ratios = convergence_ratios()
    assert np.all(errs > 1e-12), errs                # well above round-off
    assert np.all((ratios > 7.0) & (ratios < 9.0)), ratios


SWAPPED = ("fsoracle.c", "B2[q] = 0.75 * B0[q] + 0.25 * (B1[q] + h * F[q]);",
           "B2[q] = 0.25 * B0[q] + 0.75 * (B1[q] + h * F[q]);")
EULER = ("fsoracle.c", "s->B[q] = (1.0 / 3.0) * B0[q] + (2.0 / 3.0) * (B2[q] + h * F[q]);",
         "s->B[q] = B1[q];")


@pytest.mark.parametrize("mistake", [SWAPPED, EULER], ids=["swapped-stage-weights", "euler"])
def test_planted_rk_mistakes_fail_the_pins(mistake):
    with O.variant([mistake]):
        p = frozen_box(1, 0.1)
        B, k, s, comps = run_frozen(p, 0, 4, 0.3, 12)
        ref = expected(k, s, p["dx"], 0.3, 12, 0.1, comps, B)
        assert np.max(np.abs(B[:, comps] - ref[:, comps])) > 1e-6
        _, ratios = convergence_ratios()
        assert not np.all((ratios > 7.0) & (ratios < 9.0)), ratios
