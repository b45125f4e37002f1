"""Pin of the time-centred ion-field coupling (reading R16 of the oracle).

The paper's runs use dHybridR (Sec. 2), whose ion-field coupling is second
order in time; the reading R16 deposits the density at x^{n+1} and the flux
at the midpoint of each move with v^{n+1/2}, advances B with the moments
frozen at t_{n+1/2} and extrapolates the flux to t_{n+1} for E^{n+1}.

What pins it is the order of accuracy: at fixed grid and particles the
scheme is a time discretisation of one semi-discrete system, so runs with
dt, dt/2, dt/4, dt/8 must approach a dt/64 reference run as dt^2 (error
ratio ~4 per halving), where the first-order coupling R4 goes as dt (ratio
~2).  Periodic 1D boxes with two finite-amplitude seeded modes, cold and
warm ions, warm electrons, oblique B0, the continuous deposit (the
fixed-point deposit's quantisation would floor the errors), and a leapfrog
start from the same t = 0 state for every dt (velocities taken back half a
step with a Boris step of -dt/2).  Three planted mistakes, each a plausible
slip of the scheme, fall back to first order.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

NX = 64


def run(coupling, dt, beta_i, T=1.0):
    p = W.params(dim=1, nx=NX, dx=0.5, dt=dt, ppc=64, xbc="periodic", inject=False, beta_i=beta_i, beta_e=1.0,
                 u_sh=0.0, theta_deg=30.0, n_modes=2, mode_amp=0.1, seed=11, precision=64, coupling=coupling,
                 wall_th="open")
    o = O.Oracle(p, "continuous")
    o.init()
    o.leapfrog_start()
    for _ in range(int(round(T / dt))):
        o.step()
    pt = o.particles(0)
    k = np.argsort(pt["id"])
    return o.B(), pt["cell"][k, 0] + pt["off"][k, 0]


def convergence(coupling, beta_i, dts=(0.02, 0.01, 0.005, 0.0025)):
    Bref, xref = run(coupling, dts[0] / 64, beta_i)
    e = []
    for dt in dts:
        B, x = run(coupling, dt, beta_i)
        d = x - xref
        d -= NX * np.round(d / NX)
        e.append((np.max(np.abs(B - Bref)), np.max(np.abs(d))))
    e = np.array(e)
    return e, e[:-1] / e[1:]


@pytest.mark.parametrize("beta_i", [0.0, 1.0], ids=["cold", "warm"])
def test_time_centred_coupling_is_second_order(beta_i):
    e2, r2 = convergence(2, beta_i)
    e1, r1 = convergence(1, beta_i)
    print(f"beta_i {beta_i}: R16 B ratios {r2[:, 0]}, x ratios {r2[:, 1]}; R4 B ratios {r1[:, 0]}")
    assert np.all(r2[:, 0] > 3.3) and r2[-1, 0] < 6.0, r2
    assert np.all(r2[:, 1] > 3.3) and np.all(r2[:, 1] < 6.0), r2
    assert np.all((r1[:, 0] > 1.7) & (r1[:, 0] < 2.5)), r1
    # and more accurate at every dt of the sweep
    assert np.all(e2[:, 0] * 5 < e1[:, 0]), (e2, e1)


MIDPOINT_AT_END = ("fsoracle.c", "double hdtdx = 0.5 * dtdx;", "double hdtdx = dtdx;")
NO_EXTRAPOLATION = ("fsoracle.c", "s->fg[q] = 1.5 * gh - 0.5 * s->fg_prev[q];", "s->fg[q] = gh;")
DENSITY_NOT_CENTRED = ("fsoracle.c",
                       "for (int64_t q = 0; q < nn; ++q) s->fn[q] = 0.5 * (s->fn_prev[q] + fn1[q]);", "")


@pytest.mark.parametrize("mistake", [MIDPOINT_AT_END, NO_EXTRAPOLATION, DENSITY_NOT_CENTRED],
                         ids=["flux-at-new-position", "no-extrapolation", "density-not-centred"])
def test_planted_coupling_mistakes_lose_second_order(mistake):
    with O.variant([mistake]):
        _, r = convergence(2, 1.0)
    assert r[-1, 0] < 2.6, r
