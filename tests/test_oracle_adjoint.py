"""Pins of the oracle's reverse-mode derivative (fsoracle_adj.c) against
central finite differences of the forward oracle.

The derivative is that of the continuous-deposit step with every discrete
decision (cell, wall reflection, removal, injection count, density floor)
held fixed along the forward trajectory.  A finite difference is a valid
check only if no decision flips between the +h and -h runs; every
whole-gradient test asserts that the per-step event counts of the two runs
are identical, and that the events the test is about (wall reflections)
actually happened.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

RNG = np.random.default_rng(20250714)


def fd_grad(p, nsteps, amps, k, rel_h=1e-6):
    """Central difference of the loss in parameter k (0 u_sh, 1 alpha_cr,
    2+m amplitude m) with h = rel_h * max(|theta|, 1e-3)."""
    a = np.array(amps, dtype=np.float64)
    base = p["u_sh"] if k == 0 else (p["alpha_cr"] if k == 1 else a[k - 2])
    h = rel_h * max(abs(base), 1e-3)

    def run(x):
        q, aa = dict(p), a.copy()
        if k == 0:
            q["u_sh"] = x
        elif k == 1:
            q["alpha_cr"] = x
        else:
            aa[k - 2] = x
        return O.forward_loss(q, nsteps, aa)

    lp, ep = run(base + h)
    lm, em = run(base - h)
    assert ep == em, f"a discrete decision changed under the perturbation of parameter {k}"
    return (lp - lm) / (2 * h), ep


# --- single pieces --------------------------------------------------------------
def test_boris_transpose_matches_fd():
    for _ in range(5):
        v, E, B = RNG.normal(size=3) * 3, RNG.normal(size=3), RNG.normal(size=3) * 4
        dt = 0.05
        lo = RNG.normal(size=3)
        out, lv, lE, lB = O.adj_boris(v, E, B, dt, lo)
        for vec, lam in ((v, lv), (E, lE), (B, lB)):
            for d in range(3):
                h = 1e-6
                vp, vm = vec.copy(), vec.copy()
                vp[d] += h
                vm[d] -= h
                args_p = [vp if x is vec else x for x in (v, E, B)]
                args_m = [vm if x is vec else x for x in (v, E, B)]
                fp = O.adj_boris(*args_p, dt, lo)[0] @ lo
                fm = O.adj_boris(*args_m, dt, lo)[0] @ lo
                assert abs((fp - fm) / (2 * h) - lam[d]) < 1e-7 * max(1.0, abs(lam[d]))


def test_boris_preserves_speed_without_E():
    # the transpose pin above checks the derivative; this checks the forward it differentiates
    v, B = np.array([1.0, -2.0, 0.5]), np.array([0.3, 0.1, 2.0])
    out = O.adj_boris(v, np.zeros(3), B, 0.1, np.zeros(3))[0]
    assert abs(np.linalg.norm(out) - np.linalg.norm(v)) < 1e-13


def test_kick_transpose_matches_fd():
    p = W.params(nx=32, u_sh=20.0, r=4.0, seed=5)
    u2 = 5.0
    for pid in range(6):
        v = np.array([30.0, 0, 0]) + RNG.normal(size=3) * 6
        delta = 0.3 + 0.4 * RNG.random()
        lx, lvo = RNG.normal(), RNG.normal(size=3)
        out, lin = O.adj_kick(p, 3, pid, v, delta, u2, lx, lvo)
        assert out[0] < 32 and out[1] < u2   # re-enters the box moving back upstream

        def f(vv, dd, uu):
            o = O.adj_kick(p, 3, pid, vv, dd, uu, 0.0, np.zeros(3))[0]
            return lx * o[0] + lvo @ o[1:]

        h = 1e-6
        g = (f(v, delta + h, u2) - f(v, delta - h, u2)) / (2 * h)
        assert abs(g - lin[0]) < 1e-6 * max(1, abs(g))
        for d in range(3):
            vp, vm = v.copy(), v.copy()
            vp[d] += h
            vm[d] -= h
            g = (f(vp, delta, u2) - f(vm, delta, u2)) / (2 * h)
            assert abs(g - lin[1 + d]) < 1e-6 * max(1, abs(g))
        g = (f(v, delta, u2 + h) - f(v, delta, u2 - h)) / (2 * h)
        assert abs(g - lin[4]) < 1e-6 * max(1, abs(g))


def _tiny_fields(p):
    o = O.Oracle(p, "continuous")
    nc, nn = o.ncent, o.nnode
    B = np.tile([1.0, 0.2, -0.1], nc) + 0.05 * RNG.normal(size=3 * nc)
    fn = 1.0 + 0.3 * RNG.random(nn)
    fg = 0.5 * RNG.normal(size=3 * nn)
    return B, fn, fg


@pytest.mark.parametrize("dim,xbc", [(1, "box"), (2, "box"), (2, "periodic"), (3, "box")])
def test_ohm_transpose_matches_fd(dim, xbc):
    p = W.params(dim=dim, nx=6, ny=4, nz=4, dx=0.5, xbc=xbc, eta=0.01, j_ext=0.1)
    B, fn, fg = _tiny_fields(p)
    lE = RNG.normal(size=3 * len(fn))
    _, lB, lfn, lfg = O.adj_ohm(p, B, fn, fg, lE)
    h = 1e-6
    for x, lam in ((B, lB), (fn, lfn), (fg, lfg)):
        dirn = RNG.normal(size=x.shape)
        xp, xm = x + h * dirn, x - h * dirn
        args_p = [xp if y is x else y for y in (B, fn, fg)]
        args_m = [xm if y is x else y for y in (B, fn, fg)]
        fd = (O.adj_ohm(p, *args_p, lE)[0] @ lE - O.adj_ohm(p, *args_m, lE)[0] @ lE) / (2 * h)
        assert abs(fd - lam @ dirn) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("dim", [1, 2])
def test_rk3_transpose_matches_fd(dim):
    p = W.params(dim=dim, nx=8, ny=4, dx=0.5, dt=0.01, n_sub=2)
    B, fn, fg = _tiny_fields(p)
    lo = RNG.normal(size=B.shape)
    _, lB, lfn, lfg = O.adj_rk3(p, B, fn, fg, lo)
    h = 1e-6
    for x, lam in ((B, lB), (fn, lfn), (fg, lfg)):
        dirn = RNG.normal(size=x.shape)
        xp, xm = x + h * dirn, x - h * dirn
        args_p = [xp if y is x else y for y in (B, fn, fg)]
        args_m = [xm if y is x else y for y in (B, fn, fg)]
        fd = (O.adj_rk3(p, *args_p, lo)[0] @ lo - O.adj_rk3(p, *args_m, lo)[0] @ lo) / (2 * h)
        assert abs(fd - lam @ dirn) < 1e-7 * max(1.0, abs(fd))


# --- the whole gradient -----------------------------------------------------------
# (parameters, steps, index of the event count that must be non-zero:
#  1 wall reflections, 6 CR injections)
CASES = {
    # CRs injected at the wall, thermal ions open there, 40 steps
    "cic_cr_inject": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="open",
                           wall_cr="faux_shock", n_modes=3, mode_amp=0.05, seed=7), 40, 6),
    # FS acting on the thermal ions (reflections and their kick), TSC shape
    "tsc_th_fs": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, shape="tsc",
                       wall_th="faux_shock", wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=11,
                       u_sh=19.3), 12, 1),
    # 2D box with an oblique field, two RK substeps, FS on both species
    "2d_oblique": (dict(dim=2, nx=8, ny=4, dx=0.5, dt=0.0047, ppc=4, ppc_cr=4, n_cr=0.05, theta_deg=30.0,
                        wall_th="faux_shock", wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=13,
                        n_sub=2), 8, 1),
    # the reflecting wall (SPECULAR) on the thermal ions, FS on the CRs
    "specular_th": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="specular",
                         wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=19, u_sh=19.3), 12, 1),
    # the same with the conducting field boundary at the wall
    "specular_conducting": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="specular",
                                 wall_cr="faux_shock", wall_field=1, n_modes=2, mode_amp=0.05, seed=19,
                                 u_sh=19.3), 12, 1),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_gradient_matches_central_fd(case):
    kw, nsteps, must = CASES[case]
    p = W.params(**kw)
    loss, grad = O.adjoint(p, nsteps)
    fwd, events = O.forward_loss(p, nsteps)
    assert loss == fwd
    assert sum(e[must] for e in events) > 0, "the event this case is about did not happen"
    amps = O._amps(p, None)
    for k in range(len(grad)):
        fd, _ = fd_grad(p, nsteps, amps, k)
        # the build's bar is 1e-4; the oracle meets it with a wide margin
        assert abs(grad[k] - fd) <= 1e-6 * max(abs(fd), 1e-8), (k, grad[k], fd)


def test_gradient_of_amplitudes_at_step_zero_is_the_closed_form():
    """With no step taken, L = sum over the precursor centres of
    (B_y^2 + B_z^2) of the initial field, and the initial modes give
    dL/dA_m = 2 sum (B_y cos(k_m x + phi_m) + B_z sin(k_m x + phi_m)) over
    those centres: written out here from the mode definition, with the phases
    drawn from the FOURIER stream."""
    p = W.params(dim=1, nx=16, dx=0.5, ppc=8, n_modes=3, mode_amp=0.05, seed=3)
    loss, grad = O.adjoint(p, 0)
    o = O.Oracle(p, "continuous")
    o.init(O._amps(p, None))
    B = o.B()
    assert abs(loss - o.loss()) < 1e-15
    L = p["nx"] * p["dx"]
    x = (np.arange(16) + 0.5) * p["dx"]
    sel = np.arange(16) >= 8
    for m in range(1, 4):
        r = int(O.philox([m, 0, 0, 0], [p["seed"], 5])[0])
        phi = 2 * np.pi * ((r >> 11) + 0.5) * 2.0 ** -53
        arg = 2 * np.pi * m * x / L + phi
        want = 2 * np.sum(B[sel, 1] * np.cos(arg[sel]) + B[sel, 2] * np.sin(arg[sel]))
        assert abs(grad[1 + m] - want) < 1e-12 * max(1, abs(want))
    # nothing else depends on u_sh or alpha_cr before the first step except E^0,
    # which the loss does not see
    assert grad[0] == 0.0 and grad[1] == 0.0
