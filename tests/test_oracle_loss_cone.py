"""Pins of the loss cone of the prescribed wall (reading R15 of the oracle).

The paper expects highly oblique shocks not to fill the CR loss cone
isotropically, changing the return probability and energy gain (Sec. 3.2),
and leaves the anisotropy to calibration (Sec. 1).  The reading: downstream
CRs gyrate about the compressed downstream field b2 ~ (cos th, r sin th, 0);
a return direction n lies in the loss cone when its field-aligned motion
alone outruns the receding shock, (n . s) |b2_x| > a = u2 / w, with s the
field direction pointing upstream; returns outside it are removed with
probability lc_depletion.

The pins derive the share C of the isotropic return flux that lies in the
cone by quadrature in coordinates centred on the cone axis (the flux of a
direction is proportional to its speed toward the box, (n . (-x)) - a, where
positive), independently of how the oracle draws and tests directions, and
hold the oracle's return frequency to rho^2 (C + (1 - lc_depletion)(1 - C))
and its share of returns inside the cone to C / (C + (1 - lc_depletion)(1 - C)),
within binomial error.  Special cases: no depletion and the parallel shock
(whose cone holds every return direction) give the R12 wall bit for bit; a
shock so oblique that |b2_x| < a has an empty cone.  Two planted mistakes
(the uncompressed field, the cone about the downstream-pointing field) fail.
"""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

U_SH, R = 20.0, 4.0
U2 = U_SH / R


def wall(theta, dep, **kw):
    return W.params(dim=1, nx=64, u_sh=U_SH, r=R, wall_th="faux_shock", wall_model=1, ret_f0=1.0,
                    ret_alpha=0.0, gain=1.0, kappa=0.0, lc_depletion=dep, theta_deg=theta, precision=64,
                    seed=4242, **kw)


def crossers(n, wabs, seed):
    """n crossers of downstream-frame speed wabs moving into the wall."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, 0] = np.abs(d[:, 0])
    v = wabs * d
    v[:, 0] += U2
    ids = np.arange(1, n + 1, dtype=np.uint64) * 7919
    return ids, np.full(n, 0.1), v


def cone_axis(theta):
    th = math.radians(theta)
    bn, bt = math.cos(th), R * math.sin(th)
    nb = math.hypot(bn, bt)
    return bn / nb, bt / nb          # |b2_x|, the y part of the upstream-pointing axis (negated)


def cone_share(theta, a, n=3000):
    """Share of the isotropic return flux, weight (mu' - a)+ per solid angle,
    inside the cone of half-angle acos(a / |b2_x|) about s = (-cx, -sy, 0),
    by midpoint quadrature over (alpha, beta) about s."""
    cx, sy = cone_axis(theta)
    if a >= cx:
        return 0.0
    ac = math.acos(a / cx)
    al = (np.arange(n) + 0.5) * (ac / n)
    be = (np.arange(n) + 0.5) * (2 * math.pi / n)
    A, Bt = np.meshgrid(al, be, indexing="ij")
    # n = cos(al) s + sin(al) (cos(be) e1 + sin(be) z), e1 = (-sy, cx, 0)
    mu = np.cos(A) * cx + np.sin(A) * np.cos(Bt) * sy      # n . (-x)
    f = np.clip(mu - a, 0.0, None) * np.sin(A)
    inside = f.sum() * (ac / n) * (2 * math.pi / n)
    return inside / (math.pi * (1 - a) ** 2)


def in_cone(theta, v, wabs):
    cx, sy = cone_axis(theta)
    w = v - np.array([U2, 0.0, 0.0])
    nvec = w / np.linalg.norm(w, axis=1, keepdims=True)
    ns = -nvec[:, 0] * cx - nvec[:, 1] * sy
    return ns * cx > U2 / wabs


def test_no_depletion_and_parallel_shock_are_the_r12_wall():
    ids, delta, v = crossers(20000, 30.0, 1)
    r12 = dict(wall(45.0, 0.0))
    del r12["lc_depletion"]
    same = [(O.wall_list(r12, 7, 0, ids, delta, v), O.wall_list(wall(45.0, 0.0), 7, 0, ids, delta, v)),
            (O.wall_list(wall(0.0, 0.0), 7, 0, ids, delta, v), O.wall_list(wall(0.0, 0.7), 7, 0, ids, delta, v))]
    for ref, got in same:
        assert ref[0].sum() > 0
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)


@pytest.mark.parametrize("theta,wabs", [(30.0, 30.0), (45.0, 30.0), (60.0, 60.0), (89.0, 30.0)])
def test_return_frequency_and_cone_share(theta, wabs):
    dep = 0.6
    n = 200000
    ids, delta, v = crossers(n, wabs, 2)
    out, vn, _ = O.wall_list(wall(theta, dep), 11, 0, ids, delta, v)
    a = U2 / wabs
    rho2 = ((wabs - U2) / (wabs + U2)) ** 2
    C = cone_share(theta, a)
    P = rho2 * (C + (1 - dep) * (1 - C))
    freq = out.mean()
    assert abs(freq - P) < 4.5 * math.sqrt(P * (1 - P) / n), (freq, P, C)
    ret = vn[out == 1]
    share = in_cone(theta, ret, wabs).mean()
    want = C / (C + (1 - dep) * (1 - C))
    m = len(ret)
    assert abs(share - want) < 4.5 * math.sqrt(max(want * (1 - want), 1e-12) / m) + 1e-9, (share, want)
    if theta == 89.0:
        assert C == 0.0 and share == 0.0       # |b2_x| < a: the cone is empty
    # returns keep |w| (gain 1) and leave into the box faster than u2
    w = np.linalg.norm(ret - np.array([U2, 0, 0]), axis=1)
    np.testing.assert_allclose(w, wabs, rtol=1e-13)
    assert np.all(ret[:, 0] < 0)


def mean_return_cosine(theta, a, dep, n=2000):
    """Expected direction cosine mu' of a return, by quadrature over the
    return hemisphere in (mu', phi) about -x with the flux weight (mu' - a)
    and the cone's filling (1 inside, 1 - dep outside)."""
    cx, sy = cone_axis(theta)
    mu = a + (1 - a) * (np.arange(n) + 0.5) / n
    ph = 2 * math.pi * (np.arange(n) + 0.5) / n
    M, Ph = np.meshgrid(mu, ph, indexing="ij")
    ns = M * cx - np.sqrt(1 - M * M) * np.cos(Ph) * sy
    g = np.where(ns * cx > a, 1.0, 1.0 - dep)
    wgt = (M - a) * g
    return float((M * wgt).sum() / wgt.sum())


def test_the_depletion_changes_the_energy_gain_at_oblique_shocks():
    # the returns that stay are weighted toward the cone, so their mean
    # direction cosine, and with it the speed they carry back into the box,
    # moves away from the isotropic a + 2 (1 - a) / 3
    theta, wabs, dep, n = 20.0, 60.0, 0.9, 200000
    a = U2 / wabs
    ids, delta, v = crossers(n, wabs, 3)
    out, vn, _ = O.wall_list(wall(theta, dep), 5, 0, ids, delta, v)
    mu = (U2 - vn[out == 1, 0]) / wabs
    want = mean_return_cosine(theta, a, dep)
    err = mu.std() / math.sqrt(len(mu))
    assert abs(mu.mean() - want) < 4.5 * err, (mu.mean(), want, err)
    iso = a + 2 * (1 - a) / 3
    assert abs(want - iso) > 10 * err, (want, iso, err)
    assert abs(mean_return_cosine(theta, a, 0.0) - iso) < 1e-6


UNCOMPRESSED = ("fsoracle.c", "double bn = cos(th), bt = r * sin(th);", "double bn = cos(th), bt = sin(th);")
WRONG_AXIS = ("fsoracle.c", "double ns = mu * cx - (st * cos(phi)) * sy;",
              "double ns = -mu * cx + (st * cos(phi)) * sy;")


@pytest.mark.parametrize("mistake", [UNCOMPRESSED, WRONG_AXIS], ids=["uncompressed-field", "downstream-axis"])
def test_planted_loss_cone_mistakes_fail(mistake):
    with O.variant([mistake]):
        with pytest.raises(AssertionError):
            test_return_frequency_and_cone_share(45.0, 30.0)
