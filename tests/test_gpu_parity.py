"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every test starts both sides from the same seeded input (their own Philox
initial load from the same seed, or the same state from tests/inputs.py) and
compares what they produce: ids, cells, wall counts and fixed-point moments
bit for bit; floating-point state within 1e-12 (FP64 mode) or 1e-5 per step
(FP32 mode).  A cell index that differs is accepted only where the oracle's
position lies within rounding of a cell boundary (a certified straddle).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W
from tests import inputs
from tests.certify import certify_moments

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F = None


def lib():
    global F
    if F is None:
        from paper_2507_14282_amd import fshybrid
        F = fshybrid
    return F


OFLAGS = {1: O.PUSH | O.BOUNDARY, 4: O.INJECT, 8: O.DEPOSIT, 16: O.FIELD}


def oracle_flags(gflags):
    return sum(v for k, v in OFLAGS.items() if gflags & k)


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: v[o] for k, v in d.items()}


def rel(a, b):
    den = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / max(den, 1e-300)) if a.size else 0.0


def compare_particles(g, o, p, tol, straddle=1e-5):
    g, o = by_id(g), by_id(o)
    assert np.array_equal(g["id"], o["id"]), "particle id sets differ"
    D = p["dim"]
    sizes = [p["nx"], p["ny"], p["nz"]]
    xg = g["cell"][:, :D] + g["off"][:, :D]
    xo = o["cell"][:, :D] + o["off"][:, :D]
    d = xg - xo
    for k in range(D):
        if k > 0 or p["xbc"] == "periodic":
            d[:, k] -= sizes[k] * np.round(d[:, k] / sizes[k])
    scale = max(float(np.max(np.abs(xo))) if xo.size else 1.0, 1.0)
    assert np.max(np.abs(d)) <= tol * scale, f"positions differ by {np.max(np.abs(d))}"
    mism = np.any(g["cell"][:, :D] != o["cell"][:, :D], axis=1)
    nstr = int(mism.sum())
    if nstr:
        fr = xo[mism] - np.floor(xo[mism])
        near = np.minimum(fr, 1 - fr)
        assert np.all(near < straddle), f"{nstr} cell mismatches not at cell boundaries"
    assert rel(g["v"], o["v"]) <= tol, f"velocities differ (rel {rel(g['v'], o['v'])})"
    return nstr


def setup_pair(p, state, B, step0=0, species=0):
    """GPU simulation and oracle loaded with the same particles and B."""
    sim = lib().Simulation(p, "cuda:0")
    sim.load_particles(species, state["cell"], state["off"], state["v"], state["id"])
    nid = int(state["id"].max()) + 1 if len(state["id"]) else 0
    sim.set_clock(nid)
    sim.set_B(B)
    sim.deposit_moments()
    sim.refresh_fields()
    o = O.Oracle(p)
    o.set_particles(species, state["cell"], state["off"], state["v"], state["id"])
    o.set_B(B)
    o.step(O.DEPOSIT)
    o.set_clock(step0, nid)
    o.compute_E()
    return sim, o


def small(dim, **kw):
    base = dict(dim=dim, nx=40 if dim == 1 else (24 if dim == 2 else 16), ny=16 if dim >= 2 else 1,
                nz=12 if dim >= 3 else 1, dx=0.5 if dim < 3 else 1.0, ppc=8, seed=77, theta_deg=30.0)
    base.update(kw)
    return W.params(**base)


# --------------------------------------------------------------------------
# initial load
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_init_plasma_fp64_matches_oracle(dim):
    p = small(dim, precision=64, n_modes=5, mode_amp=0.01)
    sim = lib().Simulation(p, "cuda:0")
    sim.init_plasma()
    o = O.Oracle(p)
    o.init()
    g, r = sim.particles(0), o.particles(0)
    assert len(g["id"]) == len(r["id"]) == sim.count(0)
    compare_particles(g, r, p, 1e-13)
    gs, rs = by_id(g), by_id(r)
    assert np.array_equal(gs["off"], rs["off"])          # Philox uniforms are exact
    assert rel(sim.get_B(), o.B()) < 1e-13
    assert np.array_equal(sim.moments(0), o.moments(0))
    assert rel(sim.get_E(), o.E()) < 1e-12
    assert sim.next_id == o.next_id


# --------------------------------------------------------------------------
# FP64 mode: free-running against the oracle
# --------------------------------------------------------------------------
def _free_run(p, nsteps, check_every=10):
    sim = lib().Simulation(p, "cuda:0")
    sim.init_plasma()
    o = O.Oracle(p)
    o.init()
    tot = 0
    for s in range(nsteps):
        st = sim.step(s)
        so = o.step()
        for k in ("incident", "reflected", "transmitted", "open_removed", "escaped", "injected_th",
                  "injected_cr"):
            assert st[k] == so[k], (s, k, st[k], so[k])
        tot += st["incident"]
        if (s + 1) % check_every == 0 or s == nsteps - 1:
            for sp in range(2 if p["n_cr"] > 0 else 1):
                assert sim.count(sp) == o.count(sp)
                nstr = compare_particles(sim.particles(sp), o.particles(sp), p, 1e-12, straddle=1e-9)
                if nstr == 0:
                    assert np.array_equal(sim.moments(sp), o.moments(sp)), (s, sp)
            assert rel(sim.get_B(), o.B()) < 1e-12
            assert rel(sim.get_E(), o.E()) < 1e-12
    return tot


def test_fp64_cfg1_50_steps():
    tot = _free_run(W.preset("cfg1", precision=64), 50)
    assert tot > 0


def test_fp64_cr_tsc_box_30_steps():
    p = W.preset("cfg5", nx=128, ppc=32, ppc_cr=32, precision=64, n_modes=8, mode_amp=0.01, shape="tsc")
    _free_run(p, 30)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp64_multid_box_20_steps(dim):
    p = small(dim, precision=64, n_modes=3, mode_amp=0.02, u_sh=20.0, dt=0.005)
    _free_run(p, 20, check_every=5)


# --------------------------------------------------------------------------
# deposit: bit-exact from the same state
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("dim,shape", [(1, "cic"), (1, "tsc"), (2, "cic"), (2, "tsc"), (3, "cic"), (3, "tsc")])
@pytest.mark.parametrize("xbc", ["box", "periodic"])
def test_deposit_bit_exact(precision, dim, shape, xbc):
    p = small(dim, precision=precision, shape=shape, xbc=xbc)
    st = inputs.particle_state(p, 6, seed=5 + dim, drift=3.0, sigma=40.0)
    B = inputs.magnetic_field(p, 0.1, seed=3)
    sim, o = setup_pair(p, st, B)
    for sp in (0,):
        assert np.array_equal(sim.moments(sp), o.moments(sp))


def test_deposit_permutation_invariant_on_gpu():
    p = small(3, precision=32)
    st = inputs.particle_state(p, 8, seed=9, drift=5.0, sigma=2.0)
    B = inputs.magnetic_field(p, 0.0, seed=1)
    sim, _ = setup_pair(p, st, B)
    m1 = sim.moments(0)
    perm = np.random.default_rng(1).permutation(len(st["id"]))
    sim.load_particles(0, st["cell"][perm], st["off"][perm], st["v"][perm], st["id"][perm])
    sim.deposit_moments()
    assert np.array_equal(sim.moments(0), m1)
    sim.deposit_moments()
    assert np.array_equal(sim.moments(0), m1)


# --------------------------------------------------------------------------
# wall: identical decisions from the same crossers
# --------------------------------------------------------------------------
@pytest.mark.parametrize("policy", ["faux_shock", "specular"])
def test_wall_list_matches_oracle(policy):
    p = W.params(dim=1, nx=64, u_sh=20.0, r=4.0, wall_th=policy, seed=31, precision=32)
    ids, delta, v = inputs.crosser_list(20000, seed=4, u2=5.0, wmin=0.5, wmax=80.0)
    sim = lib().Simulation(p, "cuda:0")
    out_g, v_g, xi_g = sim.apply_faux_shock(0, 123, ids, delta, v)
    out_o, v_o, xi_o = O.wall_list(p, 123, 0, ids, delta, v)
    assert np.array_equal(out_g, out_o)
    assert out_g.sum() > 0 and (policy == "specular" or out_g.sum() < len(out_g))
    assert rel(v_g, v_o) < 1e-14
    assert rel(xi_g[out_g == 1], xi_o[out_o == 1]) < 1e-14


# --------------------------------------------------------------------------
# FP64 field update from the same B and moments
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("xbc", ["box", "periodic"])
def test_field_update_fp64(dim, xbc):
    p = small(dim, precision=64, xbc=xbc, beta_e=1.0, eta=0.01, j_ext=0.1, n_sub=2)
    st = inputs.particle_state(p, 6, seed=21, drift=4.0, sigma=1.0)
    B = inputs.magnetic_field(p, 0.05, seed=8)
    sim, o = setup_pair(p, st, B)
    assert rel(sim.get_E(), o.E()) < 1e-12
    sim.field_update()
    o.step(O.FIELD)
    assert rel(sim.get_B(), o.B()) < 1e-12
    assert rel(sim.get_E(), o.E()) < 1e-12


# --------------------------------------------------------------------------
# FP32 mode: one step from the same state, per sub-step and full
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_push_fp32_one_step(dim, shape):
    p = small(dim, precision=32, shape=shape, dt=0.01)
    st = inputs.particle_state(p, 8, seed=50 + dim, drift=20.0, sigma=1.0)
    B = inputs.magnetic_field(p, 0.3, seed=6)
    sim, o = setup_pair(p, st, B, step0=7)
    g = sim.step(7, lib().PUSH)
    r = o.step(oracle_flags(lib().PUSH))
    assert (g["incident"], g["reflected"], g["transmitted"], g["escaped"]) == \
           (r["incident"], r["reflected"], r["transmitted"], r["escaped"])
    compare_particles(sim.particles(0), o.particles(0), p, 1e-5)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_full_step_fp32_one_step(dim):
    p = small(dim, precision=32, dt=0.01, n_cr=0.01, ppc_cr=4, wall_th="open", wall_cr="faux_shock")
    st = inputs.particle_state(p, 8, seed=70 + dim, drift=20.0, sigma=0.7)
    B = inputs.magnetic_field(p, 0.2, seed=16)
    sim, o = setup_pair(p, st, B, step0=3)
    g = sim.step(3, lib().ALL)
    r = o.step(O.ALL)
    for k in ("incident", "reflected", "transmitted", "open_removed", "escaped", "injected_th", "injected_cr"):
        assert g[k] == r[k], k
    compare_particles(sim.particles(0), o.particles(0), p, 1e-5)
    if g["injected_cr"]:
        compare_particles(sim.particles(1), o.particles(1), p, 1e-5)
    for sp in (0, 1):
        certify_moments(p, sp, sim.particles(sp), o.particles(sp), sim.moments(sp), o.moments(sp), o.b, o.sv)
    assert rel(sim.get_B(), o.B()) < 1e-5
    assert rel(sim.get_E(), o.E()) < 1e-5


def test_injection_matches_oracle():
    p = W.preset("cfg2", nx=64, ppc=64, ppc_cr=64, precision=64)
    sim = lib().Simulation(p, "cuda:0")
    sim.set_clock(1000)
    o = O.Oracle(p)
    o.set_clock(11, 1000)
    g = sim.step(11, lib().INJECT)
    r = o.step(O.INJECT)
    assert g["injected_th"] == r["injected_th"] > 0
    assert g["injected_cr"] == r["injected_cr"] > 0
    compare_particles(sim.particles(0), o.particles(0), p, 1e-13)
    compare_particles(sim.particles(1), o.particles(1), p, 1e-13)
    assert sim.next_id == o.next_id


def test_resume_is_bit_identical():
    p = W.preset("cfg1", nx=128, ppc=32, precision=32)
    a = lib().Simulation(p, "cuda:0")
    a.init_plasma()
    for s in range(10):
        a.step(s, stats=False)
    state = a.particles(0)
    B = a.get_B()
    b = lib().Simulation(p, "cuda:0")
    b.load_particles(0, state["cell"], state["off"], state["v"], state["id"])
    b.set_B(B)
    b.set_clock(a.next_id)
    b.deposit_moments()
    b.refresh_fields()
    for s in range(10, 20):
        a.step(s)
        b.step(s)
    ga, gb = by_id(a.particles(0)), by_id(b.particles(0))
    for k in ("id", "cell", "off", "v"):
        assert np.array_equal(ga[k], gb[k])
    assert np.array_equal(a.get_B(), b.get_B())
    assert np.array_equal(a.moments(0), b.moments(0))


def test_diagnostics_match_oracle():
    p = W.preset("cfg5", nx=128, ppc=16, ppc_cr=16, precision=64, n_modes=4, mode_amp=0.02)
    sim = lib().Simulation(p, "cuda:0")
    sim.init_plasma()
    o = O.Oracle(p)
    o.init()
    for s in range(10):
        sim.step(s)
        o.step()
    dg, do = sim.diagnostics(), o.diag()
    for k in ("field_energy", "kinetic_th", "kinetic_cr", "n_th", "n_cr", "loss", "bperp2"):
        assert abs(dg[k] - do[k]) <= 1e-12 * max(abs(do[k]), 1e-300), k
    assert dg["max_divB"] < 1e-12
    assert rel(dg["profile"], o.profile()) < 1e-12
