"""Degenerate and ragged inputs on the GPU against the oracle: empty boxes,
CRs injected into a box without thermal ions, a box whose ions all leave,
a single ion, and grids whose sizes are not multiples of the tile shape.
Same bars as the parity tests: ids, cells and counts exact; FP64 state
within 1e-12.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W
from tests.test_gpu_parity import _free_run, by_id, rel, setup_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

COUNTS = ("incident", "reflected", "transmitted", "open_removed", "escaped", "injected_th", "injected_cr")


def lib():
    from paper_2507_14282_amd import fshybrid
    return fshybrid


def compare(sim, o, p, sp):
    assert sim.count(sp) == o.count(sp)
    g, r = by_id(sim.particles(sp)), by_id(o.particles(sp))
    assert np.array_equal(g["id"], r["id"])
    if len(g["id"]):
        assert np.array_equal(g["cell"], r["cell"])
        assert np.max(np.abs(g["off"] - r["off"])) < 1e-12
        assert rel(g["v"], r["v"]) < 1e-12
    assert np.array_equal(sim.moments(sp), o.moments(sp))


def run_pair(p, n, every=5):
    sim = lib().Simulation(p, "cuda:0")
    sim.init_plasma()
    o = O.Oracle(p)
    o.init()
    nsp = 2 if p["n_cr"] > 0 else 1
    for s in range(n):
        st, so = sim.step(s), o.step()
        for k in COUNTS:
            assert st[k] == so[k], (s, k)
        if (s + 1) % every == 0 or s == n - 1:
            for sp in range(nsp):
                compare(sim, o, p, sp)
            assert rel(sim.get_B(), o.B()) < 1e-12
            assert np.all(np.isfinite(sim.get_E()))
            assert np.max(np.abs(sim.get_E() - o.E())) <= 1e-12 * max(np.max(np.abs(o.E())), 1.0)
    return sim, o


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_empty_box(dim):
    p = W.params(dim=dim, nx=40, ny=12, nz=6, dx=0.5, ppc=0, xbc="periodic", inject=False, theta_deg=30.0,
                 precision=64)
    sim, o = run_pair(p, 5)
    assert sim.count(0) == 0
    assert np.all(sim.get_E() == 0.0)
    B = sim.get_B()
    assert np.all(B == B[0]) and rel(B, o.B()) < 1e-15


def test_cr_injection_into_a_box_without_thermal_ions():
    p = W.params(dim=1, nx=64, dx=0.5, ppc=0, n_cr=0.01, ppc_cr=16, wall_th="open", wall_cr="faux_shock",
                 precision=64)
    sim, _ = run_pair(p, 15)
    assert sim.count(0) == 0 and sim.count(1) > 0


def test_box_that_empties_through_the_open_wall():
    # 0.2 cells per step toward the open wall: the 16 cells empty in ~80 steps
    p = W.params(dim=1, nx=16, dx=0.5, ppc=32, inject=False, wall_th="open", precision=64, seed=3)
    sim, _ = run_pair(p, 110, every=10)
    assert sim.count(0) == 0
    assert not sim.moments(0).any()


def test_single_ion():
    p = W.params(dim=3, nx=16, ny=8, nz=8, dx=1.0, ppc=1, xbc="periodic", inject=False, precision=64)
    st = dict(cell=np.array([[3, 4, 2]]), off=np.array([[0.3, 0.6, 0.9]]), v=np.array([[5.0, -3.0, 2.0]]),
              id=np.array([0], dtype=np.uint64))
    rng = np.random.default_rng(2)
    L = lib().layout(p)
    B = np.tile([1.0, 0.2, 0.1], (int(L.ncent), 1)) + 0.01 * rng.normal(size=(int(L.ncent), 3))
    sim, o = setup_pair(p, st, B)
    for s in range(20):
        sim.step(s, lib().ALL)
        o.step(O.ALL)
    compare(sim, o, p, 0)
    assert rel(sim.get_B(), o.B()) < 1e-12


@pytest.mark.parametrize("dim,shape", [(2, "tsc"), (3, "tsc"), (3, "cic")])
def test_ragged_grids_fp64(dim, shape):
    p = W.params(dim=dim, nx=37 if dim == 2 else 35, ny=13 if dim == 2 else 11, nz=6, dx=0.5 if dim == 2 else 1.0,
                 ppc=8, shape=shape, precision=64, n_modes=3, mode_amp=0.02, seed=41, theta_deg=20.0)
    assert _free_run(p, 12, check_every=4) >= 0
