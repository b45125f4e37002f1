"""The 3D field update (k_fluid, the z-marching k_stage3 and k_ohm3)
against the FP64 oracle on grids that reach every boundary and blocking
path of those kernels, from one state: B^{n+1}, E^{n+1} and the gather grid
(E and the centre-averaged B at the nodes) within 1e-12, twice in a row.

  * box and periodic x, the conducting wall, CIC and TSC (whose fluid clamp
    reaches two nodes in), thermal ions alone and with CRs, fixed-point and
    continuous moments, one and two sub-steps;
  * a grid smaller than one 32 x 8 block column in every direction (the
    kernels' halos wrap around y and z several times), and one of several
    blocks in x and y with two runs of z planes, the second ragged.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W
from tests import inputs
from tests.test_gpu_parity import lib, rel

pytestmark = pytest.mark.gpu

TINY = dict(nx=13, ny=5, nz=3)
WIDE = dict(nx=70, ny=20, nz=52)

CASES = {
    "tiny-box": (TINY, {}),
    "tiny-periodic": (TINY, dict(xbc="periodic")),
    "wide-box": (WIDE, {}),
    "wide-periodic": (WIDE, dict(xbc="periodic")),
    "wide-box-tsc-cr": (WIDE, dict(shape="tsc", n_cr=0.05, ppc_cr=2)),
    "wide-box-conducting-nsub2": (WIDE, dict(wall_field=1, n_sub=2)),
    "tiny-box-continuous-cr": (TINY, dict(deposit_mode="continuous", n_cr=0.05, ppc_cr=3)),
    "wide-periodic-fp32": (WIDE, dict(xbc="periodic", precision=32)),
}


def _setup(p, seed):
    sim = lib().Simulation(p, "cuda:0")
    o = O.Oracle(p, p.get("deposit_mode", "fixed"))
    st = inputs.particle_state(p, 3, seed=seed, drift=4.0, sigma=1.0)
    sim.load_particles(0, st["cell"], st["off"], st["v"], st["id"])
    o.set_particles(0, st["cell"], st["off"], st["v"], st["id"])
    nid = int(st["id"].max()) + 1
    if p.get("n_cr", 0.0) > 0.0:
        cr = inputs.particle_state(p, int(p["ppc_cr"]), seed=seed + 1, drift=-30.0, sigma=20.0, id0=nid)
        sim.load_particles(1, cr["cell"], cr["off"], cr["v"], cr["id"])
        o.set_particles(1, cr["cell"], cr["off"], cr["v"], cr["id"])
        nid = int(cr["id"].max()) + 1
    B = inputs.magnetic_field(p, 0.1, seed=seed + 2)
    sim.set_clock(nid)
    sim.set_B(B)
    sim.deposit_moments()
    sim.refresh_fields()
    o.set_B(B)
    o.step(O.DEPOSIT)
    o.set_clock(0, nid)
    o.compute_E()
    return sim, o


@pytest.mark.parametrize("case", sorted(CASES))
def test_fused_field_update_matches_oracle(case):
    size, kw = CASES[case]
    base = dict(dim=3, dx=1.0, dt=0.01, ppc=3, seed=91, theta_deg=35.0, precision=64, beta_e=1.0, eta=0.01,
                j_ext=0.1)
    base.update(size)
    base.update(kw)
    p = W.params(**base)
    sim, o = _setup(p, seed=len(case))
    print(f"case {case}: nx {p['nx']} ny {p['ny']} nz {p['nz']}", flush=True)
    for _ in range(2):
        sim.field_update()
        o.step(O.FIELD)
        eb, ee = rel(sim.get_B(), o.B()), rel(sim.get_E(), o.E())
        g = sim.get_gather().astype(np.float64)
        assert g.shape == (sim.L.nnode, 6)
        tol_g = 1e-12 if p["precision"] == 64 else 1e-6
        eg = max(rel(g[:, 0:3], o.E()), rel(g[:, 3:6], o.Bbar()))
        print(f"  B {eb:.2e}  E {ee:.2e}  gather {eg:.2e}", flush=True)
        assert eb < 1e-12 and ee < 1e-12
        assert eg < tol_g
