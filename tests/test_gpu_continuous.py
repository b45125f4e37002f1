"""The continuous deposit (deposit_mode 1: FP64 shape weights, FP64 moment
grids), which the 2D and 3D steps fuse into the push, the wall and the
injection and the 1D step runs as a pass of its own, against the FP64
oracle's continuous moments.

Free runs from the same Philox load with the eq. (1) wall on thermal ions
and CRs and injection at both ends, on boxes of several tiles in every
direction: ids, cells and wall counts exact, every moment array (R, Gx, Gy,
Gz of each species) node by node within 1e-12 of its largest entry, B and E
within 1e-12.  The continuous weights are continuous across a cell face, so
a position that rounds into the neighbouring cell moves the moments by
rounding only.
"""

import numpy as np
import pytest

from oracle import oracle as O
from tests.test_gpu_parity import compare_particles, lib, rel, small

pytestmark = pytest.mark.gpu

BOXES = {
    1: dict(nx=96),
    2: dict(nx=40, ny=20),
    3: dict(nx=40, ny=12, nz=10),
}


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_continuous_free_run_matches_oracle(dim):
    p = small(dim, precision=64, n_modes=3, mode_amp=0.02, u_sh=20.0, dt=0.005, deposit_mode="continuous",
              n_cr=0.05, ppc_cr=4, wall_th="faux_shock", wall_cr="faux_shock", seed=83, **BOXES[dim])
    sim = lib().Simulation(p, "cuda:0")
    sim.init_plasma()
    o = O.Oracle(p, "continuous")
    o.init()
    refl = inj = 0
    for s in range(20):
        st = sim.step(s)
        so = o.step()
        for k in ("incident", "reflected", "transmitted", "open_removed", "escaped", "injected_th",
                  "injected_cr"):
            assert st[k] == so[k], (s, k, st[k], so[k])
        refl += st["reflected"]
        inj += st["injected_th"] + st["injected_cr"]
        if (s + 1) % 5 == 0:
            for sp in range(2):
                assert sim.count(sp) == o.count(sp)
                compare_particles(sim.particles(sp), o.particles(sp), p, 1e-12, straddle=1e-9)
                mg = sim.moments(sp).view(np.float64).reshape(-1, 4)
                mo = o.cmoments(sp).reshape(-1, 4)
                errs = [rel(mg[:, m], mo[:, m]) for m in range(4)]
                print(f"dim {dim} step {s} species {sp}: moment errors {errs}", flush=True)
                assert max(errs) <= 1e-12, (s, sp, errs)
            assert rel(sim.get_B(), o.B()) < 1e-12
            assert rel(sim.get_E(), o.E()) < 1e-12
    # the run exercised the wall's reflections and the injection
    assert refl > 0 and inj > 0
