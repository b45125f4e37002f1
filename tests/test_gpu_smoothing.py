"""The optional binomial filter on the fluid moments (reading R13 of the
oracle) on the GPU against the oracle:

  * the FP64 field update (Ohm, SSP-RK3 Faraday, final Ohm) with 1 and 3
    passes (CIC) and 2 (TSC), box and periodic x, 1D/2D/3D, with J_ext and a
    density floor that some nodes hit: B and E within 1e-12;
  * an FP64 free run with the filter and the faux-shock wall: ids, cells and
    wall counts bit-exact;
  * the adjoint refuses the filter.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W
from tests import inputs
from tests.test_gpu_parity import _free_run, rel, setup_pair, small

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("xbc", ["box", "periodic"])
@pytest.mark.parametrize("passes,shape", [(1, "cic"), (3, "cic"), (2, "tsc")])
def test_field_update_fp64_with_smoothing(dim, xbc, passes, shape):
    # TSC fills two boundary nodes on each x side, CIC one
    p = small(dim, precision=64, xbc=xbc, beta_e=1.0, eta=0.01, j_ext=0.1, n_sub=2, smooth=passes, n_floor=0.6,
              shape=shape)
    st = inputs.particle_state(p, 6, seed=22, drift=4.0, sigma=1.0)
    B = inputs.magnetic_field(p, 0.05, seed=9)
    sim, o = setup_pair(p, st, B)
    assert rel(sim.get_E(), o.E()) < 1e-12
    for _ in range(2):
        sim.field_update()
        o.step(O.FIELD)
        assert rel(sim.get_B(), o.B()) < 1e-12
        assert rel(sim.get_E(), o.E()) < 1e-12


def test_fp64_free_run_with_smoothing():
    p = W.preset("cfg1", nx=64, precision=64, seed=1016, smooth=2)
    assert _free_run(p, 40) > 0


def test_adjoint_refuses_smoothing():
    from paper_2507_14282_amd import adjoint as A
    p = W.preset("cfg5", nx=64, ppc=16, ppc_cr=16, n_modes=4, smooth=1)
    run = A.AdjointRun(p, nsteps=2, K=1)
    run.forward(20.0, 1.0, np.full(4, 1e-3))
    with pytest.raises(F.FsError) as e:
        run.backward()
    assert e.value.code == F.FS_EINVAL
