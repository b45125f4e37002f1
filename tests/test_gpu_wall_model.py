"""The prescribed faux-shock wall (wall_model = 1) on the GPU against the
oracle: return factor and its power of |w| / cr_w, speed gain, direction
anisotropy and a compression ratio drifting in time, all switched on.

  * the wall on a crosser list: identical decisions, velocities and re-entry
    points within 1e-14, at several steps (so several u2), in both modes;
  * FP64 free runs of the whole step: ids, cells and wall counts bit-exact,
    state within 1e-12 (non-relativistic and relativistic push);
  * the loss cone of an oblique shock (lc_depletion > 0): the same checks at
    several obliquities, including one whose cone is empty.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W
from tests import inputs
from tests.test_gpu_parity import _free_run, rel

pytestmark = pytest.mark.gpu

KNOBS = dict(wall_model=1, ret_f0=0.8, ret_alpha=0.5, cr_w=60.0, gain=1.2, kappa=1.5, r_dot=0.4)


@pytest.mark.parametrize("c_light", [0.0, 150.0])
def test_prescribed_wall_list_matches_oracle(c_light):
    p = W.params(dim=1, nx=64, u_sh=20.0, r=4.0, wall_th="faux_shock", seed=41, precision=32,
                 c_light=c_light, **KNOBS)
    ids, delta, v = inputs.crosser_list(20000, seed=6, u2=5.0, wmin=0.5, wmax=40.0)
    sim = F.Simulation(p, "cuda:0")
    for step in (0, 700, 4000):
        out_g, v_g, xi_g = sim.apply_faux_shock(0, step, ids, delta, v)
        out_o, v_o, xi_o = O.wall_list(p, step, 0, ids, delta, v)
        assert np.array_equal(out_g, out_o), step
        assert 0 < out_g.sum() < len(out_g)
        assert rel(v_g, v_o) < 1e-14
        assert rel(xi_g[out_g == 1], xi_o[out_o == 1]) < 1e-14


@pytest.mark.parametrize("c_light", [0.0, 150.0])
def test_fp64_free_run_with_the_prescribed_wall(c_light):
    p = W.preset("cfg1", nx=64, precision=64, seed=1015, c_light=c_light, **KNOBS)
    tot = _free_run(p, 60)
    assert tot > 0


@pytest.mark.parametrize("c_light", [0.0, 150.0])
@pytest.mark.parametrize("theta", [30.0, 45.0, 89.0])
def test_loss_cone_wall_list_matches_oracle(theta, c_light):
    p = W.params(dim=1, nx=64, u_sh=20.0, r=4.0, wall_th="faux_shock", seed=43, precision=32,
                 c_light=c_light, theta_deg=theta, lc_depletion=0.6, **KNOBS)
    ids, delta, v = inputs.crosser_list(20000, seed=7, u2=5.0, wmin=0.5, wmax=40.0)
    sim = F.Simulation(p, "cuda:0")
    p0 = dict(p, lc_depletion=0.0)
    for step in (0, 700, 4000):
        out_g, v_g, xi_g = sim.apply_faux_shock(0, step, ids, delta, v)
        out_o, v_o, xi_o = O.wall_list(p, step, 0, ids, delta, v)
        assert np.array_equal(out_g, out_o), step
        assert 0 < out_g.sum() < len(out_g)
        assert rel(v_g, v_o) < 1e-14
        assert rel(xi_g[out_g == 1], xi_o[out_o == 1]) < 1e-14
        # the depletion only ever removes returns
        out_0, _, _ = O.wall_list(p0, step, 0, ids, delta, v)
        assert np.all(out_g <= out_0) and out_g.sum() < out_0.sum()


@pytest.mark.parametrize("c_light", [0.0, 150.0])
def test_fp64_free_run_with_the_loss_cone(c_light):
    p = W.preset("cfg1", nx=64, precision=64, seed=1016, c_light=c_light, theta_deg=45.0, lc_depletion=0.7,
                 **KNOBS)
    tot = _free_run(p, 60)
    assert tot > 0


def test_loss_cone_needs_the_prescribed_wall():
    p = W.params(dim=1, nx=64, wall_th="faux_shock", theta_deg=45.0, lc_depletion=0.5, precision=32)
    with pytest.raises(F.FsError) as e:
        F.Simulation(p, "cuda:0")
    assert e.value.code == F.FS_EINVAL
    with pytest.raises(F.FsError):
        F.Simulation(dict(p, lc_depletion=1.5, **KNOBS), "cuda:0")


def test_adjoint_refuses_the_prescribed_wall():
    from paper_2507_14282_amd import adjoint as A
    p = W.preset("cfg5", nx=64, ppc=16, ppc_cr=16, n_modes=4, **dict(KNOBS, cr_w=89.44271909999159))
    run = A.AdjointRun(p, nsteps=2, K=1)
    run.forward(20.0, 1.0, np.full(4, 1e-3))
    with pytest.raises(F.FsError) as e:
        run.backward()
    assert e.value.code == F.FS_EINVAL
