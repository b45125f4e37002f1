"""The time-centred ion-field coupling (coupling = 2) on the GPU against the
oracle (reading R16: density at x^{n+1}, flux at the move's midpoint, moments
at t_{n+1/2} over the field update, flux extrapolated for E^{n+1}).

  * FP64 free runs of whole steps in 1D (CIC with the FS wall, TSC with CRs),
    2D and 3D boxes and the relativistic push: ids, cells and wall counts
    bit-exact, moment grids bit-exact when no cell straddled, particles, B
    and E within 1e-12;
  * FP32 one step from the same state: particles within 1e-5, the density
    moments certified node by node (tests/certify.py); the flux moments,
    deposited at midpoints the FP32 push rounds on its own, are reported per
    array; the field update in lockstep (the oracle's from the GPU's
    moments) within 1e-5;
  * the configurations the mode refuses.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W
from tests import inputs
from tests.certify import certify_moments
from tests.test_gpu_parity import _free_run, compare_particles, rel, setup_pair, small

pytestmark = pytest.mark.gpu

TC = dict(coupling=2)


def test_fp64_cfg1_50_steps_time_centred():
    assert _free_run(W.preset("cfg1", precision=64, **TC), 50) > 0


def test_fp64_cr_tsc_box_30_steps_time_centred():
    p = W.preset("cfg5", nx=128, ppc=32, ppc_cr=32, precision=64, n_modes=8, mode_amp=0.01, shape="tsc", **TC)
    _free_run(p, 30)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp64_multid_box_20_steps_time_centred(dim):
    p = small(dim, precision=64, n_modes=3, mode_amp=0.02, u_sh=20.0, dt=0.005, **TC)
    _free_run(p, 20, check_every=5)


def test_fp64_relativistic_50_steps_time_centred():
    assert _free_run(W.preset("cfg1", precision=64, c_light=150.0, **TC), 50) > 0


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_fp32_one_step_time_centred(dim):
    p = small(dim, precision=32, dt=0.01, n_cr=0.01, ppc_cr=4, wall_th="open", wall_cr="faux_shock", **TC)
    st = inputs.particle_state(p, 8, seed=170 + dim, drift=20.0, sigma=0.7)
    B = inputs.magnetic_field(p, 0.2, seed=16)
    sim, o = setup_pair(p, st, B, step0=3)
    g = sim.step(3, F.ALL)
    r = o.step(O.PUSH | O.BOUNDARY | O.INJECT | O.DEPOSIT)
    for k in ("incident", "reflected", "transmitted", "open_removed", "escaped", "injected_th", "injected_cr"):
        assert g[k] == r[k], k
    compare_particles(sim.particles(0), o.particles(0), p, 1e-5)
    if g["injected_cr"]:
        compare_particles(sim.particles(1), o.particles(1), p, 1e-5)
    for sp in (0, 1):
        raw, nnear = certify_moments(p, sp, sim.particles(sp), o.particles(sp), sim.moments(sp), o.moments(sp),
                                     o.b, o.sv, columns=(0,))
        print(f"dim {dim} species {sp}: flux moments at the midpoints, raw per-array differences "
              + ", ".join(f"{k} {v:.2e}" for k, v in raw.items()), flush=True)
    # the field update in lockstep: the oracle's from the GPU's moments (a
    # flux code that the FP32 midpoint rounds across a boundary moves B by
    # ~1e-5 through the update, which is the moments' difference, not the
    # update's)
    for sp in (0, 1):
        o.set_moments(sp, sim.moments(sp))
    o.step(O.FIELD)
    print(f"dim {dim}: B {rel(sim.get_B(), o.B()):.2e}, E {rel(sim.get_E(), o.E()):.2e}", flush=True)
    assert rel(sim.get_B(), o.B()) < 1e-5
    assert rel(sim.get_E(), o.E()) < 1e-5


def test_time_centred_coupling_refusals():
    base = W.params(dim=1, nx=64, ppc=8, precision=32, **TC)
    for bad in (dict(smooth=1), dict(deposit_mode="continuous"), dict(coupling=3)):
        with pytest.raises(F.FsError) as e:
            F.Simulation(dict(base, **bad), "cuda:0")
        assert e.value.code == F.FS_EINVAL
    sim = F.Simulation(base, "cuda:0")
    sim.init_plasma()
    with pytest.raises(F.FsError) as e:
        sim.checkpoint()
    assert e.value.code == F.FS_EINVAL
