"""GPU reverse mode against the FP64 oracle adjoint (itself pinned against
central finite differences in test_oracle_adjoint.py), on tiny boxes.

The GPU runs the continuous-deposit step (deposit_mode 1) and its adjoint
through the C ABI (fs_step_record, fs_adjoint_step, fs_adjoint_init) with
checkpoints every K steps.  FP64 mode must match the oracle's gradient to
round-off; FP32 mode (FP32 particles and particle adjoints, FP64 fields)
to the accuracy an FP32 trajectory allows.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "cic_cr_inject": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="open",
                           wall_cr="faux_shock", n_modes=3, mode_amp=0.05, seed=7), 40),
    "tsc_th_fs": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, shape="tsc",
                       wall_th="faux_shock", wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=11,
                       u_sh=19.3), 12),
    "2d_oblique": (dict(dim=2, nx=8, ny=4, dx=0.5, dt=0.0047, ppc=4, ppc_cr=4, n_cr=0.05, theta_deg=30.0,
                        wall_th="faux_shock", wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=13,
                        n_sub=2), 8),
    "3d_box": (dict(dim=3, nx=8, ny=4, nz=4, dx=0.5, dt=0.0047, ppc=2, ppc_cr=2, n_cr=0.05, theta_deg=20.0,
                    wall_th="faux_shock", wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=17), 6),
    # the reflecting wall (SPECULAR) on the thermal ions: the mirror's transpose
    "specular_th": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="specular",
                         wall_cr="faux_shock", n_modes=2, mode_amp=0.05, seed=19, u_sh=19.3), 12),
    "specular_conducting": (dict(dim=1, nx=16, dx=0.5, dt=0.0047, ppc=8, ppc_cr=8, n_cr=0.05, wall_th="specular",
                                 wall_cr="faux_shock", wall_field=1, n_modes=2, mode_amp=0.05, seed=19,
                                 u_sh=19.3), 12),
    "2d_conducting": (dict(dim=2, nx=8, ny=4, dx=0.5, dt=0.0047, ppc=4, ppc_cr=4, n_cr=0.05, theta_deg=30.0,
                           wall_th="specular", wall_cr="faux_shock", wall_field=1, n_modes=2, mode_amp=0.05,
                           seed=21, n_sub=2), 8),
}


def gpu_grad(p, nsteps, K, precision=64):
    from paper_2507_14282_amd import adjoint as A
    run = A.AdjointRun(dict(p, precision=precision), nsteps, K=K)
    amps = np.full(int(p["n_modes"]), float(p["mode_amp"]))
    loss = run.forward(p["u_sh"], p["alpha_cr"], amps)
    return loss, run.backward()


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_gradient_matches_oracle_adjoint(case):
    kw, nsteps = CASES[case]
    p = W.params(**kw)
    lo, go = O.adjoint(p, nsteps)
    print(f"case {case}: oracle loss {lo:.12e} grad {go}", flush=True)
    # K = 7 splits the run into uneven checkpoint segments
    lg, gg = gpu_grad(p, nsteps, K=7)
    print(f"case {case}: gpu    loss {lg:.12e} grad {gg}", flush=True)
    assert abs(lg - lo) <= 1e-11 * abs(lo)
    scale = np.max(np.abs(go))
    assert np.max(np.abs(gg - go)) <= 1e-8 * scale, (gg, go)


def test_checkpoint_interval_does_not_change_the_gradient():
    kw, nsteps = CASES["cic_cr_inject"]
    p = W.params(**kw)
    _, g1 = gpu_grad(p, nsteps, K=nsteps)
    _, g2 = gpu_grad(p, nsteps, K=5)
    assert np.max(np.abs(g1 - g2)) <= 1e-10 * np.max(np.abs(g1))


@pytest.mark.parametrize("case", ["cic_cr_inject", "tsc_th_fs"])
def test_fp32_gradient_near_fp64_oracle(case):
    kw, nsteps = CASES[case]
    p = W.params(**kw)
    _, go = O.adjoint(p, nsteps)
    _, gg = gpu_grad(p, nsteps, K=10, precision=32)
    print(f"case {case}: fp32 grad {gg}\n oracle {go}", flush=True)
    # FP32 particle state: the trajectory itself differs at the 1e-6 level
    assert np.max(np.abs(gg - go)) <= 2e-3 * np.max(np.abs(go)), (gg, go)


def test_autograd_function_matches_direct_backward():
    import torch
    from paper_2507_14282_amd import adjoint as A
    kw, nsteps = CASES["cic_cr_inject"]
    p = W.params(**kw, precision=64)
    run = A.AdjointRun(p, nsteps, K=10)
    u = torch.tensor(p["u_sh"], dtype=torch.float64, requires_grad=True)
    a = torch.tensor(p["alpha_cr"], dtype=torch.float64, requires_grad=True)
    amps = torch.full((p["n_modes"],), p["mode_amp"], dtype=torch.float64, requires_grad=True)
    L = A.precursor_energy(u, a, amps, run)
    L.backward()
    lo, go = O.adjoint(p, nsteps)
    got = np.concatenate([[u.grad.item(), a.grad.item()], amps.grad.numpy()])
    assert abs(L.item() - lo) <= 1e-11 * abs(lo)
    assert np.max(np.abs(got - go)) <= 1e-8 * np.max(np.abs(go))


def test_adjoint_entry_points_reject_fixed_point_mode():
    from paper_2507_14282_amd import fshybrid as F
    p = W.params(dim=1, nx=16, ppc=4)
    sim = F.Simulation(p, "cuda:0")
    sim.init_plasma()
    rec = F.FsRecord()
    with pytest.raises(F.FsError) as e:
        sim.step_record(0, rec)
    assert e.value.code == F.FS_EINVAL
