"""Workload definitions: raw parameter sets of the synthetic runs.

Pure data, no arithmetic of the method: each preset is a plain dict of the
physical and numerical parameters of one run, shaped like the paper's 1D/2D/3D
faux-shock runs (Table 1 lists box sizes, M_A, dt, theta_Bn, n_cr/n_g and
p_iso for Runs A and B).  The GPU library binding and the CPU oracle both take
such a dict; each derives everything else (u2 = u_sh/r, injection rates,
macro-particle weights, fixed-point format) on its own.

Units are the paper's (Sec. 2): lengths in d_i, time in 1/Omega_ci, speeds in
v_A, fields in B0, densities in n_g.  The flow enters at x = 0 and moves in +x
toward the faux-shock wall at x = L.
"""

from __future__ import annotations

import copy

# Defaults shared by every preset (a parameter missing from a preset takes this).
DEFAULTS = dict(
    dim=1, nx=64, ny=1, nz=1, dx=0.5, dt=0.005,
    ppc=16, ppc_cr=16, shape="cic",
    u_sh=20.0, beta_i=1.0, beta_e=1.0, gamma_e=5.0 / 3.0,
    theta_deg=0.0, r=4.0,
    n_cr=0.0, cr_w=89.44271909999159, alpha_cr=1.0, j_ext=0.0,
    wall_th="faux_shock", wall_cr="faux_shock", xbc="box",
    n_floor=0.05, eta=0.0, n_sub=1, v_max=1024.0,
    c_light=0.0,   # c / v_A; 0 is the non-relativistic push, > 0 the relativistic one
    seed=1000, n_modes=0, mode_amp=1e-3, inject=True,
    # wall_model 1 is the prescribed faux shock (return factor and its power
    # of |w| / cr_w, speed gain, direction anisotropy, d r / d t); 0 is eq. (1)
    wall_model=0, ret_f0=1.0, ret_alpha=0.0, gain=1.0, kappa=0.0, r_dot=0.0,
    # prescribed wall: share of the return flux outside the field-aligned loss
    # cone that is removed (0: the isotropic downstream population)
    lc_depletion=0.0,
    # ion-field time coupling: 1 first order (moments of the new positions,
    # frozen over the field update), 2 time-centred (moments at t_{n+1/2},
    # flux extrapolated to t_{n+1} for E^{n+1})
    coupling=1,
    smooth=0,      # passes of the 1-2-1 filter on the fluid moments (0: none)
    wall_field=0,  # 1: conducting wall at x = L (E_y = E_z = 0 there)
    precision=32, steps=10,
)

# cr_w is the CR speed in the downstream frame, sqrt(20) u_sh, so that the CR
# kinetic energy m cr_w^2 / 2 is ten times m u_sh^2 (written out as a literal
# for each Mach number; Run A of the paper uses p_iso / m = 5 u_sh).
PRESETS = {
    # 1D3V FP64 parity box: 512 cells, 64 ppc, FS acting on the thermal ions.
    # Ions the wall reflects pile up in front of it (the last tile reaches
    # ~1.8 times the mean load within the 1000 steps), hence four-fold bins.
    "cfg1": dict(dim=1, nx=512, dx=0.5, dt=0.005, ppc=64, u_sh=20.0, beta_i=1.0,
                 theta_deg=0.0, n_cr=0.0, wall_th="faux_shock", seed=1001,
                 precision=64, steps=1000, cap_factor_th=4.0),
    # 1D3V FP32: 32768 cells, 1024 ppc, TSC, CRs at 1% density from the wall.
    # Over its 20000 steps the CR-driven precursor compresses the thermal
    # plasma in front of the wall to about twice the mean tile load, so the
    # thermal bins get four times the mean (the default is two).
    "cfg2": dict(dim=1, nx=32768, dx=0.5, dt=0.0025, ppc=1024, ppc_cr=1024,
                 shape="tsc", u_sh=20.0, beta_i=1.0, theta_deg=0.0, n_cr=0.01,
                 cr_w=89.44271909999159, wall_th="open", wall_cr="faux_shock",
                 seed=1002, precision=32, steps=20000, cap_factor_th=4.0),
    # 2D3V FP32: 8192 x 512 cells, 16 ppc, M_A = 30, CRs from the wall.
    "cfg3": dict(dim=2, nx=8192, ny=512, dx=0.5, dt=0.002, ppc=16, ppc_cr=16,
                 u_sh=30.0, beta_i=1.0, theta_deg=0.0, n_cr=0.01,
                 cr_w=134.16407864998737, wall_th="open", wall_cr="faux_shock",
                 seed=1003, precision=32, steps=5000),
    # 3D3V FP32: 1024 x 192 x 192 cells, 8 ppc, theta_Bn = 45 deg.
    "cfg4": dict(dim=3, nx=1024, ny=192, nz=192, dx=1.0, dt=0.005, ppc=8,
                 u_sh=20.0, beta_i=1.0, theta_deg=45.0, n_cr=0.0,
                 wall_th="faux_shock", seed=1004, precision=32, steps=2000),
    # 1D3V adjoint run: 2048 cells, 256 ppc, CRs, 64 seeded Fourier modes.
    "cfg5": dict(dim=1, nx=2048, dx=0.5, dt=0.005, ppc=256, ppc_cr=256,
                 u_sh=20.0, beta_i=1.0, theta_deg=0.0, n_cr=0.01,
                 cr_w=89.44271909999159, wall_th="open", wall_cr="faux_shock",
                 n_modes=64, mode_amp=1e-3, seed=1005, precision=32, steps=400),
    # Reflecting-wall (RW) boxes, the paper's benchmark setup (Sec. 3, Table 1
    # Runs C and 3D): the frame is the downstream one, the flow enters at
    # u_sh = 20 v_A and the thermal ions bounce off a mirror at x = L, so a
    # real shock forms there and runs upstream at about u_sh / (r - 1).  No
    # CRs are injected.  The downstream holds r ~ 3-4 times the inflow
    # density (overshoots reach ~5 over a tile), hence six-fold bins.
    # rw1: 1D, theta_Bn = 80 deg as in Run 3D (a quasi-perpendicular shock
    # forms within ~2 / Omega_ci), sized for the oracle.
    "rw1": dict(dim=1, nx=512, dx=0.5, dt=0.005, ppc=32, u_sh=20.0, beta_i=1.0,
                theta_deg=80.0, n_cr=0.0, wall_th="specular", seed=1011,
                precision=32, steps=2400, cap_factor_th=6.0),
    # rw2: 2D, theta_Bn = 0 and dx = 1.5 d_i as in Run C (Table 1), 8192 x
    # 512 cells = 12288 x 768 d_i (Run C: 20000 x 300), with a conducting
    # wall: with the open field boundary the last cell's field grows without
    # bound between t = 12.5 and 15 (eight field substeps and a density floor
    # of 0.2 do not prevent it).  It runs to t = 20.  (rw1 keeps the open
    # boundary: in 1D the conducting wall empties the cells next to it after
    # t ~ 8.)
    "rw2": dict(dim=2, nx=8192, ny=512, dx=1.5, dt=0.005, ppc=16, u_sh=20.0,
                beta_i=1.0, theta_deg=0.0, n_cr=0.0, wall_th="specular",
                wall_field=1, seed=1012, precision=32, steps=4000,
                cap_factor_th=6.0),
}


def preset(name: str, **overrides) -> dict:
    """Full parameter dict of a named preset, with overrides applied."""
    p = copy.deepcopy(DEFAULTS)
    p.update(PRESETS[name])
    p.update(overrides)
    return p


def params(**kw) -> dict:
    """Parameter dict from the defaults with the given overrides."""
    p = copy.deepcopy(DEFAULTS)
    p.update(kw)
    return p
