"""Seeded synthetic inputs shared by the GPU library and the CPU oracle.

Plain numpy random arrays with the shapes and value ranges of the runs:
particle states (cell, offset, velocity, id), magnetic fields and crosser
lists.  Every value is representable in FP32 so that the FP32 and FP64 sides
start from bit-identical states.  Nothing here computes any part of the
method.
"""

import numpy as np


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _unit_f32(rng, shape):
    u = rng.random(shape).astype(np.float32)
    return np.minimum(u, np.nextafter(np.float32(1), np.float32(0))).astype(np.float64)


def active_dims(p):
    nyc = p["ny"] if p["dim"] >= 2 else 1
    nzc = p["nz"] if p["dim"] >= 3 else 1
    return p["nx"], nyc, nzc


def particle_state(p, ppc, seed, drift=None, sigma=None, id0=0, margin=0):
    """ppc particles per cell at uniform random offsets, Maxwellian velocities
    (drift along x, thermal spread sigma), ids id0.. in cell-major order.
    `margin` keeps particles that many cells away from both x ends."""
    rng = np.random.default_rng(seed)
    nx, nyc, nzc = active_dims(p)
    drift = p["u_sh"] if drift is None else drift
    sigma = np.sqrt(p["beta_i"] / 2) if sigma is None else sigma
    xs = np.arange(margin, nx - margin)
    cells = np.array([(i, j, k) for k in range(nzc) for j in range(nyc) for i in xs], dtype=np.int64)
    cell = np.repeat(cells, ppc, axis=0)
    n = len(cell)
    off = _unit_f32(rng, (n, 3))
    off[:, p["dim"]:] = 0.0
    v = _f32(rng.normal(0.0, 1.0, (n, 3)) * sigma)
    v[:, 0] = _f32(v[:, 0] + drift)
    ids = np.arange(id0, id0 + n, dtype=np.uint64)
    return dict(cell=cell, off=off, v=v, id=ids)


def magnetic_field(p, amp, seed, theta_deg=None):
    """B0 (cos theta, sin theta, 0) plus random perturbations of size amp at
    every cell centre, as an (ncent, 3) array in x-fastest order."""
    rng = np.random.default_rng(seed)
    nx, nyc, nzc = active_dims(p)
    th = np.radians(p["theta_deg"] if theta_deg is None else theta_deg)
    n = nx * nyc * nzc
    B = np.zeros((n, 3))
    B[:, 0] = np.cos(th)
    B[:, 1] = np.sin(th)
    B += amp * rng.normal(0.0, 1.0, (n, 3))
    return B


def crosser_list(n, seed, u2, wmin, wmax):
    """n ions just past the wall: ids, overshoot in cells, velocities with
    downstream-frame speeds in [wmin, wmax] and a positive normal velocity."""
    rng = np.random.default_rng(seed)
    ids = rng.choice(2**31, size=n, replace=False).astype(np.uint64)
    delta = _f32(rng.random(n) * 0.5)
    w = rng.uniform(wmin, wmax, n)
    mu = rng.uniform(0.05, 1.0, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - mu**2)
    v = np.stack([u2 + w * mu, w * st * np.cos(phi), w * st * np.sin(phi)], 1)
    return ids, delta, _f32(v)
