"""Pins of the oracle's definitions of the paper's Sec. 3 diagnostics: the
momentum phase space / spectrum counts and the B_perp power spectrum.

The counts are checked against a brute-force loop (values on the edges,
negative components, NaN), and their sum against the number of ions; the
spectrum against a single mode's closed form, Parseval's identity and the
seeded Fourier modes of the initial load.  All run on the CPU.
"""

import math

import numpy as np

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W


def brute_counts(cell3, v3, nx, comp, edges, xpb):
    nb = len(edges) - 1
    out = np.zeros((-(-nx // xpb), nb), dtype=np.int64)
    for c, v in zip(cell3, v3):
        if comp < 0:
            q = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]
            E = [e * e for e in edges]
        else:
            q = v[comp]
            E = list(edges)
        for j in range(nb):
            if E[j] <= q < E[j + 1]:
                out[c[0] // xpb, j] += 1
                break
    return out


def test_phase_space_counts_by_brute_force():
    rng = np.random.default_rng(4)
    n, nx = 3000, 40
    cell = np.zeros((n, 3), dtype=np.int64)
    cell[:, 0] = rng.integers(0, nx, n)
    v = rng.normal(0.0, 3.0, (n, 3))
    edges_p = np.linspace(0.0, 9.0, 19)
    edges_c = np.linspace(-7.0, 7.0, 15)
    # values exactly on edges, and a NaN, must land as the definition says
    v[0] = [edges_c[3], 0.0, 0.0]
    v[1] = [edges_c[-1], 0.0, 0.0]
    v[2] = [3.0, 4.0, 0.0]               # |p| = 5 is an edge of edges_p
    v[3] = [np.nan, 1.0, 1.0]
    for comp, edges in ((-1, edges_p), (0, edges_c), (1, edges_c), (2, edges_c)):
        for xpb in (1, 3, 7):
            got = O.phase_space(cell, v, nx, comp, edges, xpb)
            assert np.array_equal(got, brute_counts(cell, v, nx, comp, edges, xpb)), (comp, xpb)
    # all ions inside wide edges are counted exactly once
    wide = np.array([0.0, 1.0, 2.0, 1e9])
    assert O.phase_space(cell, v, nx, -1, wide, 5).sum() == n - 1   # the NaN ion is dropped


def test_bperp_spectrum_single_mode_and_parseval():
    nx, nyc, nzc = 64, 3, 2
    x = np.arange(nx)
    A, m, phi = 0.37, 5, 0.8
    B = np.zeros((nzc, nyc, nx, 3))
    B[..., 0] = 1.0
    B[..., 1] = A * np.cos(2 * np.pi * m * x / nx + phi)
    B[..., 2] = A * np.sin(2 * np.pi * m * x / nx + phi)
    P = O.bperp_spectrum(B.reshape(-1, 3), nx, nyc, nzc)
    want = np.zeros(nx // 2 + 1)
    want[m] = A**2 / 2
    assert np.max(np.abs(P - want)) < 1e-15
    # Parseval for an arbitrary field: mean square = P0 + 2 sum_{0<k<nx/2} P_k + P_{nx/2}
    rng = np.random.default_rng(1)
    B = rng.normal(size=(nzc * nyc * nx, 3))
    P = O.bperp_spectrum(B, nx, nyc, nzc)
    ms = np.mean(B[:, 1] ** 2 + B[:, 2] ** 2)
    assert abs(P[0] + 2 * P[1:-1].sum() + P[-1] - ms) < 1e-13 * ms


def test_bperp_spectrum_of_the_seeded_initial_field():
    """The load's Fourier modes (amplitude A, m = 1..M) give A^2/2 at each m
    and (B0 sin theta)^2 at k = 0, nothing else."""
    p = W.params(dim=2, nx=128, ny=4, dx=0.5, ppc=1, n_modes=6, mode_amp=0.03, theta_deg=30.0, seed=12)
    o = O.Oracle(p)
    o.init()
    P = O.bperp_spectrum(o.B(), p["nx"], o.nyc, o.nzc)
    want = np.zeros(p["nx"] // 2 + 1)
    want[0] = math.sin(math.radians(30.0)) ** 2
    want[1:7] = 0.03**2 / 2
    assert np.max(np.abs(P - want)) < 1e-15
