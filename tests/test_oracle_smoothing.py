"""Pins of the optional 1-2-1 binomial filter on the fluid moments (reading
R13 of the oracle: N passes along x, then y, then z, on the boundary-filled
n_e = max(n, n_floor) and on Gamma, before Ohm's law).

Each test sets the same integer moment pattern in two oracles, without and
with the filter, and compares their node density and flux:
  * a Fourier mode of wavenumber k is scaled by cos^2(k dx / 2) per pass and
    axis (the filter's transfer function, measured by FFT), separately
    along x and y in 2D;
  * the Nyquist mode is removed exactly;
  * the periodic sum is conserved;
  * in the box, a linear profile is unchanged away from the boundary fill;
  * the floor applies before the filter.
"""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_14282_amd import workloads as W

BASE = 2.0 ** 30


def _pair(p, dens, flux=None, smooth=1):
    """Fluid (n, Gamma) without and with `smooth` passes from the moment
    pattern dens(i, j, k) (and flux(i, j, k) -> 3 values), in units of
    BASE integer moment counts."""
    out = []
    for sm in (0, smooth):
        o = O.Oracle(dict(p, smooth=sm))
        g = (o.ndx - o.nxn) // 2
        M = np.zeros((o.ndep, 4), dtype=np.int64)
        for k in range(o.nzc):
            for j in range(o.nyc):
                for i in range(o.nxn):
                    d = (i + g) + o.ndx * (j + o.nyc * k)
                    M[d, 0] = int(round(BASE * dens(i, j, k)))
                    if flux is not None:
                        M[d, 1:] = [int(round(BASE * f)) for f in flux(i, j, k)]
        o.set_moments(0, M)
        o.compute_E()
        out.append(o.fluid())
    return out


def _periodic(dim, nx=32, ny=16):
    return W.params(dim=dim, nx=nx, ny=ny if dim >= 2 else 1, nz=1, xbc="periodic", inject=False, ppc=16,
                    n_floor=1e-6)


@pytest.mark.parametrize("m,passes", [(1, 1), (3, 1), (5, 2), (9, 3)])
def test_transfer_function_along_x(m, passes):
    p = _periodic(1)
    nx = p["nx"]
    (n0, g0), (n1, g1) = _pair(p, lambda i, j, k: 1.0 + 0.3 * math.cos(2 * math.pi * m * i / nx + 0.4),
                               lambda i, j, k: (0.2 * math.sin(2 * math.pi * m * i / nx), 0.0, 0.1),
                               smooth=passes)
    want = math.cos(math.pi * m / nx) ** (2 * passes)
    f0, f1 = np.fft.rfft(n0), np.fft.rfft(n1)
    assert abs(f1[m] / f0[m] - want) < 1e-12
    assert abs(f1[0] / f0[0] - 1.0) < 1e-14          # the mean (periodic sum) is kept
    h0, h1 = np.fft.rfft(g0[:, 0]), np.fft.rfft(g1[:, 0])
    assert abs(h1[m] / h0[m] - want) < 1e-12
    np.testing.assert_allclose(g1[:, 2], g0[:, 2], rtol=1e-15)   # a constant is a fixed point


def test_transfer_function_in_2d_is_separable():
    p = _periodic(2)
    nx, ny = p["nx"], p["ny"]
    mx, my = 3, 2
    (n0, _), (n1, _) = _pair(p, lambda i, j, k: 1.0 + 0.2 * math.cos(2 * math.pi * (mx * i / nx + my * j / ny)))
    f0 = np.fft.fft2(n0.reshape(ny, nx))
    f1 = np.fft.fft2(n1.reshape(ny, nx))
    want = math.cos(math.pi * mx / nx) ** 2 * math.cos(math.pi * my / ny) ** 2
    assert abs(f1[my, mx] / f0[my, mx] - want) < 1e-12


def test_nyquist_mode_is_removed():
    p = _periodic(1)
    (n0, _), (n1, _) = _pair(p, lambda i, j, k: 1.0 + 0.5 * (-1) ** i)
    assert np.ptp(n1) == 0.0 and n1[0] == 0.5 * (n0[0] + n0[1])


def test_floor_applies_before_the_filter():
    p = dict(_periodic(1), n_floor=0.05)
    (n0, _), (n1, _) = _pair(p, lambda i, j, k: 0.0 if i % 2 else 2.0)
    # alternating floor and high value: the Nyquist mode of max(n, floor)
    assert np.allclose(n1, 0.5 * (0.05 + n0.max()), rtol=1e-15, atol=0)


def test_box_keeps_a_linear_profile_away_from_the_boundary_fill():
    p = W.params(dim=1, nx=32, xbc="box", inject=False, ppc=16, n_floor=1e-6)
    # 1 + i/64 is exact in integer moments, so the input is exactly linear
    (n0, _), (n1, _) = _pair(p, lambda i, j, k: 1.0 + i / 64.0, smooth=1)
    mclamp = 1                                       # CIC: one node on each side is filled
    inner = slice(mclamp + 1, p["nx"] - mclamp)
    assert np.array_equal(n1[inner], n0[inner])
