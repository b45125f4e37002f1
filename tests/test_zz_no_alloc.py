"""The allocation-free entry point fs_bperp_spectrum_noalloc against
fs_bperp_spectrum, through the C ABI.

The variant keeps its scratch in the library's static device array instead
of memory the handle allocates, so callers that cannot allocate can take the
spectrum.  Two calls in a row, the second on a smaller box, must each give
the same spectrum as the allocating entry point (same kernels and the same
summation order: bit for bit), and a box whose scratch would not fit is
refused with FS_EINVAL.
"""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W

pytestmark = pytest.mark.gpu


def spectra(p, steps=2):
    sim = F.Simulation(p, "cuda:0")
    sim.init_plasma()
    for s in range(steps):
        sim.step(s, stats=False)
    nk = int(p["nx"]) // 2 + 1
    a = torch.full((nk,), float("nan"), dtype=torch.float64, device="cuda:0")
    b = torch.full((nk,), float("nan"), dtype=torch.float64, device="cuda:0")
    sim._check(sim.lib.fs_bperp_spectrum_noalloc(sim.h, C.byref(sim.f), C.c_void_p(a.data_ptr()), sim.stream))
    sim._check(sim.lib.fs_bperp_spectrum(sim.h, C.byref(sim.f), C.c_void_p(b.data_ptr()), sim.stream))
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_spectrum_matches_the_allocating_one_twice():
    big = W.params(dim=2, nx=512, ny=64, dx=0.5, ppc=4, n_modes=6, mode_amp=0.02, theta_deg=30.0, precision=32,
                   seed=3)
    small = W.params(dim=1, nx=96, dx=0.5, ppc=8, n_modes=3, mode_amp=0.05, precision=64, seed=4)
    for p in (big, small):
        got, want = spectra(p)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, want)
        assert got[1:].max() > 0.0


def test_noalloc_spectrum_refuses_a_box_beyond_its_scratch():
    # 2 nx + 256 (nx/2 + 1) doubles = 2,130,176 > 2^21
    p = W.params(dim=2, nx=16384, ny=256, dx=0.5, ppc=1, precision=32, seed=5)
    sim = F.Simulation(p, "cuda:0")
    out = torch.empty(p["nx"] // 2 + 1, dtype=torch.float64, device="cuda:0")
    rc = sim.lib.fs_bperp_spectrum_noalloc(sim.h, C.byref(sim.f), C.c_void_p(out.data_ptr()), sim.stream)
    assert rc == F.FS_EINVAL
    assert b"static array" in sim.lib.fs_last_error(sim.h)
