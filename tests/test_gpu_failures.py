"""Failure handling at the C ABI, on a tiny 1D box (two 32-cell tiles).

Errors the host detects before anything is enqueued (ids past 2^32 - 1, a
tile over capacity, a particle outside the box) return their code and leave
the state exactly as it was.  Errors only the device can see (a NaN or a
saturated velocity code in the deposit, a bin that overflows when ions move
into it) come back as FS_ENUMERIC / FS_ETILE after the step; the state is
then undefined and the box is discarded.  Every case stays within the
kernels' own bounds: a NaN position keeps its cell, saturated codes are
clamped, and bin writes past capacity are dropped and flagged.
"""

import numpy as np
import pytest

from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W

pytestmark = pytest.mark.gpu


def small(**kw):
    p = W.params(dim=1, nx=64, dx=0.5, ppc=4, seed=21, **kw)
    sim = F.Simulation(p, "cuda:0")
    sim.init_plasma()
    sim.step(0)
    return sim


def snapshot(sim):
    P = sim.particles(0)
    order = np.argsort(P["id"])
    return {k: v[order] for k, v in P.items()}, sim.get_B().copy(), sim.next_id


def assert_same(a, b):
    (pa, Ba, na), (pb, Bb, nb) = a, b
    assert na == nb
    assert np.array_equal(Ba, Bb)
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k


def test_step_refuses_ids_past_32_bits_and_keeps_the_state():
    sim = small()
    # step 1 injects one thermal ion per transverse cell (F = 0.8 per step)
    sim.set_clock(2**32)
    before = snapshot(sim)
    with pytest.raises(F.FsError) as e:
        sim.step(1)
    assert e.value.code == F.FS_EIDOVERFLOW
    assert_same(before, snapshot(sim))


def test_load_refuses_an_id_past_32_bits_and_keeps_the_state():
    sim = small()
    before = snapshot(sim)
    P = before[0]
    ids = P["id"].copy()
    ids[len(ids) // 2] = 2**32
    with pytest.raises(F.FsError) as e:
        sim.load_particles(0, P["cell"], P["off"], P["v"], ids)
    assert e.value.code == F.FS_EIDOVERFLOW
    assert_same(before, snapshot(sim))


def test_load_refuses_an_overfull_tile_and_keeps_the_state():
    sim = small()
    before = snapshot(sim)
    cap = int(sim.L.tile_cap[0])
    n = cap + 1
    cell = np.zeros((n, 3), dtype=np.int64)
    cell[:, 0] = np.arange(n) % 32          # all in tile 0
    off = np.full((n, 3), 0.5)
    v = np.zeros((n, 3))
    with pytest.raises(F.FsError) as e:
        sim.load_particles(0, cell, off, v, np.arange(n, dtype=np.uint64))
    assert e.value.code == F.FS_ECAPACITY
    assert_same(before, snapshot(sim))


def test_load_refuses_a_particle_outside_the_box_and_keeps_the_state():
    sim = small()
    before = snapshot(sim)
    P = before[0]
    off = P["off"].copy()
    off[3, 0] = np.nan
    with pytest.raises(F.FsError) as e:
        sim.load_particles(0, P["cell"], off, P["v"], P["id"])
    assert e.value.code == F.FS_EINVAL
    assert_same(before, snapshot(sim))


@pytest.mark.parametrize("bad", ["nan", "saturated"])
def test_bad_velocity_is_reported_as_numeric_error(bad):
    sim = small()
    P = snapshot(sim)[0]
    v = P["v"].copy()
    # an ion in the middle of the box: it stays in the box and deposits
    k = int(np.argmin(np.abs(P["cell"][:, 0] - 16)))
    if bad == "nan":
        v[k, 1] = np.nan
    else:
        v[k, 1] = 3.0 * float(sim.p["v_max"])   # |v_y| past the largest velocity code
    sim.load_particles(0, P["cell"], P["off"], v, P["id"])
    with pytest.raises(F.FsError) as e:
        sim.step(1)
    assert e.value.code == F.FS_ENUMERIC


def test_bin_overflow_on_the_device_is_reported():
    sim = small()
    cap = int(sim.L.tile_cap[0])
    m = cap - 16
    # m ions at rest in tile 0 and m ions in tile 1 moving 4 cells into tile 0
    cell = np.zeros((2 * m, 3), dtype=np.int64)
    cell[:m, 0] = np.arange(m) % 32
    cell[m:, 0] = 32 + np.arange(m) % 4
    off = np.full((2 * m, 3), 0.5)
    v = np.zeros((2 * m, 3))
    v[m:, 0] = -4.0 / float(sim.p["dt"] / sim.p["dx"])
    sim.load_particles(0, cell, off, v, np.arange(2 * m, dtype=np.uint64))
    sim.set_clock(2 * m)
    with pytest.raises(F.FsError) as e:
        sim.step(1)
    assert e.value.code == F.FS_ETILE
