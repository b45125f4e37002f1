"""CPU-side checks of the HIP library: it loads, exports every entry point
that include/fshybrid.h declares, and its host logic (layout, validation)
behaves.  No GPU compute is called."""

import ctypes as C
import os
import re

import pytest

from paper_2507_14282_amd import fshybrid as F
from paper_2507_14282_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "fshybrid.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(F.LIB_PATH)
    names = header_functions()
    assert "fs_step" in names and "fs_init_plasma" in names
    for n in names:
        assert hasattr(lib, n), n
    for n in F.exported_symbols():
        assert n in names


def header_arity():
    """Number of parameters of every fs_* function declared in the header."""
    txt = open(os.path.join(ROOT, "include", "fshybrid.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(fs_[a-z_0-9]+)\s*\(([^;{]*?)\)\s*;", txt, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    lib = F.library()
    ar = header_arity()
    assert len(ar) >= 20
    for name, n in ar.items():
        assert len(getattr(lib, name).argtypes) == n, name


def test_struct_sizes_match_header():
    # sizes of the C structs as laid out by the compiler for the ABI
    assert C.sizeof(F.FsConfig) == 19 * 8 + 8 + 16 * 4 + 5 * 8 + 2 * 4 + 8 + 2 * 4
    assert C.sizeof(F.FsParticles) == 5 * 8 + 2 * 8 + 2 * 4
    assert C.sizeof(F.FsFields) == 5 * 8
    assert C.sizeof(F.FsRecord) == 9 * 8
    assert C.sizeof(F.FsAdjoint) == 24 * 8 + 2 * 8 + 2 * 4 + 2 * 8


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"])
def test_layout_of_presets(name):
    p = W.preset(name)
    L = F.layout(p)
    nx = p["nx"]
    nyc = p["ny"] if p["dim"] >= 2 else 1
    nzc = p["nz"] if p["dim"] >= 3 else 1
    assert L.ncent == nx * nyc * nzc
    assert L.nnode == (nx + 1) * nyc * nzc
    assert L.ntiles == L.ntile[0] * L.ntile[1] * L.ntile[2]
    cells = L.tile[0] * L.tile[1] * L.tile[2]
    assert L.tile_cap[0] >= p["ppc"] * cells
    assert L.capacity[0] == L.ntiles * L.tile_cap[0]
    assert L.buf_bytes[0] >= L.capacity[0] * (8 + (p["dim"] + 3) * L.real_bytes)
    assert sum(L.cell_bits) <= 31
    assert L.sv_bits == 13  # v_max = 1024 v_A
    assert (L.tile_cap[1] > 0) == (p["n_cr"] > 0)


def test_layout_rejects_bad_configs():
    bad = [dict(dim=4), dict(shape="cic", nx=2), dict(precision=16), dict(dt=0.0), dict(v_max=-1.0),
           dict(dim=2, ny=1), dict(n_sub=0),
           # relativistic mode: c must exceed every sampled speed
           dict(c_light=-1.0), dict(c_light=25.0), dict(c_light=60.0, n_cr=0.01),
           # prescribed wall: model 0 or 1, positive factor and gain, kappa > -2,
           # a power of |w| / cr_w only with cr_w > 0
           dict(wall_model=2), dict(wall_model=1, ret_f0=0.0), dict(wall_model=1, gain=0.0),
           dict(wall_model=1, kappa=-2.0), dict(wall_model=1, ret_alpha=1.0, cr_w=0.0),
           dict(wall_model=1, r_dot=float("nan")), dict(smooth=-1), dict(smooth=65),
           dict(wall_field=2)]
    for b in bad:
        p = W.params(**{k: v for k, v in b.items()})
        if "precision" in b:
            p["precision"] = b["precision"]
        with pytest.raises(F.FsError) as e:
            F.layout(p)
        assert e.value.code == F.FS_EINVAL


def test_fixed_point_format_per_dimension():
    for dim, shape, b, sw in [(1, "cic", 22, 22), (2, "cic", 11, 22), (3, "cic", 7, 21),
                              (1, "tsc", 10, 21), (2, "tsc", 5, 22), (3, "tsc", 3, 21)]:
        p = W.params(dim=dim, nx=16, ny=8, nz=8, shape=shape)
        L = F.layout(p)
        assert (L.b_bits, L.sw_bits) == (b, sw)
        # every weight x velocity code is a 24 x 24 bit product
        assert sw <= 22


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(F, "_lib", None)
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        F.library()
