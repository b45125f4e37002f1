"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the FP64 CPU oracle.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads ``oracle/libfsoracle.so`` (built from ``fsoracle.c`` by
``build_oracle()``), takes the same plain parameter dict as the GPU library,
and returns numpy arrays.  It imports nothing from the GPU package.
"""

from __future__ import annotations

import contextlib
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsoracle.so")
SOURCES = ["fsoracle.c", "fsoracle_adj.c"]

PUSH, BOUNDARY, INJECT, DEPOSIT, FIELD = 1, 2, 4, 8, 16
ALL = 31
WALL = {"open": 0, "faux_shock": 1, "specular": 2}
XBC = {"box": 0, "periodic": 1}
SHAPE = {"cic": 1, "tsc": 2, 1: 1, 2: 2}


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(HERE, "fsoracle.h")])
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", LIB_PATH + ".tmp"] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OraCfg(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("dt", C.c_double),
        ("u_sh", C.c_double), ("beta_i", C.c_double), ("beta_e", C.c_double),
        ("gamma_e", C.c_double), ("theta_deg", C.c_double), ("r", C.c_double),
        ("n_cr", C.c_double), ("cr_w", C.c_double), ("alpha_cr", C.c_double),
        ("j_ext", C.c_double),
        ("n_floor", C.c_double), ("eta", C.c_double), ("mode_amp", C.c_double),
        ("v_max", C.c_double), ("c_light", C.c_double),
        ("seed", C.c_uint64),
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ppc", C.c_int32), ("ppc_cr", C.c_int32), ("shape", C.c_int32),
        ("deposit_mode", C.c_int32),
        ("wall_th", C.c_int32), ("wall_cr", C.c_int32), ("xbc", C.c_int32),
        ("n_sub", C.c_int32),
        ("n_modes", C.c_int32), ("inject", C.c_int32), ("replay", C.c_int32),
        ("wall_model", C.c_int32),
        ("ret_f0", C.c_double), ("ret_alpha", C.c_double), ("gain", C.c_double),
        ("kappa", C.c_double), ("r_dot", C.c_double), ("smooth", C.c_int32), ("wall_field", C.c_int32),
        ("lc_depletion", C.c_double), ("coupling", C.c_int32),
    ]


class OraStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "incident", "reflected", "transmitted", "open_removed", "escaped",
        "injected_th", "injected_cr", "saturated", "out_of_range")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def make_cfg(p: dict, deposit_mode: str = "fixed") -> OraCfg:
    c = OraCfg()
    for k in ("dx", "dt", "u_sh", "beta_i", "beta_e", "gamma_e", "theta_deg", "r", "n_cr",
              "cr_w", "alpha_cr", "j_ext", "n_floor", "eta", "mode_amp", "v_max"):
        setattr(c, k, float(p[k]))
    c.c_light = float(p.get("c_light", 0.0))
    c.seed = int(p["seed"])
    for k in ("dim", "nx", "ny", "nz", "ppc", "ppc_cr", "n_sub", "n_modes"):
        setattr(c, k, int(p[k]))
    c.shape = SHAPE[p["shape"]]
    c.deposit_mode = 0 if deposit_mode == "fixed" else 1
    c.wall_th = WALL[p["wall_th"]]
    c.wall_cr = WALL[p["wall_cr"]]
    c.xbc = XBC[p["xbc"]]
    c.inject = 1 if p.get("inject", True) else 0
    c.wall_model = int(p.get("wall_model", 0))
    for k, d in (("ret_f0", 1.0), ("ret_alpha", 0.0), ("gain", 1.0), ("kappa", 0.0), ("r_dot", 0.0)):
        setattr(c, k, float(p.get(k, d)))
    c.smooth = int(p.get("smooth", 0))
    c.wall_field = int(p.get("wall_field", 0))
    c.lc_depletion = float(p.get("lc_depletion", 0.0))
    c.coupling = int(p.get("coupling", 1))
    return c


_lib = None


def _load(path: str):
    L = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.ora_new.restype = vp
    L.ora_new.argtypes = [C.POINTER(OraCfg)]
    L.ora_free.argtypes = [vp]
    L.ora_init.argtypes = [vp, vp]
    L.ora_step.argtypes = [vp, i32, C.POINTER(OraStats)]
    for f in ("ora_count",):
        getattr(L, f).restype = i64
        getattr(L, f).argtypes = [vp, i32]
    for f in ("ora_next_id", "ora_get_step"):
        getattr(L, f).restype = i64
        getattr(L, f).argtypes = [vp]
    L.ora_set_clock.argtypes = [vp, i64, i64]
    L.ora_set_particles.argtypes = [vp, i32, i64, vp, vp, vp, vp]
    L.ora_get_particles.argtypes = [vp, i32, vp, vp, vp, vp]
    for f in ("ora_set_B", "ora_get_B", "ora_set_E", "ora_get_E", "ora_get_Bbar",
              "ora_profile", "ora_diag", "ora_sizes", "ora_fixed_point"):
        getattr(L, f).argtypes = [vp, vp]
    L.ora_compute_E.argtypes = [vp]
    for f in ("ora_get_moments", "ora_get_cmoments", "ora_set_moments"):
        getattr(L, f).argtypes = [vp, i32, vp]
    L.ora_get_fluid.argtypes = [vp, vp, vp]
    L.ora_loss.restype = dp
    L.ora_loss.argtypes = [vp]
    L.ora_wall_list.argtypes = [C.POINTER(OraCfg), i64, i32, i64, vp, vp, vp, vp, vp]
    L.ora_philox.argtypes = [vp, C.c_uint64, C.c_uint64, vp]
    L.ora_inject_counts.argtypes = [C.POINTER(OraCfg), i64, vp]
    L.ora_record.argtypes = [vp, i32]
    L.ora_leapfrog_start.argtypes = [vp]
    pc = C.POINTER(OraCfg)
    L.ora_push_sample.argtypes = [pc, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.ora_ohm_sample.argtypes = [pc, vp, vp, vp, i64, vp, vp, vp]
    L.ora_adjoint.restype = C.c_int
    L.ora_adjoint.argtypes = [pc, vp, i64, vp, vp]
    L.ora_adj_boris.argtypes = [vp, vp, vp, dp, vp, vp, vp, vp, vp]
    L.ora_adj_kick.argtypes = [pc, i64, C.c_uint64, vp, dp, dp, dp, vp, vp, vp]
    L.ora_adj_ohm.argtypes = [pc, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ora_adj_rk3.argtypes = [pc, vp, vp, vp, vp, vp, vp, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        _lib = _load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def variant(replacements):
    """Planted-mistake oracle, for the tests that show a pin has teeth.

    Builds a copy of the oracle sources in a temporary directory with each
    (old, new) or (file, old, new) text replacement applied (each `old` must
    occur exactly once in the sources, or in that file), and makes it the library that everything created inside
    the `with` block uses.  The oracle's own sources and library are not
    touched."""
    global _lib
    tmp = tempfile.mkdtemp(prefix="fsoracle_variant_")
    saved = lib()
    try:
        texts = {}
        for s in SOURCES + ["fsoracle.h"]:
            with open(os.path.join(HERE, s)) as f:
                texts[s] = f.read()
        for rep in replacements:
            # (old, new) anywhere in the sources, or (file, old, new)
            files = [rep[0]] if len(rep) == 3 else list(texts)
            old, new = rep[-2], rep[-1]
            total = sum(texts[s].count(old) for s in files)
            if total != 1:
                raise ValueError(f"replacement target occurs {total} times: {old!r}")
            hit = next(s for s in files if old in texts[s])
            texts[hit] = texts[hit].replace(old, new)
        for s, t in texts.items():
            with open(os.path.join(tmp, s), "w") as f:
                f.write(t)
        out = os.path.join(tmp, "libfsoracle_variant.so")
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", out] + \
              [os.path.join(tmp, s) for s in SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True, capture_output=True)
        _lib = _load(out)
        yield _lib
    finally:
        _lib = saved
        shutil.rmtree(tmp, ignore_errors=True)


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    """Philox4x64-10 block for a 4-word counter and 2-word key (uint64)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_philox(_p(c), int(key[0]), int(key[1]), _p(out))
    return out


def inject_counts(p: dict, step: int):
    out = np.zeros(2, dtype=np.int64)
    lib().ora_inject_counts(C.byref(make_cfg(p)), int(step), _p(out))
    return int(out[0]), int(out[1])


def wall_list(p: dict, step: int, species: int, ids, delta, v):
    """Apply the wall to a list of crossers; returns (outcome, v_new, xi_new)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    v = np.ascontiguousarray(np.array(v, dtype=np.float64).reshape(-1, 3))
    n = len(ids)
    xi = np.zeros(n)
    out = np.zeros(n, dtype=np.int32)
    lib().ora_wall_list(C.byref(make_cfg(p)), int(step), int(species), n, _p(ids), _p(delta),
                        _p(v), _p(xi), _p(out))
    return out, v, xi


class Oracle:
    """One FP64 simulation box held by the C oracle."""

    def __init__(self, p: dict, deposit_mode: str = "fixed"):
        self.p = dict(p)
        self.cfg = make_cfg(p, deposit_mode)
        self.L = lib()
        self.h = self.L.ora_new(C.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        s = np.zeros(6, dtype=np.int64)
        self.L.ora_sizes(self.h, _p(s))
        self.nxn, self.ndx, self.nyc, self.nzc, self.ncent, self.nnode = (int(x) for x in s)
        fp = np.zeros(3, dtype=np.int32)
        self.L.ora_fixed_point(self.h, _p(fp))
        self.b, self.sv, self.SW = (int(x) for x in fp)
        self.ndep = self.ndx * self.nyc * self.nzc

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.ora_free(h)
            self.h = None

    # --- evolution -------------------------------------------------------
    def init(self, amps=None):
        a = None
        if amps is not None:
            a = np.ascontiguousarray(amps, dtype=np.float64)
        return self.L.ora_init(self.h, _p(a) if a is not None else None)

    def step(self, flags: int = ALL) -> dict:
        st = OraStats()
        self.L.ora_step(self.h, int(flags), C.byref(st))
        return st.as_dict()

    def compute_E(self):
        self.L.ora_compute_E(self.h)

    def leapfrog_start(self):
        self.L.ora_leapfrog_start(self.h)

    # --- state -----------------------------------------------------------
    @property
    def step_index(self) -> int:
        return int(self.L.ora_get_step(self.h))

    @property
    def next_id(self) -> int:
        return int(self.L.ora_next_id(self.h))

    def set_clock(self, step: int, next_id: int):
        self.L.ora_set_clock(self.h, int(step), int(next_id))

    def count(self, species: int = 0) -> int:
        return int(self.L.ora_count(self.h, species))

    def particles(self, species: int = 0) -> dict:
        n = self.count(species)
        cell = np.zeros((n, 3), dtype=np.int64)
        off = np.zeros((n, 3))
        v = np.zeros((n, 3))
        ids = np.zeros(n, dtype=np.uint64)
        if n:
            self.L.ora_get_particles(self.h, species, _p(cell), _p(off), _p(v), _p(ids))
        return dict(cell=cell, off=off, v=v, id=ids)

    def set_particles(self, species: int, cell, off, v, ids):
        cell = np.ascontiguousarray(np.asarray(cell, dtype=np.int64).reshape(-1, 3))
        off = np.ascontiguousarray(np.asarray(off, dtype=np.float64).reshape(-1, 3))
        v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 3))
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        self.L.ora_set_particles(self.h, species, len(ids), _p(cell), _p(off), _p(v), _p(ids))

    def B(self):
        out = np.zeros((self.ncent, 3))
        self.L.ora_get_B(self.h, _p(out))
        return out

    def set_B(self, B):
        B = np.ascontiguousarray(np.asarray(B, dtype=np.float64).reshape(self.ncent, 3))
        self.L.ora_set_B(self.h, _p(B))

    def E(self):
        out = np.zeros((self.nnode, 3))
        self.L.ora_get_E(self.h, _p(out))
        return out

    def set_E(self, E):
        E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(self.nnode, 3))
        self.L.ora_set_E(self.h, _p(E))

    def Bbar(self):
        out = np.zeros((self.nnode, 3))
        self.L.ora_get_Bbar(self.h, _p(out))
        return out

    def moments(self, species: int = 0):
        out = np.zeros((self.ndep, 4), dtype=np.int64)
        self.L.ora_get_moments(self.h, species, _p(out))
        return out

    def set_moments(self, species: int, m):
        m = np.ascontiguousarray(np.asarray(m, dtype=np.int64).reshape(self.ndep, 4))
        self.L.ora_set_moments(self.h, species, _p(m))

    def cmoments(self, species: int = 0):
        out = np.zeros((self.ndep, 4))
        self.L.ora_get_cmoments(self.h, species, _p(out))
        return out

    def fluid(self):
        n = np.zeros(self.nnode)
        g = np.zeros((self.nnode, 3))
        self.L.ora_get_fluid(self.h, _p(n), _p(g))
        return n, g

    def profile(self):
        out = np.zeros(int(self.p["nx"]))
        self.L.ora_profile(self.h, _p(out))
        return out

    def loss(self) -> float:
        return float(self.L.ora_loss(self.h))

    def diag(self) -> dict:
        out = np.zeros(8)
        self.L.ora_diag(self.h, _p(out))
        keys = ("field_energy", "kinetic_th", "kinetic_cr", "n_th", "n_cr", "loss",
                "max_divB", "bperp2")
        return dict(zip(keys, (float(x) for x in out)))

    def record(self, on: bool = True):
        self.L.ora_record(self.h, 1 if on else 0)


# --- reverse mode (fsoracle_adj.c) ------------------------------------------
def _amps(p: dict, amps):
    if amps is None:
        return np.full(int(p["n_modes"]), float(p["mode_amp"]))
    return np.ascontiguousarray(amps, dtype=np.float64)


def adjoint(p: dict, nsteps: int, amps=None):
    """Loss (precursor magnetic energy after `nsteps` continuous-deposit
    steps) and its gradient [d/du_sh, d/dalpha_cr, d/dA_1 .. d/dA_M]."""
    cfg = make_cfg(p, "continuous")
    a = _amps(p, amps)
    loss = np.zeros(1)
    grad = np.zeros(2 + int(p["n_modes"]))
    rc = lib().ora_adjoint(C.byref(cfg), _p(a) if a.size else None, int(nsteps), _p(loss), _p(grad))
    if rc != 0:
        raise ValueError("oracle adjoint rejected the configuration")
    return float(loss[0]), grad


def forward_loss(p: dict, nsteps: int, amps=None):
    """The same loss from a plain forward run (continuous deposit), with the
    per-step event counts so a finite-difference caller can check that no
    discrete decision changed."""
    o = Oracle(p, "continuous")
    o.init(_amps(p, amps) if int(p["n_modes"]) else None)
    events = []
    for _ in range(nsteps):
        st = o.step()
        events.append((st["incident"], st["reflected"], st["transmitted"], st["open_removed"],
                       st["escaped"], st["injected_th"], st["injected_cr"], o.count(0), o.count(1)))
    return o.loss(), events


def adj_boris(v, E, B, dt, lam_out):
    v, E, B, lo = (np.ascontiguousarray(x, dtype=np.float64) for x in (v, E, B, lam_out))
    out, lv, lE, lB = (np.zeros(3) for _ in range(4))
    lib().ora_adj_boris(_p(v), _p(E), _p(B), float(dt), _p(lo), _p(out), _p(lv), _p(lE), _p(lB))
    return out, lv, lE, lB


def adj_kick(p: dict, step: int, pid: int, v, delta: float, u2: float, lam_x: float, lam_v):
    """FS kick of a reflected particle and its transpose: returns
    (x', v'), and the adjoints of (x_pre, v_pre, u2)."""
    cfg = make_cfg(p)
    v = np.ascontiguousarray(v, dtype=np.float64)
    lv = np.ascontiguousarray(lam_v, dtype=np.float64)
    out, lin = np.zeros(4), np.zeros(5)
    lib().ora_adj_kick(C.byref(cfg), int(step), int(pid), _p(v), float(delta), float(u2), float(lam_x),
                       _p(lv), _p(out), _p(lin))
    return out, lin


def adj_ohm(p: dict, B, fn, fg, lam_E):
    """E = Ohm(B, fn, fg) at every node and the transpose applied to lam_E."""
    cfg = make_cfg(p, "continuous")
    B, fn, fg, lE = (np.ascontiguousarray(x, dtype=np.float64) for x in (B, fn, fg, lam_E))
    E = np.zeros_like(lE)
    lB, lfn, lfg = np.zeros_like(B), np.zeros_like(fn), np.zeros_like(fg)
    lib().ora_adj_ohm(C.byref(cfg), _p(B), _p(fn), _p(fg), _p(lE), _p(E), _p(lB), _p(lfn), _p(lfg))
    return E, lB, lfn, lfg


def adj_rk3(p: dict, B, fn, fg, lam_out):
    """One SSP-RK3 field update and its transpose applied to lam_out."""
    cfg = make_cfg(p, "continuous")
    B, fn, fg = (np.ascontiguousarray(x, dtype=np.float64) for x in (B, fn, fg))
    lB = np.array(lam_out, dtype=np.float64)
    Bo = np.zeros_like(B)
    lfn, lfg = np.zeros_like(fn), np.zeros_like(fg)
    lib().ora_adj_rk3(C.byref(cfg), _p(B), _p(fn), _p(fg), _p(Bo), _p(lB), _p(lfn), _p(lfg))
    return Bo, lB, lfn, lfg


# --- diagnostics of the paper's Sec. 3 figures ----------------------------------
def phase_space(cell3, v3, nx: int, component: int, edges, x_cells_per_bin: int = 1) -> np.ndarray:
    """Counts of ions per (x bin, momentum bin), by definition: x bin = cell x
    index // x_cells_per_bin; component -1 bins |p|^2 = (p_x p_x + p_y p_y) +
    p_z p_z against the squared edges, component 0..2 bins p_c against the
    edges; bin j holds edge_j <= q < edge_{j+1}; ions outside are dropped.
    p is the stored velocity variable (four-velocity in relativistic mode)."""
    cell3 = np.asarray(cell3, dtype=np.int64).reshape(-1, 3)
    v = np.asarray(v3, dtype=np.float64).reshape(-1, 3)
    e = np.asarray(edges, dtype=np.float64)
    if component < 0:
        q = (v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2]
        E = e * e
    else:
        q = v[:, component].copy()
        E = e
    nb = len(e) - 1
    nxb = -(-int(nx) // int(x_cells_per_bin))
    j = np.searchsorted(E, q, side="right") - 1
    ok = (q >= E[0]) & (q < E[-1])
    counts = np.zeros((nxb, nb), dtype=np.int64)
    np.add.at(counts, (cell3[ok, 0] // int(x_cells_per_bin), j[ok]), 1)
    return counts


def bperp_spectrum(B3, nx: int, nyc: int, nzc: int) -> np.ndarray:
    """Mean over the (y, z) lines of |B^_y(k)|^2 + |B^_z(k)|^2, k = 0..nx/2,
    with B^(k) = (1/nx) sum_x B(x) exp(-2 pi i k x / nx) (numpy's FFT); B3 is
    (ncent, 3) with centre index i + nx (j + nyc k)."""
    B = np.asarray(B3, dtype=np.float64).reshape(nzc, nyc, nx, 3)
    Fy = np.fft.rfft(B[..., 1], axis=-1) / nx
    Fz = np.fft.rfft(B[..., 2], axis=-1) / nx
    return np.mean(np.abs(Fy) ** 2 + np.abs(Fz) ** 2, axis=(0, 1))


# --- sampled evaluation -------------------------------------------------------
def push_sample(p: dict, E3, Bb3, cell3, off3, v3):
    """Gather + Boris + move of given particles (no boundaries) in given
    node fields (nnode x 3 each); returns (cell3, off3, v3) after the push."""
    cfg = make_cfg(p)
    E3, Bb3 = (np.ascontiguousarray(x, dtype=np.float64) for x in (E3, Bb3))
    cell3 = np.ascontiguousarray(cell3, dtype=np.int64)
    off3, v3 = (np.ascontiguousarray(x, dtype=np.float64) for x in (off3, v3))
    n = len(cell3)
    co, oo, vo = np.zeros((n, 3), dtype=np.int64), np.zeros((n, 3)), np.zeros((n, 3))
    rc = lib().ora_push_sample(C.byref(cfg), _p(E3), _p(Bb3), n, _p(cell3), _p(off3), _p(v3), _p(co), _p(oo), _p(vo))
    if rc:
        raise ValueError("oracle rejected the configuration")
    return co, oo, vo


def ohm_sample(p: dict, B3, M0, M1, nodes3):
    """E and Bbar at given nodes from B (ncent x 3) and fixed-point moments."""
    cfg = make_cfg(p)
    B3 = np.ascontiguousarray(B3, dtype=np.float64)
    M0 = np.ascontiguousarray(M0, dtype=np.int64)
    M1 = None if M1 is None else np.ascontiguousarray(M1, dtype=np.int64)
    nodes3 = np.ascontiguousarray(nodes3, dtype=np.int64)
    n = len(nodes3)
    E, Bb = np.zeros((n, 3)), np.zeros((n, 3))
    rc = lib().ora_ohm_sample(C.byref(cfg), _p(B3), _p(M0), _p(M1) if M1 is not None else None, n, _p(nodes3),
                              _p(E), _p(Bb))
    if rc:
        raise ValueError("oracle rejected the configuration")
    return E, Bb

