"""Python binding of the faux-shock hybrid library (``libfshybrid.so``).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/fshybrid.h``.  PyTorch provides the
device memory (the caller-owned buffers of the ABI) and the HIP stream.
The names follow the C entry points (``fs_init_plasma``, ``fs_step``,
``fs_deposit_moments``, ``fs_apply_faux_shock``, ``fs_field_update``).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfshybrid.so")

FS_OK, FS_EINVAL, FS_ECAPACITY, FS_EIDOVERFLOW, FS_ENUMERIC, FS_EDEVICE, FS_ETILE = 0, -1, -2, -3, -4, -5, -6
FS_PACK_IONS = 1
PUSH, INJECT, DEPOSIT, FIELD = 1, 4, 8, 16
ALL = PUSH | INJECT | DEPOSIT | FIELD
WALL = {"open": 0, "faux_shock": 1, "specular": 2}
XBC = {"box": 0, "periodic": 1}
SHAPE = {"cic": 1, "tsc": 2, 1: 1, 2: 2}

_ERRNAMES = {FS_EINVAL: "FS_EINVAL", FS_ECAPACITY: "FS_ECAPACITY", FS_EIDOVERFLOW: "FS_EIDOVERFLOW",
             FS_ENUMERIC: "FS_ENUMERIC", FS_EDEVICE: "FS_EDEVICE", FS_ETILE: "FS_ETILE"}


class FsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class FsConfig(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("dt", C.c_double),
        ("u_sh", C.c_double), ("beta_i", C.c_double), ("beta_e", C.c_double),
        ("gamma_e", C.c_double), ("theta_deg", C.c_double), ("r", C.c_double),
        ("n_cr", C.c_double), ("cr_w", C.c_double), ("alpha_cr", C.c_double), ("j_ext", C.c_double),
        ("n_floor", C.c_double), ("eta", C.c_double), ("mode_amp", C.c_double), ("v_max", C.c_double),
        ("cap_factor_th", C.c_double), ("cap_factor_cr", C.c_double), ("c_light", C.c_double),
        ("seed", C.c_uint64),
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ppc", C.c_int32), ("ppc_cr", C.c_int32), ("shape", C.c_int32), ("precision", C.c_int32),
        ("wall_th", C.c_int32), ("wall_cr", C.c_int32), ("xbc", C.c_int32), ("n_sub", C.c_int32),
        ("n_modes", C.c_int32), ("inject", C.c_int32), ("deposit_mode", C.c_int32), ("wall_model", C.c_int32),
        ("ret_f0", C.c_double), ("ret_alpha", C.c_double), ("gain", C.c_double), ("kappa", C.c_double),
        ("r_dot", C.c_double), ("smooth", C.c_int32), ("wall_field", C.c_int32),
        ("lc_depletion", C.c_double), ("coupling", C.c_int32), ("pad_coupling", C.c_int32),
    ]


class FsLayout(C.Structure):
    _fields_ = [
        ("ncent", C.c_int64), ("nnode", C.c_int64), ("ndep", C.c_int64),
        ("nxn", C.c_int64), ("ndx", C.c_int64), ("nyc", C.c_int64), ("nzc", C.c_int64),
        ("ntiles", C.c_int64),
        ("tile_cap", C.c_int64 * 2), ("capacity", C.c_int64 * 2), ("buf_bytes", C.c_int64 * 2),
        ("gather_bytes", C.c_int64),
        ("tile", C.c_int32 * 3), ("ntile", C.c_int32 * 3),
        ("b_bits", C.c_int32), ("sv_bits", C.c_int32), ("sw_bits", C.c_int32),
        ("cell_bits", C.c_int32 * 3),
        ("real_bytes", C.c_int32), ("pad", C.c_int32),
    ]


class FsParticles(C.Structure):
    _fields_ = [
        ("buf", C.c_void_p * 2), ("tile_count", C.c_void_p * 2), ("count", C.c_void_p),
        ("capacity", C.c_int64), ("tile_cap", C.c_int64), ("cur", C.c_int32), ("species", C.c_int32),
    ]


class FsFields(C.Structure):
    _fields_ = [("B", C.c_void_p), ("E", C.c_void_p), ("gather", C.c_void_p), ("mom", C.c_void_p * 2)]


class FsStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "incident", "reflected", "transmitted", "open_removed", "escaped",
        "injected_th", "injected_cr", "saturated", "out_of_range")] + [
        ("count", C.c_int64 * 2), ("next_id", C.c_int64), ("flags", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        d = {n: int(getattr(self, n)) for n, _ in self._fields_[:9]}
        d["count"] = [int(self.count[0]), int(self.count[1])]
        d["next_id"] = int(self.next_id)
        d["flags"] = int(self.flags)
        return d


class FsRecord(C.Structure):
    _fields_ = [("dst", C.c_void_p * 2), ("capacity", C.c_int64 * 2), ("id0", C.c_int64), ("stages", C.c_void_p),
                ("B_in", C.c_void_p), ("gather_in", C.c_void_p), ("fluid", C.c_void_p)]


class FsAdjoint(C.Structure):
    _fields_ = [("x", (C.c_void_p * 3) * 2 * 2), ("v", (C.c_void_p * 3) * 2 * 2), ("capacity", C.c_int64 * 2),
                ("cur", C.c_int32), ("pad", C.c_int32), ("lB", C.c_void_p), ("lE", C.c_void_p)]


class FsPacked(C.Structure):
    _fields_ = [("buf", C.c_void_p * 2), ("toff", C.c_void_p * 2), ("dst", C.c_void_p * 2), ("n", C.c_int64 * 2),
                ("status", C.c_void_p)]


DEPOSIT_MODE = {"fixed": 0, "continuous": 1, 0: 0, 1: 1}

_lib = None


def library():
    """Load the HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        L.fs_layout.argtypes = [C.POINTER(FsConfig), C.POINTER(FsLayout)]
        L.fs_create.argtypes = [C.POINTER(FsConfig), C.POINTER(vp)]
        L.fs_destroy.argtypes = [vp]
        L.fs_destroy.restype = None
        L.fs_last_error.argtypes = [vp]
        L.fs_last_error.restype = C.c_char_p
        P, F = C.POINTER(FsParticles), C.POINTER(FsFields)
        L.fs_init_plasma.argtypes = [vp, P, F, vp, vp]
        L.fs_step.argtypes = [vp, P, F, i64, u32, C.POINTER(FsStats), vp]
        L.fs_deposit_moments.argtypes = [vp, P, F, vp]
        L.fs_apply_faux_shock.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp, vp, vp]
        L.fs_field_update.argtypes = [vp, F, vp]
        L.fs_refresh_fields.argtypes = [vp, F, vp]
        L.fs_load_particles.argtypes = [vp, P, i64, vp, vp, vp, vp, vp]
        L.fs_read_particles.argtypes = [vp, P, C.POINTER(C.c_int64), vp, vp, vp, vp, vp]
        L.fs_set_clock.argtypes = [vp, i64]
        L.fs_next_id.argtypes = [vp]
        L.fs_next_id.restype = i64
        L.fs_diagnostics.argtypes = [vp, P, F, vp, vp, vp]
        L.fs_phase_space.argtypes = [vp, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
        L.fs_bperp_spectrum.argtypes = [vp, F, vp, vp]
        L.fs_bperp_spectrum_noalloc.argtypes = [vp, F, vp, vp]
        L.fs_checkpoint_bytes.argtypes = [vp, P, vp, vp]
        L.fs_checkpoint.argtypes = [vp, P, F, vp, i64, vp]
        L.fs_restore.argtypes = [vp, P, F, vp, i64, vp]
        L.fs_timing_enable.argtypes = [vp, i32]
        L.fs_timing_read.argtypes = [vp, vp, vp, vp]
        R, A = C.POINTER(FsRecord), C.POINTER(FsAdjoint)
        L.fs_step_record.argtypes = [vp, P, F, i64, R, C.POINTER(FsPacked), C.POINTER(FsStats), vp]
        K = C.POINTER(FsPacked)
        L.fs_tape_pack.argtypes = [vp, P, K, P, R, K, u32, vp]
        L.fs_tape_unpack.argtypes = [vp, K, P, vp]
        L.fs_adjoint_step.argtypes = [vp, K, F, K, F, vp, vp, i64, i64, A, vp, vp]
        L.fs_adjoint_park.argtypes = [vp, K, A, vp, i64, vp]
        L.fs_adjoint_unpark.argtypes = [vp, K, A, vp, i64, vp]
        L.fs_adjoint_init.argtypes = [vp, K, F, A, vp, vp]
        L.fs_precursor_loss.argtypes = [vp, F, vp, vp]
        L.fs_adjoint_seed.argtypes = [vp, F, A, vp, vp]
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points the binding expects the library to export."""
    return ["fs_layout", "fs_create", "fs_destroy", "fs_last_error", "fs_init_plasma", "fs_step",
            "fs_deposit_moments", "fs_apply_faux_shock", "fs_field_update", "fs_refresh_fields",
            "fs_load_particles", "fs_read_particles", "fs_set_clock", "fs_next_id", "fs_diagnostics",
            "fs_phase_space", "fs_bperp_spectrum", "fs_checkpoint_bytes", "fs_checkpoint", "fs_restore",
            "fs_timing_enable", "fs_timing_read", "fs_step_record", "fs_adjoint_step", "fs_adjoint_init",
            "fs_precursor_loss", "fs_adjoint_seed", "fs_bperp_spectrum_noalloc", "fs_tape_pack",
            "fs_adjoint_park", "fs_adjoint_unpark", "fs_tape_unpack"]


def make_config(p: dict) -> FsConfig:
    c = FsConfig()
    for k in ("dx", "dt", "u_sh", "beta_i", "beta_e", "gamma_e", "theta_deg", "r", "n_cr", "cr_w",
              "alpha_cr", "j_ext", "n_floor", "eta", "mode_amp", "v_max"):
        setattr(c, k, float(p[k]))
    c.cap_factor_th = float(p.get("cap_factor_th", 0.0))
    c.cap_factor_cr = float(p.get("cap_factor_cr", 0.0))
    c.c_light = float(p.get("c_light", 0.0))
    c.seed = int(p["seed"])
    for k in ("dim", "nx", "ny", "nz", "ppc", "ppc_cr", "n_sub", "n_modes"):
        setattr(c, k, int(p[k]))
    c.shape = SHAPE[p["shape"]]
    c.precision = int(p.get("precision", 32))
    c.wall_th = WALL[p["wall_th"]]
    c.wall_cr = WALL[p["wall_cr"]]
    c.xbc = XBC[p["xbc"]]
    c.inject = 1 if p.get("inject", True) else 0
    c.deposit_mode = DEPOSIT_MODE[p.get("deposit_mode", "fixed")]
    c.wall_model = int(p.get("wall_model", 0))
    for k, d in (("ret_f0", 1.0), ("ret_alpha", 0.0), ("gain", 1.0), ("kappa", 0.0), ("r_dot", 0.0)):
        setattr(c, k, float(p.get(k, d)))
    c.smooth = int(p.get("smooth", 0))
    c.wall_field = int(p.get("wall_field", 0))
    c.lc_depletion = float(p.get("lc_depletion", 0.0))
    c.coupling = int(p.get("coupling", 1))
    return c


def layout(p: dict) -> FsLayout:
    L = FsLayout()
    cfg = make_config(p)
    rc = library().fs_layout(C.byref(cfg), C.byref(L))
    if rc:
        raise FsError(rc, library().fs_last_error(None).decode())
    return L


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Simulation:
    """One run on one GPU: caller-owned buffers (torch) plus a library handle."""

    def __init__(self, p: dict, device: str | torch.device = "cuda:0"):
        self.p = dict(p)
        self.lib = library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the faux-shock library runs on a ROCm GPU only")
        self.cfg = make_config(p)
        self.L = layout(p)
        L = self.L
        dev = self.device
        self.real = torch.float64 if self.cfg.precision == 64 else torch.float32
        self.has_cr = float(p["n_cr"]) > 0.0
        self._keep = []
        self.counts = []
        self.bufs, self.cnts = [], []     # per species: the two particle buffers and their tile counts
        self.sp = (FsParticles * 2)()
        for s in range(2):
            nb = int(L.buf_bytes[s]) if (s == 0 or self.has_cr) else 0
            bufs = [torch.empty(max(nb, 256), dtype=torch.uint8, device=dev) for _ in range(2)]
            cnts = [torch.zeros(2 * int(L.ntiles), dtype=torch.int32, device=dev) for _ in range(2)]
            count = torch.zeros(1, dtype=torch.int64, device=dev)
            self._keep += bufs + cnts + [count]
            self.counts.append(count)
            self.bufs.append(bufs)
            self.cnts.append(cnts)
            P = self.sp[s]
            P.buf[0], P.buf[1] = bufs[0].data_ptr(), bufs[1].data_ptr()
            P.tile_count[0], P.tile_count[1] = cnts[0].data_ptr(), cnts[1].data_ptr()
            P.count = count.data_ptr()
            P.capacity = int(L.capacity[s])
            P.tile_cap = int(L.tile_cap[s])
            P.cur = 0
            P.species = s
        self.B = torch.zeros(3, int(L.ncent), dtype=torch.float64, device=dev)
        self.E = torch.zeros(3, int(L.nnode), dtype=torch.float64, device=dev)
        self.gather = torch.zeros(int(L.nnode), 6, dtype=self.real, device=dev)
        self.mom = [torch.zeros(int(L.ndep), 4, dtype=torch.int64, device=dev) for _ in range(2)]
        self.f = FsFields()
        self.f.B, self.f.E, self.f.gather = self.B.data_ptr(), self.E.data_ptr(), self.gather.data_ptr()
        self.f.mom[0], self.f.mom[1] = self.mom[0].data_ptr(), self.mom[1].data_ptr()
        h = C.c_void_p()
        self._check(self.lib.fs_create(C.byref(self.cfg), C.byref(h)), None)
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.fs_destroy(h)
            self.h = None

    # --- plumbing --------------------------------------------------------
    def _check(self, rc, h=True):
        if rc:
            msg = self.lib.fs_last_error(self.h if h else None)
            raise FsError(rc, msg.decode() if msg else "")

    @property
    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # --- the ABI calls ---------------------------------------------------
    def init_plasma(self, amps: torch.Tensor | None = None):
        if amps is not None:
            amps = amps.to(device=self.device, dtype=torch.float64).contiguous()
        self._check(self.lib.fs_init_plasma(self.h, self.sp, C.byref(self.f), _ptr(amps), self.stream))

    def step(self, step: int, flags: int = ALL, stats: bool = True):
        st = FsStats() if stats else None
        rc = self.lib.fs_step(self.h, self.sp, C.byref(self.f), int(step), int(flags),
                              C.byref(st) if st is not None else None, self.stream)
        self._check(rc)
        return st.as_dict() if st is not None else None

    def step_record(self, step: int, rec: "FsRecord", stats: bool = False, pack_in: "FsPacked | None" = None):
        """Full step that writes the record the reverse sweep needs
        (continuous deposit mode only), and with pack_in packs its input
        state's ions there."""
        st = FsStats() if stats else None
        rc = self.lib.fs_step_record(self.h, self.sp, C.byref(self.f), int(step), C.byref(rec),
                                     C.byref(pack_in) if pack_in is not None else None,
                                     C.byref(st) if st is not None else None, self.stream)
        self._check(rc)
        return st.as_dict() if st is not None else None

    def deposit_moments(self):
        self._check(self.lib.fs_deposit_moments(self.h, self.sp, C.byref(self.f), self.stream))

    def field_update(self):
        self._check(self.lib.fs_field_update(self.h, C.byref(self.f), self.stream))

    def refresh_fields(self):
        self._check(self.lib.fs_refresh_fields(self.h, C.byref(self.f), self.stream))

    def apply_faux_shock(self, species: int, step: int, ids, delta, v):
        """FS wall on a crosser list; returns (outcome, v_new, xi_new) as numpy."""
        dev = self.device
        n = len(ids)
        tid = torch.as_tensor(np.asarray(ids, dtype=np.uint32).view(np.int32), device=dev)
        tdel = torch.as_tensor(np.asarray(delta, dtype=np.float64), device=dev)
        tv = torch.as_tensor(np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n, 3).T), device=dev)
        tout = torch.zeros(n, dtype=torch.int32, device=dev)
        txi = torch.zeros(n, dtype=torch.float64, device=dev)
        self._check(self.lib.fs_apply_faux_shock(self.h, int(species), int(step), n, _ptr(tid), _ptr(tdel),
                                                 _ptr(tv), _ptr(tout), _ptr(txi), self.stream))
        torch.cuda.synchronize(dev)
        return tout.cpu().numpy(), tv.cpu().numpy().T.copy(), txi.cpu().numpy()

    # --- state access ----------------------------------------------------
    def set_clock(self, next_id: int):
        self._check(self.lib.fs_set_clock(self.h, int(next_id)))

    @property
    def next_id(self) -> int:
        return int(self.lib.fs_next_id(self.h))

    def load_particles(self, species: int, cell, off, v, ids):
        cell = np.ascontiguousarray(np.asarray(cell, dtype=np.int64).reshape(-1, 3))
        off = np.ascontiguousarray(np.asarray(off, dtype=np.float64).reshape(-1, 3))
        v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 3))
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        n = len(ids)
        torch.cuda.synchronize(self.device)
        self._check(self.lib.fs_load_particles(self.h, C.byref(self.sp[species]), n, cell.ctypes.data,
                                               off.ctypes.data, v.ctypes.data, ids.ctypes.data, self.stream))

    def particles(self, species: int = 0) -> dict:
        torch.cuda.synchronize(self.device)
        n = C.c_int64(0)
        self._check(self.lib.fs_read_particles(self.h, C.byref(self.sp[species]), C.byref(n), None, None, None,
                                               None, self.stream))
        k = n.value
        cell = np.zeros((k, 3), dtype=np.int64)
        off = np.zeros((k, 3))
        v = np.zeros((k, 3))
        ids = np.zeros(k, dtype=np.uint64)
        if k:
            self._check(self.lib.fs_read_particles(self.h, C.byref(self.sp[species]), C.byref(n), cell.ctypes.data,
                                                   off.ctypes.data, v.ctypes.data, ids.ctypes.data, self.stream))
        return dict(cell=cell, off=off, v=v, id=ids)

    def sections(self, species: int = 0, which: int | None = None) -> dict:
        """Views of one particle buffer's sections (the layout fshybrid.h
        documents: cell, off[dim], v[3], id, each on a 256-byte boundary):
        cell and id as int32, off and v in the particle precision."""
        cur = int(self.sp[species].cur) if which is None else int(which)
        buf = self.bufs[species][cur]
        cap = int(self.L.capacity[species])
        rb = 8 if self.real == torch.float64 else 4
        dim = int(self.p["dim"])
        out, pos = {}, 0

        def take(nbytes, dtype):
            nonlocal pos
            t = buf[pos:pos + nbytes].view(dtype)
            pos += (nbytes + 255) // 256 * 256
            return t

        out["cell"] = take(cap * 4, torch.int32)
        out["off"] = [take(cap * rb, self.real) for _ in range(dim)]
        out["v"] = [take(cap * rb, self.real) for _ in range(3)]
        out["id"] = take(cap * 4, torch.int32)
        out["counts"] = self.cnts[species][cur]
        out["tile_cap"] = int(self.L.tile_cap[species])
        return out

    def count(self, species: int = 0) -> int:
        return int(self.counts[species].item())

    def get_B(self) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.B.cpu().numpy().T.copy()

    def set_B(self, B):
        self.B.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(B, dtype=np.float64).T), device=self.device))

    def get_E(self) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.E.cpu().numpy().T.copy()

    def get_gather(self) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.gather.cpu().numpy()

    def set_gather_E(self, E):
        """Overwrite the E part of the gather grid (frozen-field tests)."""
        g = self.gather.cpu().numpy()
        g[:, 0:3] = np.asarray(E).reshape(-1, 3)
        self.gather.copy_(torch.as_tensor(g, device=self.device))

    def moments(self, species: int = 0) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.mom[species].cpu().numpy()

    def set_moments(self, species: int, m):
        self.mom[species].copy_(torch.as_tensor(np.asarray(m, dtype=np.int64), device=self.device))

    def timing(self, on: bool = True):
        self._check(self.lib.fs_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        """(ms, n) per phase: push, wall, inject, field, whole step."""
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.int64)
        self._check(self.lib.fs_timing_read(self.h, ms.ctypes.data, n.ctypes.data, self.stream))
        return ms, n

    def phase_space(self, species: int, component: int, edges, x_cells_per_bin: int = 1) -> np.ndarray:
        """Counts of ions per (x bin, momentum bin); component -1 bins |p|,
        0..2 bin p_x, p_y, p_z (see fs_phase_space)."""
        e = torch.as_tensor(np.ascontiguousarray(edges, dtype=np.float64), device=self.device)
        nb = int(e.numel()) - 1
        nxb = -(-int(self.p["nx"]) // int(x_cells_per_bin))
        counts = torch.zeros((nxb, max(nb, 1)), dtype=torch.int64, device=self.device)
        self._check(self.lib.fs_phase_space(self.h, self.sp, int(species), int(component), int(x_cells_per_bin),
                                            nb, _ptr(e), _ptr(counts), self.stream))
        torch.cuda.synchronize(self.device)
        return counts.cpu().numpy()

    def checkpoint(self, device: bool = False):
        """The current state (ions, B, id counter) as a byte blob: a numpy
        array on the host, or a uint8 tensor on the device."""
        nb = C.c_int64(0)
        self._check(self.lib.fs_checkpoint_bytes(self.h, self.sp, C.byref(nb), self.stream))
        if device:
            buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            ptr = _ptr(buf)
        else:
            buf = np.empty(nb.value, dtype=np.uint8)
            ptr = buf.ctypes.data
        self._check(self.lib.fs_checkpoint(self.h, self.sp, C.byref(self.f), ptr, nb.value, self.stream))
        return buf

    def restore(self, blob):
        """Load a checkpoint (numpy array or device tensor) written by a run
        of the same layout; E and the moments are recomputed."""
        if isinstance(blob, torch.Tensor):
            ptr, n = _ptr(blob), blob.numel() * blob.element_size()
        else:
            blob = np.ascontiguousarray(blob, dtype=np.uint8)
            ptr, n = blob.ctypes.data, blob.nbytes
        self._check(self.lib.fs_restore(self.h, self.sp, C.byref(self.f), ptr, int(n), self.stream))
        torch.cuda.synchronize(self.device)

    def bperp_spectrum(self) -> np.ndarray:
        """Mean over (y, z) lines of |B^_y(k)|^2 + |B^_z(k)|^2, k = 0 .. nx/2."""
        out = torch.zeros(int(self.p["nx"]) // 2 + 1, dtype=torch.float64, device=self.device)
        self._check(self.lib.fs_bperp_spectrum(self.h, C.byref(self.f), _ptr(out), self.stream))
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def diagnostics(self) -> dict:
        out = np.zeros(8)
        prof = torch.zeros(int(self.p["nx"]), dtype=torch.float64, device=self.device)
        self._check(self.lib.fs_diagnostics(self.h, self.sp, C.byref(self.f), out.ctypes.data, _ptr(prof),
                                            self.stream))
        torch.cuda.synchronize(self.device)
        keys = ("field_energy", "kinetic_th", "kinetic_cr", "n_th", "n_cr", "loss", "max_divB", "bperp2")
        d = dict(zip(keys, (float(x) for x in out)))
        d["profile"] = prof.cpu().numpy()
        return d
