"""Reverse mode of the faux-shock step on the GPU, with checkpointing.

The loss is the precursor magnetic energy after N steps,
L = sum over cell centres with i >= nx/2 of (B_y^2 + B_z^2), and the
gradient is taken with respect to the upstream flow speed u_sh, the CR
macro-weight multiplier alpha_cr and the amplitudes of the seeded Fourier
modes of the initial field (the paper's Sec. 2 set-up: the flow speed sets
u2 = u_sh / r at the FS wall; the CR current drives the Bell instability that
fills the precursor).  The derivative is that of the continuous-deposit step
with every discrete decision of the forward run held fixed (pathwise, common
random numbers).

Everything numeric runs in the library (``fs_precursor_loss``,
``fs_adjoint_seed``, ``fs_step_record``, ``fs_tape_pack`` /
``fs_tape_unpack``, ``fs_adjoint_step``, ``fs_adjoint_park`` /
``fs_adjoint_unpark``, ``fs_adjoint_init``); this module owns the buffers
and the schedule: a forward pass that keeps a checkpoint every K steps (the
live ions packed, and the fields), and a reverse pass that re-runs each
K-step segment from its checkpoint with recording and walks it backwards.
The re-run unpacks the checkpoint into the simulation's own bins and steps
between its two buffers; every state of the segment is packed to its live
ions into the tape (``fs_packed``), together with where the step put every
ion.  Particle adjoints are indexed like the packed states, in two buffers
the reverse steps ping-pong, so the reverse passes stream them in the order
of the particles.  The tape, the records and the adjoint buffers are
allocated once and reused by every later reverse pass of the run.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import fshybrid as F


class _Bins:
    """Particle bins the reverse pass re-runs its segments on: buffers of
    their own (own=True), or one of the simulation's two buffers (`which`),
    whose forward state is not needed once the forward pass is done."""

    def __init__(self, sim: F.Simulation, nsp: int, which: int, own: bool = False):
        take = torch.empty_like if own else (lambda t: t)
        self.buf = [take(sim.bufs[k][which]) for k in range(nsp)]
        self.cnt = [take(sim.cnts[k][which]) for k in range(nsp)]

    @staticmethod
    def bytes(sim: F.Simulation, nsp: int) -> int:
        return int(sum(sim.bufs[k][0].numel() + 4 * sim.cnts[k][0].numel() for k in range(nsp)))

    def particles(self, sim: F.Simulation):
        """fs_particles structs pointing at these bins (cur 0)."""
        sp = (F.FsParticles * 2)()
        for k in range(2):
            kk = min(k, len(self.buf) - 1)
            P = sp[k]
            P.buf[0] = P.buf[1] = self.buf[kk].data_ptr()
            P.tile_count[0] = P.tile_count[1] = self.cnt[kk].data_ptr()
            P.count = sim.counts[kk].data_ptr()
            P.capacity = int(sim.L.capacity[k])
            P.tile_cap = int(sim.L.tile_cap[k])
            P.cur = 0
            P.species = k
        return sp

    # The structs only hold addresses: of these bins and of the simulation's
    # device particle count, so each is built once per simulation and kept
    # (the reverse pass would otherwise spend more host time building them
    # than the GPU spends on the small boxes' steps).
    def sp(self, sim: F.Simulation):
        key = tuple(c.data_ptr() for c in sim.counts)
        if self.__dict__.get("_sp_key") != key:
            self._sp, self._sp_key = self.particles(sim), key
        return self._sp

    def step_to(self, sim: F.Simulation, post: "_Bins"):
        """fs_particles of a step that reads these bins and writes post's
        (cur 0)."""
        key = (tuple(c.data_ptr() for c in sim.counts), post.buf[0].data_ptr())
        cache = self.__dict__.setdefault("_to", {})
        if key not in cache:
            sp = self.particles(sim)
            for k in range(len(self.buf)):
                sp[k].buf[1] = post.buf[k].data_ptr()
                sp[k].tile_count[1] = post.cnt[k].data_ptr()
            cache[key] = sp
        return cache[key]


class _Fields:
    """The grid part of a state: B, the gather grid and the moment grids,
    and (stages, for a tape state with one RK sub-step) the RK stages of the
    step that produced it, and (fluid) the fluid state its field update used.
    The reverse step does not read E, so every state shares one array for it
    (the recorded steps write it)."""

    def __init__(self, sim: F.Simulation, nsp: int, E: torch.Tensor, copy: bool = False, stages: bool = False,
                 fluid: bool = False):
        def take(t):
            return t.clone() if copy else torch.empty_like(t)
        self.B = take(sim.B)
        self.E = E
        self.gather = take(sim.gather)
        self.mom = [take(m) for m in sim.mom[:nsp]]
        self.stages = torch.empty((2,) + tuple(sim.B.shape), dtype=torch.float64, device=sim.B.device) \
            if stages else None
        self.fluid = torch.empty(5 * int(sim.L.nnode), dtype=torch.float64, device=sim.B.device) if fluid else None

    def stages_ptr(self):
        return self.stages.data_ptr() if self.stages is not None else None

    def fluid_ptr(self):
        return self.fluid.data_ptr() if self.fluid is not None else None

    def fields(self, sim: F.Simulation) -> F.FsFields:
        f = F.FsFields()
        f.B, f.E, f.gather = self.B.data_ptr(), self.E.data_ptr(), self.gather.data_ptr()
        f.mom[0] = self.mom[0].data_ptr()
        f.mom[1] = self.mom[1].data_ptr() if len(self.mom) > 1 else None
        return f

    def f(self, sim: F.Simulation) -> F.FsFields:
        if "_f" not in self.__dict__:
            self._f = self.fields(sim)
        return self._f


def _section_bytes(n: int, dim: int, rb: int) -> int:
    """Bytes of particle sections of n entries (cell, off[dim], v[3], id,
    each on a 256-byte boundary, the layout of the library's buffers)."""
    r = lambda x: (x + 255) // 256 * 256
    return r(4 * n) + (dim + 3) * r(rb * n) + r(4 * n)


class _Packed:
    """One packed state (fs_packed): the live ions of each species, the tile
    offsets and (with_dst, the tape's states) the record of the step that
    leaves the state."""

    def __init__(self, sim: F.Simulation, nsp: int, n, status: torch.Tensor, with_dst: bool = True):
        dim = int(sim.p["dim"])
        rb = torch.finfo(sim.real).bits // 8
        nt = int(sim.L.ntiles)
        dev = sim.device
        self.s = F.FsPacked()
        self.keep = []
        self.n, self.dim, self.real = [int(x) for x in n], dim, sim.real
        for k in range(nsp):
            # never empty: an empty tensor has no address (a species with
            # no ion yet still needs its arrays)
            buf = torch.empty(max(_section_bytes(int(n[k]), dim, rb), 256), dtype=torch.uint8, device=dev)
            toff = torch.empty(nt + 1, dtype=torch.int32, device=dev)
            dst = torch.empty(max(int(n[k]), 1) if with_dst else 1, dtype=torch.int32, device=dev)
            self.s.buf[k], self.s.toff[k], self.s.dst[k] = buf.data_ptr(), toff.data_ptr(), dst.data_ptr()
            self.s.n[k] = int(n[k])
            self.keep += [buf, toff, dst]
        self.s.status = status.data_ptr()

    def sections(self, k: int) -> dict:
        """Views of species k's packed ions (cell, off[dim], v[3], id), its
        tile offsets and its record."""
        buf, toff, dst = self.keep[3 * k:3 * k + 3]
        n, rb = self.n[k], torch.finfo(self.real).bits // 8
        out, pos = {}, 0

        def take(nbytes, dtype):
            nonlocal pos
            t = buf[pos:pos + nbytes].view(dtype)
            pos += (nbytes + 255) // 256 * 256
            return t

        out["cell"] = take(4 * n, torch.int32)
        out["off"] = [take(rb * n, self.real) for _ in range(self.dim)]
        out["v"] = [take(rb * n, self.real) for _ in range(3)]
        out["id"] = take(4 * n, torch.int32)
        out["toff"], out["dst"] = toff, dst[:n]
        return out

    @staticmethod
    def bytes(sim: F.Simulation, nsp: int, n, with_dst: bool = True) -> int:
        dim = int(sim.p["dim"])
        rb = torch.finfo(sim.real).bits // 8
        return sum(_section_bytes(int(n[k]), dim, rb) + 4 * ((int(n[k]) if with_dst else 1) + int(sim.L.ntiles) + 2)
                   for k in range(nsp))


class _Checkpoint:
    """A state the forward pass keeps: its ions packed (the unpacked bins
    give a re-run the same trajectories), B, the gather grid, the moment
    grids and the id counter."""

    def __init__(self, sim: F.Simulation, nsp: int, E: torch.Tensor, status: torch.Tensor):
        self.counts = [sim.count(k) for k in range(nsp)]
        self.next_id = sim.next_id
        self.packed = _Packed(sim, nsp, self.counts, status, with_dst=False)
        self.fields = _Fields(sim, nsp, E, copy=True)
        sim._check(sim.lib.fs_tape_pack(sim.h, sim.sp, C.byref(self.packed.s), None, None, None, F.FS_PACK_IONS,
                                        sim.stream))

    @staticmethod
    def bytes(sim: F.Simulation, nsp: int, n) -> int:
        return _Packed.bytes(sim, nsp, n, with_dst=False) + _fields_bytes(sim, nsp)


def _recorded_step(sim: F.Simulation, n: int, pre: _Bins, f_pre, post: _Bins, f_post, rec: F.FsRecord,
                   pack_in: "_Packed"):
    """Step n from the bins of `pre` (fields f_pre) into the bins of `post`
    (fields f_post) without copying particles or grids: the step reads B and
    the gather grid of f_pre and writes those of f_post, packing pre's ions
    into pack_in (whose offsets are set) as the push reads them."""
    rec.B_in = f_pre.B.data_ptr()
    rec.gather_in = f_pre.gather.data_ptr()
    rec.stages = f_post.stages_ptr()
    rec.fluid = f_post.fluid_ptr()
    sp = pre.step_to(sim, post)
    rc = sim.lib.fs_step_record(sim.h, sp, C.byref(f_post.f(sim)), int(n), C.byref(rec), C.byref(pack_in.s), None,
                                sim.stream)
    for k in range(2):
        sp[k].cur = 0          # the step flips it
    sim._check(rc)


def checkpoint_interval(nsteps: int, K: int, state_bytes: int, free_bytes: int, share: float = 0.8,
                        tape_bytes: int | None = None) -> int:
    """Checkpoint interval for a reverse pass that must fit in memory.

    The forward keeps ceil(nsteps / k) checkpoints of state_bytes each and
    the reverse a tape of k states of tape_bytes each (state_bytes when not
    given).  Returns the largest k <= K for which both fit in `share` of
    free_bytes.  Raises MemoryError if no interval fits.  The gradient does
    not depend on k."""
    nsteps, K = max(1, int(nsteps)), max(1, int(K))
    tape = float(state_bytes if tape_bytes is None else tape_bytes)
    budget = share * float(free_bytes)
    for k in range(min(K, nsteps), 0, -1):
        if (-(-nsteps // k)) * float(state_bytes) + k * tape <= budget:
            return k
    raise MemoryError(f"a reverse pass over {nsteps} steps needs at least "
                      f"{2 * (nsteps ** 0.5) * (state_bytes * tape) ** 0.5 / 1e9:.1f} GB of checkpoints and tape "
                      f"({state_bytes / 1e9:.2f} GB per checkpoint, {tape / 1e9:.2f} GB per tape state), "
                      f"{free_bytes / 1e9:.1f} GB are free")


def _fields_bytes(sim: F.Simulation, nsp: int, stages: bool = False, fluid: bool = False) -> int:
    """Bytes of the grids of one state (E is shared), with the two RK stages
    and the fluid state of a tape state."""
    t = [sim.B, sim.gather] + list(sim.mom[:nsp])
    return int(sum(x.numel() * x.element_size() for x in t) + (2 * 8 * sim.B.numel() if stages else 0)
               + (5 * 8 * int(sim.L.nnode) if fluid else 0))


def _fixed_bytes(sim: F.Simulation, nsp: int, n) -> int:
    """Bytes the reverse pass holds besides checkpoints, tape and working
    bins of its own: the bin record, the shared E, the adjoints (two buffers
    of n per species and the grid adjoints) and the id-indexed parking
    scratch."""
    dim = int(sim.p["dim"])
    rb = torch.finfo(sim.real).bits // 8
    work = sum(4 * int(sim.L.capacity[k]) for k in range(nsp))
    work += sim.E.numel() * sim.E.element_size()
    lam = sum(2 * (dim + 3) * rb * int(n[k]) for k in range(nsp)) + 8 * (3 * int(sim.L.ncent) + 6 * int(sim.L.nnode))
    park = nsp * (dim + 3) * rb * int(sim.next_id + sim.next_id // 8 + 4096)
    return work + lam + park


class AdjointRun:
    """Forward and reverse passes of N steps of one configuration.

    p: parameter dict (the deposit is forced to the continuous mode);
    nsteps: N; K: checkpoint interval.
    """

    def __init__(self, p: dict, nsteps: int, K: int = 20, device: str | torch.device = "cuda:0"):
        self.p = dict(p, deposit_mode="continuous")
        self.nsteps = int(nsteps)
        self.K = max(1, int(K))
        self.device = torch.device(device)
        self.sim = None
        self.checkpoints = {}
        self._bufs = None      # tape, records and adjoints, kept for later reverse passes
        self._E = None         # the E every kept state shares
        self._status = None    # overflow flag of every packed state

    # --- forward ----------------------------------------------------------
    def forward(self, u_sh: float, alpha_cr: float, amps) -> float:
        p = dict(self.p, u_sh=float(u_sh), alpha_cr=float(alpha_cr))
        self.p_run = p
        self.checkpoints = {}
        self.sim = None
        sim = F.Simulation(p, self.device)
        self.sim = sim
        self.nsp = 2 if sim.has_cr else 1
        a = None
        if int(p["n_modes"]) > 0:
            a = torch.as_tensor(np.asarray(amps, dtype=np.float64), device=self.device)
        sim.init_plasma(a)
        # the interval actually used: the requested one, or less if the
        # checkpoints and the tape would not fit in the memory free on the
        # device plus what the allocator holds unused; the tape's packed
        # states are sized here from the initial load (the reverse pass sizes
        # them exactly from the counts the forward pass saw)
        free, _ = torch.cuda.mem_get_info(self.device)
        free += torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        if self._bufs is not None and self._bufs["key"] == self._key(sim):
            free += self._bufs["bytes"]          # reused, already counted out of free
        else:
            self._bufs = None
        if self._E is None or self._E.shape != sim.E.shape or self._E.dtype != sim.E.dtype:
            self._E = torch.empty_like(sim.E)
            self._status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._status.zero_()
        # a packed state holds at most the initial ions plus those injected
        # since: bounded here by (ppc + ppc_cr) per transverse cell and step
        # (the CFL-limited inflow) and a sixteenth
        ntr = int(sim.L.nyc) * int(sim.L.nzc)
        grow = self.nsteps * ntr * (int(p["ppc"]) + int(p.get("ppc_cr", 0)))
        n0 = [sim.count(k) for k in range(self.nsp)]
        n_est = [c + c // 16 + grow + 4096 for c in n0]
        free -= _fixed_bytes(sim, self.nsp, n_est)
        # a tape state keeps the RK stages of its step (one sub-step only),
        # which the reverse step would otherwise recompute
        self.keep_stages = int(p["n_sub"]) == 1
        tape = _fields_bytes(sim, self.nsp, self.keep_stages) + _Packed.bytes(sim, self.nsp, n_est)
        ckb = _Checkpoint.bytes(sim, self.nsp, n_est)
        # the re-runs step between two bin buffers of their own when those
        # fit beside the requested interval (measured 5% faster on the 2D box
        # than stepping on the simulation's own buffers), else on the
        # simulation's
        own = 2 * _Bins.bytes(sim, self.nsp)
        want = min(self.K, self.nsteps)
        try:
            k_own = checkpoint_interval(self.nsteps, self.K, ckb, free - own, tape_bytes=tape)
        except MemoryError:
            k_own = 0
        self.own_bins = k_own == want
        self.K_run = k_own if self.own_bins else checkpoint_interval(self.nsteps, self.K, ckb, free, tape_bytes=tape)
        # a tape state also keeps its step's fluid state, which the reverse
        # step would otherwise recompute from the moments, where that does
        # not shorten the interval (unfiltered moments)
        self.keep_fluid = False
        if int(p.get("smooth", 0)) == 0:
            tape_fl = tape + _fields_bytes(sim, self.nsp, self.keep_stages, True) \
                - _fields_bytes(sim, self.nsp, self.keep_stages)
            try:
                k_fl = checkpoint_interval(self.nsteps, self.K, ckb, free - (own if self.own_bins else 0),
                                           tape_bytes=tape_fl)
            except MemoryError:
                k_fl = 0
            self.keep_fluid = k_fl == self.K_run
        for n in range(self.nsteps):
            if n % self.K_run == 0:
                self.checkpoints[n] = _Checkpoint(sim, self.nsp, self._E, self._status)
            # the last step of each segment reports its counters, so a tile
            # bin or crosser list that overflowed raises (FS_ETILE) rather
            # than dropping ions from the differentiated run
            sim.step(n, stats=(n + 1) % self.K_run == 0 or n + 1 == self.nsteps)
        self.nid = sim.next_id
        return self.loss_value()

    def loss_value(self) -> float:
        """The precursor loss of the current state (fs_precursor_loss)."""
        sim = self.sim
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        sim._check(sim.lib.fs_precursor_loss(sim.h, C.byref(sim.f), C.c_void_p(out.data_ptr()), sim.stream))
        torch.cuda.synchronize(self.device)
        return float(out.item())

    # --- reverse ----------------------------------------------------------
    def _key(self, sim):
        return (tuple(int(sim.L.capacity[k]) for k in range(2)), int(sim.L.ncent), int(sim.L.nnode),
                sim.real, self.nsp)

    def _packed_size(self):
        """Ions a packed state of each species can hold: at most the ions of
        its segment's checkpoint plus every id the segment handed out."""
        starts = sorted(self.checkpoints)
        n = [0] * self.nsp
        for i, s0 in enumerate(starts):
            ck = self.checkpoints[s0]
            nid1 = self.checkpoints[starts[i + 1]].next_id if i + 1 < len(starts) else self.nid
            for k in range(self.nsp):
                n[k] = max(n[k], ck.counts[k] + (nid1 - ck.next_id))
        return n

    def _buffers(self):
        """The tape (packed states and their fields), the working bins, the
        bin record, the adjoint buffers and the parking scratch of this run,
        allocated by the first reverse pass and reused while they fit."""
        sim = self.sim
        K = self.K_run
        n = self._packed_size()
        b = self._bufs
        if (b is not None and b["key"] == self._key(sim) and len(b["fields"]) >= K
                and all(b["n"][k] >= n[k] for k in range(self.nsp)) and b["nid"] >= self.nid
                and (b["work"] is not None) == self.own_bins
                and (b["fields"][0].stages is not None) == self.keep_stages
                and (b["fields"][0].fluid is not None) == self.keep_fluid):
            return b
        self._bufs = b = None
        dim = int(self.p["dim"])
        dev = self.device
        keep = []
        lam = F.FsAdjoint()
        for k in range(self.nsp):
            lam.capacity[k] = n[k]
            for buf in range(2):
                for d in range(3):
                    vv = torch.empty(max(n[k], 1), dtype=sim.real, device=dev)
                    lam.v[k][buf][d] = vv.data_ptr()
                    keep.append(vv)
                    if d < dim:
                        xv = torch.empty(max(n[k], 1), dtype=sim.real, device=dev)
                        lam.x[k][buf][d] = xv.data_ptr()
                        keep.append(xv)
        lB = torch.empty(3, int(sim.L.ncent), dtype=torch.float64, device=dev)
        lE = torch.empty(6, int(sim.L.nnode), dtype=torch.float64, device=dev)
        lam.lB, lam.lE = lB.data_ptr(), lE.data_ptr()
        rec = F.FsRecord()
        for k in range(self.nsp):
            cap = int(sim.L.capacity[k])
            t = torch.empty(cap, dtype=torch.int32, device=dev)
            rec.dst[k], rec.capacity[k] = t.data_ptr(), cap
            keep.append(t)
        nid = self.nid + self.nid // 8 + 4096
        scratch = torch.empty(self.nsp * (dim + 3) * nid, dtype=sim.real, device=dev)
        fields = [_Fields(sim, self.nsp, self._E, stages=self.keep_stages, fluid=self.keep_fluid) for _ in range(K)]
        packed = [_Packed(sim, self.nsp, n, self._status) for _ in range(K + 1)]
        nbytes = _fixed_bytes(sim, self.nsp, n) + K * (_fields_bytes(sim, self.nsp, self.keep_stages, self.keep_fluid)
                                                       + _Packed.bytes(sim, self.nsp, n))
        work = [_Bins(sim, self.nsp, w, own=True) for w in range(2)] if self.own_bins else None
        if work is not None:
            nbytes += 2 * _Bins.bytes(sim, self.nsp)
        self._bufs = dict(key=self._key(sim), n=n, nid=nid, lam=lam, keep=keep, lB=lB, lE=lE, rec=rec,
                          scratch=scratch, fields=fields, packed=packed, work=work, bytes=nbytes)
        return self._bufs

    def backward(self) -> np.ndarray:
        """Gradient [dL/du_sh, dL/dalpha_cr, dL/dA_1 .. dL/dA_M] of the last
        forward pass.  Where memory is short the re-runs use the
        simulation's particle buffers (`own_bins` False), so afterwards
        `self.sim` holds its final fields but not its final particles (a
        later backward is unaffected)."""
        sim = self.sim
        lib, stream = sim.lib, sim.stream
        bufs = self._buffers()
        lam, rec, P = bufs["lam"], bufs["rec"], bufs["packed"]
        lam.cur = 0
        self.lB, self.lE = bufs["lB"], bufs["lE"]
        # the re-runs step between two bin buffers: their own, or the
        # simulation's
        work = bufs["work"] or [_Bins(sim, self.nsp, 0), _Bins(sim, self.nsp, 1)]
        grads = torch.empty(2 + int(self.p["n_modes"]), dtype=torch.float64, device=self.device)
        gptr = C.c_void_p(grads.data_ptr())
        scratch = C.c_void_p(bufs["scratch"].data_ptr())
        nid = bufs["nid"]
        # zero the particle adjoints, lE and grads; seed lB = dL/dB at the final state
        sim._check(lib.fs_adjoint_seed(sim.h, C.byref(sim.f), C.byref(lam), gptr, stream))
        K = self.K_run
        parked = False
        for s0 in sorted(self.checkpoints, reverse=True):
            s1 = min(s0 + K, self.nsteps)
            ck = self.checkpoints[s0]
            sim.set_clock(ck.next_id)
            flds = [ck.fields] + bufs["fields"]
            sim._check(lib.fs_tape_unpack(sim.h, C.byref(ck.packed.s), work[0].sp(sim), stream))
            # each state's tile offsets, then its ions as the recorded step
            # from it reads them (the segment's last state has no such step)
            sim._check(lib.fs_tape_pack(sim.h, work[0].sp(sim), C.byref(P[0].s), None, None, None, 0, stream))
            pre, id0 = work[0], []
            for j, n in enumerate(range(s0, s1)):
                post = work[(j + 1) % 2]
                _recorded_step(sim, n, pre, flds[j], post, flds[j + 1], rec, P[j])
                id0.append(int(rec.id0))
                last = F.FS_PACK_IONS if n + 1 == s1 else 0
                sim._check(lib.fs_tape_pack(sim.h, post.sp(sim), C.byref(P[j + 1].s), pre.sp(sim), C.byref(rec),
                                            C.byref(P[j].s), last, stream))
                pre = post
            m = s1 - s0
            if parked:
                # the adjoints of state s1 were parked by id from its
                # checkpoint's packing; the re-run packed the same ions in
                # another order
                sim._check(lib.fs_adjoint_unpark(sim.h, C.byref(P[m].s), C.byref(lam), scratch, nid, stream))
            for j in range(m - 1, -1, -1):
                rc = lib.fs_adjoint_step(sim.h, C.byref(P[j].s), C.byref(flds[j].f(sim)), C.byref(P[j + 1].s),
                                         C.byref(flds[j + 1].f(sim)), flds[j + 1].stages_ptr(),
                                         flds[j + 1].fluid_ptr(), id0[j], s0 + j,
                                         C.byref(lam), gptr, stream)
                sim._check(rc)
            if s0 == 0:
                sim._check(lib.fs_adjoint_init(sim.h, C.byref(P[0].s), C.byref(ck.fields.f(sim)), C.byref(lam),
                                               gptr, stream))
            else:
                sim._check(lib.fs_adjoint_park(sim.h, C.byref(P[0].s), C.byref(lam), scratch, nid, stream))
                parked = True
        torch.cuda.synchronize(self.device)
        status = int(self._status.item())
        if status == 1:
            raise RuntimeError("a packed tape state overflowed its size: the gradient is invalid")
        if status != 0:
            raise RuntimeError("the reverse pass missed ions a step injected: the gradient is invalid")
        return grads.cpu().numpy()


class PrecursorEnergy(torch.autograd.Function):
    """L(u_sh, alpha_cr, amps) = precursor magnetic energy after N steps;
    ``backward`` runs the checkpointed reverse pass of the library."""

    @staticmethod
    def forward(ctx, u_sh, alpha_cr, amps, run: AdjointRun):
        loss = run.forward(float(u_sh), float(alpha_cr), amps.detach().cpu().numpy())
        ctx.run = run
        ctx.dtype = amps.dtype
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        gr = torch.as_tensor(ctx.run.backward(), dtype=torch.float64) * g
        return gr[0], gr[1], gr[2:].to(ctx.dtype), None


def precursor_energy(u_sh, alpha_cr, amps, run: AdjointRun):
    """Differentiable entry point: ``precursor_energy(u, a, A, run).backward()``."""
    return PrecursorEnergy.apply(u_sh, alpha_cr, amps, run)
