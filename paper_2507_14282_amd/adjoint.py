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
``fs_adjoint_seed``, ``fs_step_record``, ``fs_adjoint_step``,
``fs_adjoint_init``); this module owns the buffers and
the schedule: a forward pass that keeps a checkpoint every K steps, and a
reverse pass that re-runs each K-step segment from its checkpoint with
recording and walks it backwards.  Particle adjoints are laid out like the
particle buffers (one entry per bin slot, two buffers that the reverse steps
ping-pong); each recorded step keeps where it put every ion, which is all
the reverse step needs to carry an ion's adjoint from its slot after the
step to its slot before it.  The tape, the records and the adjoint buffers
are allocated once and reused by every later reverse pass of the run.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import fshybrid as F


class _State:
    """One particle/field state held in tensors of its own: per species the
    particle buffer and its tile counts, B, E, the gather grid, the moment
    grids and the id counter.  Either a copy of a simulation's current state
    (checkpoints) or an empty slot a recorded step writes into directly."""

    def __init__(self, sim: F.Simulation, nsp: int, copy: bool = True):
        def take(t):
            return t.clone() if copy else torch.empty_like(t)
        self.buf, self.cnt = [], []
        for k in range(nsp):
            cur = int(sim.sp[k].cur)
            self.buf.append(take(sim.bufs[k][cur]))
            self.cnt.append(take(sim.cnts[k][cur]))
        self.B = take(sim.B)
        self.E = take(sim.E)
        self.gather = take(sim.gather)
        self.mom = [take(m) for m in sim.mom[:nsp]]
        self.next_id = sim.next_id if copy else -1

    def particles(self, sim: F.Simulation):
        """fs_particles structs pointing at this state's buffers."""
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

    def fields(self, sim: F.Simulation) -> F.FsFields:
        f = F.FsFields()
        f.B, f.E, f.gather = self.B.data_ptr(), self.E.data_ptr(), self.gather.data_ptr()
        f.mom[0] = self.mom[0].data_ptr()
        f.mom[1] = self.mom[1].data_ptr() if len(self.mom) > 1 else None
        return f


def _recorded_step(sim: F.Simulation, n: int, a: _State, b: _State, rec: F.FsRecord):
    """Step n from state a into state b without copying particles: the
    step reads a's buffers and writes b's (the field update works in place,
    so B and the gather grid of a are first copied into b)."""
    b.B.copy_(a.B)
    b.gather.copy_(a.gather)
    b.E.copy_(a.E)
    sp = a.particles(sim)
    for k in range(len(a.buf)):
        sp[k].buf[1] = b.buf[k].data_ptr()
        sp[k].tile_count[1] = b.cnt[k].data_ptr()
    f = b.fields(sim)
    rc = sim.lib.fs_step_record(sim.h, sp, C.byref(f), int(n), C.byref(rec), None, sim.stream)
    sim._check(rc)
    b.next_id = sim.next_id


def checkpoint_interval(nsteps: int, K: int, state_bytes: int, free_bytes: int, share: float = 0.8) -> int:
    """Checkpoint interval for a reverse pass that must fit in memory.

    The forward keeps ceil(nsteps / k) checkpoints and the reverse a tape of
    k states, each state_bytes large.  Returns the largest k <= K for which
    (ceil(nsteps / k) + k) states fit in `share` of free_bytes.  Raises
    MemoryError if no interval fits.  The gradient does not depend on k."""
    nsteps, K = max(1, int(nsteps)), max(1, int(K))
    budget = share * float(free_bytes)
    for k in range(min(K, nsteps), 0, -1):
        if (-(-nsteps // k) + k) * float(state_bytes) <= budget:
            return k
    raise MemoryError(f"a reverse pass over {nsteps} steps needs at least "
                      f"{2 * (nsteps ** 0.5) * state_bytes / 1e9:.1f} GB of checkpoints and tape "
                      f"({state_bytes / 1e9:.2f} GB per state), {free_bytes / 1e9:.1f} GB are free")


def _state_bytes(sim: F.Simulation, nsp: int) -> int:
    """Bytes of one checkpoint / tape state of this simulation, with the
    step record a tape state carries (4 bytes per bin slot)."""
    t = [sim.B, sim.E, sim.gather] + list(sim.mom[:nsp])
    for k in range(nsp):
        cur = int(sim.sp[k].cur)
        t += [sim.bufs[k][cur], sim.cnts[k][cur]]
    rec = sum(4 * int(sim.L.capacity[k]) for k in range(nsp))
    return int(sum(x.numel() * x.element_size() for x in t)) + rec


def _lambda_bytes(sim: F.Simulation, nsp: int, dim: int) -> int:
    """Bytes of the two particle adjoint buffers and the grid adjoints."""
    rb = torch.finfo(sim.real).bits // 8
    part = sum(2 * (dim + 3) * rb * int(sim.L.capacity[k]) for k in range(nsp))
    return part + 8 * (3 * int(sim.L.ncent) + 6 * int(sim.L.nnode))


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
        # device plus what the allocator holds unused
        free, _ = torch.cuda.mem_get_info(self.device)
        free += torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        if self._bufs is not None and self._bufs["key"] == self._key(sim):
            free += self._bufs["bytes"]          # reused, already counted out of free
        else:
            self._bufs = None
            free -= _lambda_bytes(sim, self.nsp, int(p["dim"]))
        self.K_run = checkpoint_interval(self.nsteps, self.K, _state_bytes(sim, self.nsp), free)
        for n in range(self.nsteps):
            if n % self.K_run == 0:
                self.checkpoints[n] = _State(sim, self.nsp)
            sim.step(n, stats=False)
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

    def _buffers(self):
        """The tape states, step records and adjoint buffers of this run,
        allocated by the first reverse pass and reused afterwards."""
        sim = self.sim
        K = self.K_run
        b = self._bufs
        if b is not None and b["key"] == self._key(sim) and len(b["slots"]) >= K:
            return b
        dim = int(self.p["dim"])
        keep = []
        lam = F.FsAdjoint()
        for k in range(self.nsp):
            cap = int(sim.L.capacity[k])
            lam.capacity[k] = cap
            for buf in range(2):
                for d in range(3):
                    vv = torch.empty(cap, dtype=sim.real, device=self.device)
                    lam.v[k][buf][d] = vv.data_ptr()
                    keep.append(vv)
                    if d < dim:
                        xv = torch.empty(cap, dtype=sim.real, device=self.device)
                        lam.x[k][buf][d] = xv.data_ptr()
                        keep.append(xv)
        lB = torch.empty(3, int(sim.L.ncent), dtype=torch.float64, device=self.device)
        lE = torch.empty(6, int(sim.L.nnode), dtype=torch.float64, device=self.device)
        lam.lB, lam.lE = lB.data_ptr(), lE.data_ptr()
        recs, dsts = [], []
        for _ in range(K):
            rec = F.FsRecord()
            for k in range(self.nsp):
                cap = int(sim.L.capacity[k])
                t = torch.empty(cap, dtype=torch.int32, device=self.device)
                rec.dst[k], rec.capacity[k] = t.data_ptr(), cap
                dsts.append(t)
            recs.append(rec)
        slots = [_State(sim, self.nsp, copy=False) for _ in range(K)]
        nbytes = _lambda_bytes(sim, self.nsp, dim) + K * _state_bytes(sim, self.nsp)
        self._bufs = dict(key=self._key(sim), lam=lam, keep=keep, lB=lB, lE=lE, recs=recs, dsts=dsts, slots=slots,
                          bytes=nbytes, scratch=None)
        return self._bufs

    def _scratch(self, bufs):
        """Id-indexed scratch of the relayout between a checkpoint and its
        re-run ((dim + 3) reals per id), grown when a run hands out more ids."""
        need = (int(self.p["dim"]) + 3) * self.nid
        if bufs["scratch"] is None or bufs["scratch"].numel() < need:
            bufs["scratch"] = torch.empty(need + need // 8, dtype=self.sim.real, device=self.device)
        return bufs["scratch"]

    def backward(self) -> np.ndarray:
        """Gradient [dL/du_sh, dL/dalpha_cr, dL/dA_1 .. dL/dA_M] of the last
        forward pass."""
        sim = self.sim
        lib, stream = sim.lib, sim.stream
        bufs = self._buffers()
        lam = bufs["lam"]
        lam.cur = 0
        self.lB, self.lE = bufs["lB"], bufs["lE"]
        grads = torch.empty(2 + int(self.p["n_modes"]), dtype=torch.float64, device=self.device)
        gptr = C.c_void_p(grads.data_ptr())
        # zero the particle adjoints, lE and grads; seed lB = dL/dB at the final state
        sim._check(lib.fs_adjoint_seed(sim.h, C.byref(sim.f), C.byref(lam), gptr, stream))
        K = self.K_run
        slots, recs = bufs["slots"], bufs["recs"]
        scratch = self._scratch(bufs)
        later = None     # checkpoint that started the segment walked back last
        for s0 in sorted(self.checkpoints, reverse=True):
            s1 = min(s0 + K, self.nsteps)
            ck = self.checkpoints[s0]
            sim.set_clock(ck.next_id)
            tape = [ck]
            for j, n in enumerate(range(s0, s1)):
                _recorded_step(sim, n, tape[j], slots[j], recs[j])
                tape.append(slots[j])
            if later is not None:
                # the adjoints of state s1 sit in the slots of its checkpoint;
                # the re-run placed the same ions elsewhere
                rc = lib.fs_adjoint_relayout(sim.h, later.particles(sim), tape[-1].particles(sim), C.byref(lam),
                                             C.c_void_p(scratch.data_ptr()), int(self.nid), stream)
                sim._check(rc)
            later = ck
            for j in range(s1 - s0 - 1, -1, -1):
                a, b = tape[j], tape[j + 1]
                f_n, f_n1 = a.fields(sim), b.fields(sim)
                rc = lib.fs_adjoint_step(sim.h, a.particles(sim), C.byref(f_n), b.particles(sim), C.byref(f_n1),
                                         C.byref(recs[j]), s0 + j, C.byref(lam), gptr, stream)
                sim._check(rc)
            if s0 == 0:
                a = tape[0]
                f0 = a.fields(sim)
                rc = lib.fs_adjoint_init(sim.h, a.particles(sim), C.byref(f0), C.byref(lam), gptr, stream)
                sim._check(rc)
            del tape
        torch.cuda.synchronize(self.device)
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
