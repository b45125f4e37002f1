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
recording and walks it backwards.  Particle adjoints are indexed by particle
id, so a re-run segment may place ions in other bin slots than the first
run did.
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
    """Bytes of one checkpoint / tape state of this simulation."""
    t = [sim.B, sim.E, sim.gather] + list(sim.mom[:nsp])
    for k in range(nsp):
        cur = int(sim.sp[k].cur)
        t += [sim.bufs[k][cur], sim.cnts[k][cur]]
    return int(sum(x.numel() * x.element_size() for x in t))


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

    # --- forward ----------------------------------------------------------
    def forward(self, u_sh: float, alpha_cr: float, amps) -> float:
        p = dict(self.p, u_sh=float(u_sh), alpha_cr=float(alpha_cr))
        self.p_run = p
        sim = F.Simulation(p, self.device)
        self.sim = sim
        self.nsp = 2 if sim.has_cr else 1
        a = None
        if int(p["n_modes"]) > 0:
            a = torch.as_tensor(np.asarray(amps, dtype=np.float64), device=self.device)
        sim.init_plasma(a)
        # the interval actually used: the requested one, or less if the
        # checkpoints and the tape would not fit in the device's free memory
        free, _ = torch.cuda.mem_get_info(self.device)
        self.K_run = checkpoint_interval(self.nsteps, self.K, _state_bytes(sim, self.nsp), free)
        self.checkpoints = {}
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
    def _alloc_lambda(self):
        sim = self.sim
        dim = int(self.p["dim"])
        nid = max(self.nid, 1)
        lam = F.FsAdjoint()
        self._lam_keep = []
        # buffers only: fs_adjoint_seed fills them
        for d in range(3):
            vv = torch.empty(nid, dtype=sim.real, device=self.device)
            lam.v[d] = vv.data_ptr()
            self._lam_keep.append(vv)
            if d < dim:
                xv = torch.empty(nid, dtype=sim.real, device=self.device)
                lam.x[d] = xv.data_ptr()
                self._lam_keep.append(xv)
            else:
                lam.x[d] = None
        lam.nid = nid
        self.lB = torch.empty(3, int(sim.L.ncent), dtype=torch.float64, device=self.device)
        self.lE = torch.empty(6, int(sim.L.nnode), dtype=torch.float64, device=self.device)
        lam.lB, lam.lE = self.lB.data_ptr(), self.lE.data_ptr()
        self.lam = lam

    def backward(self) -> np.ndarray:
        """Gradient [dL/du_sh, dL/dalpha_cr, dL/dA_1 .. dL/dA_M] of the last
        forward pass."""
        sim = self.sim
        lib, stream = sim.lib, sim.stream
        self._alloc_lambda()
        grads = torch.empty(2 + int(self.p["n_modes"]), dtype=torch.float64, device=self.device)
        gptr = C.c_void_p(grads.data_ptr())
        # zero every adjoint and seed lB = dL/dB at the final state
        sim._check(lib.fs_adjoint_seed(sim.h, C.byref(sim.f), C.byref(self.lam), gptr, stream))
        K = self.K_run
        refl = [torch.empty(self.lam.nid, dtype=torch.uint8, device=self.device) for _ in range(K)]   # cleared by each recorded step
        slots = [_State(sim, self.nsp, copy=False) for _ in range(K)]
        for s0 in sorted(self.checkpoints, reverse=True):
            s1 = min(s0 + K, self.nsteps)
            ck = self.checkpoints[s0]
            sim.set_clock(ck.next_id)
            tape, recs = [ck], []
            for j, n in enumerate(range(s0, s1)):
                rec = F.FsRecord()
                rec.refl, rec.nid = refl[j].data_ptr(), self.lam.nid
                _recorded_step(sim, n, tape[j], slots[j], rec)
                tape.append(slots[j])
                recs.append(rec)
            for j in range(s1 - s0 - 1, -1, -1):
                a, b = tape[j], tape[j + 1]
                f_n, f_n1 = a.fields(sim), b.fields(sim)
                rc = lib.fs_adjoint_step(sim.h, a.particles(sim), C.byref(f_n), b.particles(sim), C.byref(f_n1),
                                         C.byref(recs[j]), s0 + j, C.byref(self.lam), gptr, stream)
                sim._check(rc)
            if s0 == 0:
                a = tape[0]
                f0 = a.fields(sim)
                rc = lib.fs_adjoint_init(sim.h, a.particles(sim), C.byref(f0), C.byref(self.lam), gptr, stream)
                sim._check(rc)
            del tape, recs
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
