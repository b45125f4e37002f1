#!/usr/bin/env python3
"""Benchmark of the faux-shock hybrid step on one MI355X.

Workload: the 3D3V FP32 faux-shock box, 1024 x 192 x 192 cells of 1 d_i,
8 thermal ions per cell (3.02e8 ions), M_A = 20 (u_sh = 20 v_A), beta = 1,
theta_Bn = 45 deg, y/z periodic, FS wall at x = L acting on the thermal
ions, int64 fixed-point moments, FP64 Ohm/Faraday field update.  Synthetic
Philox-seeded initial load, no external data.

A timed step is the whole step: push (gather + Boris + move + boundaries +
fused deposit), FS wall, injection and the FP64 field update.  `value` is
ion particle-updates per second over that whole step with everything
resident in HBM.  The line also carries the push-kernel roofline (live HIP
event timing on the library's stream) and the CPU oracle timed on a bounded
slab of the same workload on this host.
"""

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def push_bytes_dim(n_ions, L, dim, nsp, rb=4, with_id=False):
    """Algorithmic HBM bytes of one step's push launches with rb-byte reals
    (4: FP32, 8: FP64), counted as the method needs them: every ion's state
    read and written once (int32 cell, D offsets, 3 velocities: 28 B each
    way in 3D FP32), and per species launch the gather grid read once (6
    reals per node) and the int64 moments written once (32 B per node).
    with_id adds the uint32 particle id the bins carry along with each ion
    (4 B each way), which the method itself does not move."""
    ion = 2 * (4 + rb * (dim + 3)) + (8 if with_id else 0)
    return n_ions * ion + nsp * (int(L.nnode) * 6 * rb + int(L.ndep) * 32)


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_throughput(name, steps, warmup, **overrides):
    """Whole-step and push+deposit throughput of one preset, with the push
    roofline as for the 3D box (used for the 1D and 2D boxes, and for the
    relativistic push)."""
    import torch
    from paper_2507_14282_amd import fshybrid as F
    from paper_2507_14282_amd import workloads as W
    progress(f"workload {name} {overrides} ({warmup} + {steps} steps)")
    p = W.preset(name, **overrides)
    sim = F.Simulation(p, "cuda:0")
    sim.init_plasma()
    for s in range(warmup):
        sim.step(s, stats=False)
    torch.cuda.synchronize()
    nsp = 2 if sim.has_cr else 1
    count = lambda: sum(sim.count(k) for k in range(nsp))
    n0 = count()
    sim.timing(True)
    t0 = time.perf_counter()
    for k in range(steps):
        sim.step(warmup + k, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, nrec = sim.timing_read()
    n1 = count()
    st = sim.step(warmup + steps, stats=True)
    nav = 0.5 * (n0 + n1)
    push_ms = ms[0] / max(nrec[0], 1)
    dim = int(p["dim"])
    alg = push_bytes_dim(nav, sim.L, dim, nsp)
    ach = alg / (push_ms * 1e-3) / 1e9
    ach_id = push_bytes_dim(nav, sim.L, dim, nsp, with_id=True) / (push_ms * 1e-3) / 1e9
    out = {
        "workload": f"{dim}D3V FP32 {p['nx']}x{p['ny']}x{p['nz']} cells dx={p['dx']} d_i, {p['ppc']} ppc"
                    + (f" + CRs n_cr={p['n_cr']:g}" if sim.has_cr else "") + f", {p['shape']}, M_A={p['u_sh']:g}"
                    + (f", relativistic c/v_A={p['c_light']:g}" if p.get("c_light", 0) > 0 else "")
                    + (", time-centred coupling" if p.get("coupling", 1) == 2 else "")
                    + (", reflecting wall" + (" (conducting)" if p.get("wall_field", 0) else "")
                       if p["wall_th"] == "specular" else "")
                    + (f", prescribed wall (f0={p['ret_f0']:g}, gain={p['gain']:g}, kappa={p['kappa']:g}, "
                       f"r_dot={p['r_dot']:g}, loss-cone depletion={p.get('lc_depletion', 0.0):g})"
                       if p.get("wall_model", 0) else ""),
        "ions": int(nav), "steps": steps, "warmup": warmup,
        "ms_per_step": (t1 - t0) / steps * 1e3,
        "pu_per_s": nav * steps / (t1 - t0),
        "push_deposit_ms": push_ms,
        "wall_ms": ms[1] / max(nrec[1], 1),
        "field_ms": ms[3] / max(nrec[3], 1),
        "push_alg_bytes_per_step": alg, "push_GBs": ach, "push_frac_of_hbm_peak": ach / HBM_PEAK_GBS,
        "push_frac_with_id": ach_id / HBM_PEAK_GBS,
        "final_step_flags": st["flags"],
    }
    del sim
    torch.cuda.empty_cache()
    return out


def push_bytes(np_live, L, with_id=False):
    """Algorithmic HBM bytes of one launch of the fused 3D FP32 push kernel:
    56 B per ion (28 B of state in and out), 24 B of E/Bbar read and 32 B of
    int64 moments written per node, i.e. 63 B per particle-update at 8 ions
    per cell; with_id adds the 8 B of the id."""
    return push_bytes_dim(np_live, L, 3, 1, 4, with_id)


def traffic_from_profiles(kernel_hash):
    """HBM bytes per push launch measured with rocprofv3 counters, if the
    committed measurement was taken on the kernel source as it is now."""
    path = os.path.join(ROOT, "profiles", "push3d_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_hash:
        return None
    return d.get("bytes_per_launch")


def copy_calibration():
    """A plain device copy of 1 GiB, three times: what FETCH_SIZE and
    WRITE_SIZE read for a kernel of known traffic."""
    import torch
    n = 256 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty(n, dtype=torch.float32, device="cuda:0")
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


def copy_bandwidth():
    """Achieved HBM bandwidth of a plain 2 GiB device-to-device copy (read +
    write bytes over the event-timed duration), the practical ceiling a
    streaming kernel can reach on this GPU."""
    import torch
    n = 512 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def _counter(dirname, counter, name_part):
    """Per-dispatch values of one counter for kernels whose name contains
    `name_part`, from a rocprofv3 --output-format csv directory."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(dirname, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
                out[int(r["Dispatch_Id"])] = out.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    return [out[k] for k in sorted(out)]


def write_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, command):
    """HBM bytes per launch of the fused 3D push kernel from two counter runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the 1 GiB copy; written with the hash of the kernel
    source it was measured on."""
    kern = "k_push<float, 3, 1, true, false, false, false, false>"
    f = _counter(fetch_dir, "FETCH_SIZE", kern)
    w = _counter(write_dir, "WRITE_SIZE", kern)
    cf = _counter(copy_fetch_dir, "FETCH_SIZE", "copy")
    cw = _counter(copy_write_dir, "WRITE_SIZE", "copy")
    if not (f and w and cf and cw):
        raise SystemExit("missing counter values")
    gib = float(1 << 30)
    kf = gib / (max(cf) * 1024.0)   # bytes per counted byte, from the copy's reads
    kw = gib / (max(cw) * 1024.0)
    fetch = sum(f) / len(f) * 1024.0 * kf
    write = sum(w) / len(w) * 1024.0 * kw
    d = {"kernel": kern, "workload": "cfg4 3D box 1024x192x192, 8 ppc",
         "dispatches": [len(f), len(w)],
         "fetch_kib_per_dispatch": sum(f) / len(f), "write_kib_per_dispatch": sum(w) / len(w),
         "copy_fetch_kib_per_gib": max(cf), "copy_write_kib_per_gib": max(cw),
         "fetch_scale": kf, "write_scale": kw,
         "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
         "bytes_per_launch": fetch + write,
         "kernel_source_sha256": kernel_source_hash(), "command": command}
    path = os.path.join(ROOT, "profiles", "push3d_traffic.json")
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d))


# Peak LDS atomic rate used as the roofline of the deposit: 32 banks of 4 B
# per CU, so at most 16 lanes of 64-bit atomics per clock per CU, over 256
# CUs at 2.4 GHz.
LDS_U64_ATOMIC_PEAK = 16 * 256 * 2.4e9
ATOMIC_COUNTERS = ("SQ_INSTS_LDS_ATOMIC", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_ADDR_CONFLICT",
                   "SQ_WAVES", "TCC_ATOMIC_sum", "TA_FLAT_ATOMIC_WAVEFRONTS_sum")


def write_atomics(pmc_dir, command):
    """Atomic counts per launch of the fused 3D push kernel from one rocprofv3
    --pmc run of ATOMIC_COUNTERS: LDS atomic wave-instructions (the deposit
    into the tile box), LDS bank / address conflict cycles, and L2 atomic
    requests (the flush of the box into the global moment grid and the
    deposits of ions outside the box)."""
    kern = "k_push<float, 3, 1, true, false, false, false, false>"
    d = {"kernel": kern, "workload": "cfg4 3D box 1024x192x192, 8 ppc", "counters": {}}
    for c in ATOMIC_COUNTERS:
        v = _counter(pmc_dir, c.replace("_sum", "") if c.endswith("_sum") else c, kern)
        if not v:
            v = _counter(pmc_dir, c, kern)
        if not v:
            raise SystemExit(f"missing counter {c}")
        d["counters"][c] = {"per_dispatch": sum(v) / len(v), "dispatches": len(v)}
    d["kernel_source_sha256"] = kernel_source_hash()
    d["command"] = command
    path = os.path.join(ROOT, "profiles", "push3d_atomics.json")
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d))


def atomics_from_profiles(kernel_hash):
    path = os.path.join(ROOT, "profiles", "push3d_atomics.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_hash:
        return None
    return {k: v["per_dispatch"] for k, v in d["counters"].items()}


def adjoint_timing(preset="cfg5", steps=400, K=20, **overrides):
    """Forward and checkpointed reverse pass of an adjoint workload: wall
    time of each pass and their ratio (the reverse pass includes re-running
    every K-step segment from its checkpoint), in steady state: the run's
    first forward and reverse pass allocate its checkpoints, tape, records
    and adjoint buffers, the second one is timed."""
    import numpy as np
    import torch
    from paper_2507_14282_amd import adjoint as A
    from paper_2507_14282_amd import workloads as W
    p = W.preset(preset, **overrides)
    amps = np.full(p["n_modes"], p["mode_amp"])
    # start from an empty allocator cache: blocks cached by the workloads
    # before (other sizes) would otherwise be freed and allocated again inside
    # the timed passes of a run that needs most of the memory
    gc.collect()
    torch.cuda.empty_cache()
    run = A.AdjointRun(p, steps, K=K)
    run.forward(p["u_sh"], p["alpha_cr"], amps)
    run.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = run.forward(p["u_sh"], p["alpha_cr"], amps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = run.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ny = f"x{p['ny']}" if p["dim"] >= 2 else ""
    nz = f"x{p['nz']}" if p["dim"] >= 3 else ""
    crs = f" + CRs (n_cr={p['n_cr']})" if p["n_cr"] > 0 else " (no CRs)"
    out = {
        "workload": f"{p['dim']}D3V adjoint box {p['nx']}{ny}{nz} cells dx={p['dx']} d_i, {p['ppc']} ppc{crs}, "
                    f"{p['n_modes']} Fourier modes, {steps} steps, checkpoint every {run.K_run}",
        "loss": "precursor sum(By^2+Bz^2) over x in [L/2, L]",
        "params": f"u_sh, alpha_cr, {p['n_modes']} amplitudes",
        "dtype": "f32 particles / f64 fields",
        "fwd_ms_per_step": (t1 - t0) / steps * 1e3,
        "adj_ms_per_step": (t2 - t1) / steps * 1e3,
        "adjoint_over_forward": (t2 - t1) / (t1 - t0),
        "loss_value": loss,
        "grad_u_sh": float(g[0]), "grad_alpha_cr": float(g[1]), "grad_amps_norm": float(np.linalg.norm(g[2:])),
    }
    return out


# The 2D adjoint workload: the 2D faux-shock box (8192 x 512 cells, 16 ppc,
# CRs) with 16 seeded Fourier modes, 40 steps at K = 20.
ADJOINT_2D = dict(preset="cfg3", steps=40, K=20, n_modes=16, mode_amp=1e-3)

# The 3D adjoint workload: the headline 3D box (1024 x 192 x 192 cells, 8 ppc,
# 3.0e8 ions) with 16 seeded Fourier modes, 20 steps; K = 10 requested, the
# interval that fits in memory is used (reported in the workload string).
ADJOINT_3D = dict(preset="cfg4", steps=20, K=10, n_modes=16, mode_amp=1e-3)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("fs_device.h", "fs_kernels.h"):
        with open(os.path.join(ROOT, "paper_2507_14282_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cpu_baseline(params, seconds):
    """The FP64 oracle on a 64 x 48 x 48 slab of the same workload (same ppc,
    flow, wall and field update), timed over whole steps for about `seconds`."""
    from oracle import oracle as O
    p = dict(params, nx=64, ny=48, nz=48)
    o = O.Oracle(p)
    o.init()
    done, pu, t0 = 0, 0, time.perf_counter()
    while True:
        n = o.count(0)
        o.step()
        pu += n
        done += 1
        el = time.perf_counter() - t0
        if done >= 2 and el >= seconds:
            break
    out = {"value": pu / el, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 oracle, whole steps, 64x48x48 slab at 8 ppc ({n} ions), {done} steps, {el:.1f} s",
           "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "threads_used": 1}}
    from paper_2507_14282_amd import workloads as W
    # context: the 1D FP64 parity box, and the oracle's own forward/adjoint
    # pair on the 1D adjoint workload (10 steps each)
    o = O.Oracle(W.preset("cfg1"))
    o.init()
    done, pu, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < 0.3 * seconds:
        pu += o.count(0)
        o.step()
        done += 1
    el = time.perf_counter() - t0
    p5 = W.preset("cfg5")
    t0 = time.perf_counter()
    O.forward_loss(p5, 10)
    t1 = time.perf_counter()
    O.adjoint(p5, 10)
    t2 = time.perf_counter()
    out["other"] = {
        "1D FP64 box 512 cells, 64 ppc": {"value": pu / el, "unit": "particle-updates/s", "steps": done},
        "adjoint workload, 10 steps": {"forward_s": t1 - t0, "forward_plus_adjoint_s": t2 - t1,
                                       "reverse_over_forward": (t2 - t1) / (t1 - t0) - 1.0},
    }
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cfg4")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale the HBM byte counters")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write profiles/push3d_traffic.json from four rocprofv3 counter directories")
    ap.add_argument("--traffic-command", default="", help="command line recorded with --write-traffic")
    ap.add_argument("--write-atomics", metavar="PMC_DIR",
                    help="write profiles/push3d_atomics.json from a rocprofv3 run of the atomic counters")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward measurement")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the 1D, 2D, relativistic, reflecting-wall and prescribed-wall workload lines")
    ap.add_argument("--adjoint-only", action="store_true", help="only the adjoint/forward measurement")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return 0
    if args.write_traffic:
        write_traffic(*args.write_traffic, command=args.traffic_command)
        return 0
    if args.write_atomics:
        write_atomics(args.write_atomics, command=args.traffic_command)
        return 0
    if args.gpus != 1:
        msg = (f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
               "(the multi-GPU x-slab decomposition is design only)")
        print(msg, file=sys.stderr)
        print(json.dumps({"error": msg, "n_gpus": args.gpus}))
        return 2

    import torch
    from paper_2507_14282_amd import fshybrid as F
    from paper_2507_14282_amd import workloads as W

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_timing(), "adjoint_2d": adjoint_timing(**ADJOINT_2D),
                          "adjoint_3d": adjoint_timing(**ADJOINT_3D)}))
        return 0

    p = W.preset(args.workload)
    progress(f"{args.workload}: load, {args.warmup} warm-up + {args.steps} timed steps")
    sim = F.Simulation(p, "cuda:0")
    sim.init_plasma()
    for s in range(args.warmup):
        sim.step(s, stats=False)
    torch.cuda.synchronize()
    n0 = sim.count(0) + (sim.count(1) if sim.has_cr else 0)
    sim.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sim.step(args.warmup + k, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, nrec = sim.timing_read()
    n1 = sim.count(0) + (sim.count(1) if sim.has_cr else 0)
    st = sim.step(args.warmup + args.steps, stats=True)   # error flags of a final, untimed step
    elapsed = t1 - t0
    np_avg = 0.5 * (n0 + n1)
    value = np_avg * args.steps / elapsed
    push_ms = ms[0] / max(nrec[0], 1)
    region_ms = (ms[0] + ms[1] + ms[2]) / max(nrec[0], 1)
    dim = int(p["dim"])
    nsp = 2 if sim.has_cr else 1
    rb = int(sim.L.real_bytes)
    alg = push_bytes_dim(np_avg, sim.L, dim, nsp, rb)
    alg_id = push_bytes_dim(np_avg, sim.L, dim, nsp, rb, with_id=True)
    achieved = alg / (push_ms * 1e-3) / 1e9
    # the committed counters are of the 3D benchmark box's push kernel
    profiled = args.workload == "cfg4"
    traffic = traffic_from_profiles(kernel_source_hash()) if profiled else None
    pmc = atomics_from_profiles(kernel_source_hash()) if profiled else None
    # LDS atomics of the deposit: 4 moments at each of the 2^D (CIC) or 3^D
    # (TSC) corners per ion (8 x 4 for the 3D CIC box)
    corners = (3 if p["shape"] == "tsc" else 2) ** dim
    lds_ops = 4.0 * corners * np_avg
    atomics = {
        "lds_u64_lane_ops_per_launch": lds_ops,
        "lds_rate": lds_ops / (push_ms * 1e-3), "lds_peak": LDS_U64_ATOMIC_PEAK, "unit": "lane-ops/s",
        "lds_frac": lds_ops / (push_ms * 1e-3) / LDS_U64_ATOMIC_PEAK,
        "pmc": None,
    }
    if pmc:
        atomics["pmc"] = {
            "lds_atomic_wave_instructions": pmc["SQ_INSTS_LDS_ATOMIC"],
            "lds_bank_conflict_cycles": pmc["SQ_LDS_BANK_CONFLICT"],
            "lds_addr_conflict_cycles": pmc["SQ_LDS_ADDR_CONFLICT"],
            "l2_atomic_requests": pmc["TCC_ATOMIC_sum"],
            "l2_atomic_rate": pmc["TCC_ATOMIC_sum"] / (push_ms * 1e-3),
        }
    del sim
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth()
    out = {
        "metric": "ion particle-updates/sec (push+deposit+FS wall) 3D at 1 GPU; adjoint/fwd time",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if int(p["precision"]) == 64 else "f32",
        "data": "synthetic (Philox-seeded drifting Maxwellian load, no external data)",
        "config": {
            "workload": f"{dim}D3V FP{int(p['precision'])} faux-shock box {p['nx']}x{p['ny']}x{p['nz']} cells dx={p['dx']} d_i, "
                        f"{p['ppc']} ppc, M_A={p['u_sh']:g}, beta={p['beta_i']:g}, theta_Bn={p['theta_deg']:g} deg",
            "ions": int(np_avg),
            "step": "push+wall+inject+deposit (FP32 particles, int64 moments) + FP64 SSP-RK3 field update",
            "parallelism": "single GPU",
        },
        "phases_ms_per_step": {
            "push_deposit": push_ms, "wall": ms[1] / max(nrec[1], 1), "inject": ms[2] / max(nrec[2], 1),
            "field": ms[3] / max(nrec[3], 1), "step_events": ms[4] / max(nrec[4], 1)},
        "push_deposit_wall_pu_per_s": np_avg / (region_ms * 1e-3),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"k_push<{'double' if int(p['precision']) == 64 else 'float'},{dim},{p['shape'].upper()},deposit>",
            "alg_bytes_per_launch": alg,
            "alg_bytes_per_particle_update": alg / np_avg,
            "avg_launch_ms": push_ms,
            # the same launch counting the uint32 id each ion carries
            "alg_bytes_per_launch_with_id": alg_id,
            "frac_with_id": alg_id / (push_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
        },
        "atomics": atomics,
        "final_step_flags": st["flags"],
    }
    if not args.no_other:
        out["other_workloads"] = {
            "1D cfg2": workload_throughput("cfg2", 100, 10),
            "2D cfg3": workload_throughput("cfg3", 50, 10),
            # the relativistic push at the paper's c / v_A = 1000 (Run A)
            "2D cfg3 relativistic": workload_throughput("cfg3", 50, 10, c_light=1000.0),
            "3D cfg4 relativistic": workload_throughput("cfg4", 30, 10, c_light=1000.0),
            # the reflecting-wall box of Run C's shape, timed after 2000 steps
            # (t = 10) so that the reflected beams and the shock are in it
            "2D rw2 reflecting wall": workload_throughput("rw2", 50, 2000),
            # the prescribed faux shock on the 3D box
            # the time-centred (second-order) ion-field coupling, on the 3D box
            # and on the 2D box with the paper's relativistic dHybridR push
            "3D cfg4 time-centred coupling": workload_throughput("cfg4", 30, 10, coupling=2),
            "2D cfg3 relativistic, time-centred coupling": workload_throughput("cfg3", 50, 10, c_light=1000.0,
                                                                               coupling=2),
            # with the loss cone of the oblique (45 deg) shock depleted
            "3D cfg4 prescribed wall": workload_throughput("cfg4", 30, 10, wall_model=1, ret_f0=0.8, ret_alpha=0.0,
                                                            gain=1.2, kappa=1.5, r_dot=0.1, lc_depletion=0.5),
        }
    if not args.no_adjoint:
        progress("adjoint workload")
        out["adjoint"] = adjoint_timing()
        progress("2D adjoint workload")
        out["adjoint_2d"] = adjoint_timing(**ADJOINT_2D)
        progress("3D adjoint workload")
        out["adjoint_3d"] = adjoint_timing(**ADJOINT_3D)
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
