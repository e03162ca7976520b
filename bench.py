#!/usr/bin/env python3
"""Throughput of the full USP-FPM step on one MI355X.

Workload: Mach-10 N2 over a cylinder (half body), 600 x 300 cells of 1 mm,
~36.1M particles at start (FP32 particle state, FP64 cell accumulators),
VHS gas with Parker / Millikan-White collision numbers, dt = 1.25e-7 s.
A step is bin -> moments -> cell state -> the fused particle phase
(collide + conserve + advect with injection, one pass), each a call of the
C ABI on torch's current stream so HIP events bracket every phase.  `value` is particle-steps/s over exactly
--steps timed steps (inputs resident in HBM), after --warmup steps.

Also reported: the HBM roofline of the dominant kernel (algorithmic bytes
per launch / its average event-timed duration) and the CPU oracle timed on
the host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# instruction per SIMD every 4 cycles (16 lanes per cycle)
VALU_PEAK = 256 * 4 * 2.4e9 / 4
COUNTERS_GLOB = os.path.join(ROOT, "profiles", "counters_*.md")
METRIC = "particle-steps/s (full USP-FPM step) + HBM GB/s; adjoint/forward time ratio"
PHASES = ("bin", "moments", "reconstruct", "update")
# the kernel that dominates each phase (bin is a pipeline of small kernels
# around two passes; update adds two tiny tile-index kernels before and the
# injection kernels after k_update)
PHASE_KERNEL = {"update": "k_update", "moments": "k_moments", "reconstruct": "k_reconstruct"}


def algorithmic_bytes(phase, n, M):
    """Bytes a phase must move at minimum for n particles and M cells (FP32
    state: x, y, cx, cy, cz, erot 4 B each, vib 1 B, cell 4 B, pid 4 B;
    cell-state plane 8 B per field)."""
    per_particle = {
        # the bin only records the new order: read cell, write the input
        # index and the new cell of every slot
        "bin": 4 + 4 + 4,
        # read the slot's input index, then cx, cy, cz, erot, vib through it
        "moments": 4 + 17,
        "reconstruct": 0,
        # read the input index and x, y, cx, cy, cz, erot, vib, pid through
        # it plus the new cell; write every array of the new state
        "update": 4 + 33 + 33,
    }[phase]
    # per cell: offsets 8; moments 21 planes; cell state reads 21 planes and
    # writes 35 planes + a 128-byte record; update reads the record and 9
    # conservation planes
    per_cell = {"bin": 4 + 8, "moments": 21 * 8 + 8, "reconstruct": (21 + 35) * 8 + 128,
                "update": 128 + 9 * 8 + 8}[phase]
    return per_particle * n + per_cell * M


def stored_counters(kernel):
    """Per-launch PMC figures of `kernel` from the committed profile summary,
    or None when they were taken on other sources or flags than the library
    being run (fingerprint mismatch)."""
    import glob
    from paper_2508_05642_amd import build
    lines = []
    for f in sorted(glob.glob(COUNTERS_GLOB)):
        with open(f) as fh:
            lines += fh.read().splitlines()
    fp = build.fingerprint()
    for ln in lines:
        if not ln.startswith("counters:"):
            continue
        kv = dict(t.split("=", 1) for t in ln.split()[1:])
        if kv.get("kernel") == kernel and kv.get("fingerprint") == fp:
            return {k: (float(v) if k not in ("kernel", "fingerprint") else v) for k, v in kv.items()}
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _snapshot(st):
    keep = [{k: v.clone() for k, v in B.items() if k != "struct" and v is not None} for B in st.bufs]
    extra = {k: getattr(st, k).clone() for k in ("offsets", "counters")}
    for k in ("fields", "surf"):
        if getattr(st, k, None) is not None:
            extra[k] = getattr(st, k).clone()
    return keep, extra, st.cur, st.binned, [B["struct"] for B in st.bufs]


def _restore(st, snap):
    keep, extra, cur, binned, structs = snap
    for B, S, t in zip(st.bufs, keep, structs):
        for k, v in S.items():
            B[k].copy_(v)
        B["struct"] = t
    for k, v in extra.items():
        getattr(st, k).copy_(v)
    st.cur, st.binned = cur, binned


def _copy_peak(torch, dev):
    """Read + write rate of a plain 1 GiB device copy (best of 3), GB/s."""
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return round(2 * (1 << 30) / (best * 1e-3) / 1e9, 1)


def run_gpu(args):
    import numpy as np
    import torch

    import usp_workloads as W
    from paper_2508_05642_amd import usp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = W.cylinder(scale=args.scale, f32=True)
    if args.scheme == "fpm":
        import dataclasses
        prob.gas = dataclasses.replace(prob.gas, scheme=W.SCHEME_FPM)
    parts = W.particles_for(prob)
    n0 = parts["n"]
    log(f"workload ready: {n0} particles, {prob.grid.ncells} cells")
    st = usp.DeviceState(prob, parts, device="cuda:0")
    if args.sample:
        # the sampling phase of a run: field sums every step, wall sums at
        # every diffuse re-emission (cylinder in 1-degree elements)
        st.enable_sampling(args.sample)
    M = prob.grid.ncells
    step = 0

    def one_step(s, ev=None, nlog=None, k=None):
        if ev: ev[0].record()
        st.bin(gather=True)
        if nlog is not None:
            nlog[k].copy_(st.bufs[1 - st.cur]["count"][0])
        if ev: ev[1].record()
        st.do_moments()
        if args.sample:
            st.sample_fields()
        if ev: ev[2].record()
        st.do_reconstruct()
        if ev: ev[3].record()
        st.update(s)
        if ev: ev[4].record()

    for _ in range(args.warmup):
        one_step(step)
        step += 1
    torch.cuda.synchronize()
    log(f"{args.warmup} warmup steps done")
    K = args.steps
    step0 = step
    snap = _snapshot(st)
    # eager pass: per-phase times (events between the phases)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(PHASES) + 1)] for _ in range(K)]
    nlog = torch.zeros(K, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        one_step(step0 + k, evs[k], nlog, k)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    # timed pass: the same K steps from the same state, captured in one HIP
    # graph and replayed once
    _restore(st, snap)
    nlog_g = torch.zeros(K, dtype=torch.int64, device=dev)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for k in range(K):
            one_step(step0 + k, None, nlog_g, k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_graph = e0.elapsed_time(e1)
    ns = nlog_g.cpu().numpy()
    if not np.array_equal(ns, nlog.cpu().numpy()):
        raise RuntimeError("graph replay and eager pass disagree on the particle counts")
    log(f"eager {wall_eager / K * 1e3:.4f} ms/step, graph {wall / K * 1e3:.4f} ms/step")
    hbm_copy = _copy_peak(torch, dev)
    phase_ms = {ph: 0.0 for ph in PHASES}
    for k in range(K):
        for j, ph in enumerate(PHASES):
            phase_ms[ph] += evs[k][j].elapsed_time(evs[k][j + 1])
    phase_ms = {ph: v / K for ph, v in phase_ms.items()}
    total_ps = float(ns.sum())
    n_mean = float(ns.mean())
    dom = max(PHASE_KERNEL, key=lambda p: phase_ms[p])
    t_dom = phase_ms[dom] * 1e-3
    hbm = {"achieved": round(algorithmic_bytes(dom, n_mean, M) / t_dom / 1e9, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(algorithmic_bytes(dom, n_mean, M) / t_dom / 1e9 / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": int(algorithmic_bytes(dom, n_mean, M))}
    # the stored counters are those of the USP-FPM update kernel
    ctr = stored_counters(PHASE_KERNEL[dom]) if args.scheme == "usp" else None
    if ctr:
        # VALU wave-instructions per particle (PMC, same sources and flags,
        # same steps) x particles per launch / event-timed launch
        ach = ctr["valu_per_particle"] * n_mean / t_dom
        roof = {"bound": "alu", "kernel": PHASE_KERNEL[dom], "phase": dom,
                "achieved": round(ach / 1e9, 2), "peak": round(VALU_PEAK / 1e9, 1),
                "unit": "G VALU wave-instr/s", "frac": round(ach / VALU_PEAK, 4),
                "traffic": int(ctr["fetch_bytes"] + ctr["write_bytes"]),
                "valu_per_particle": ctr["valu_per_particle"], "avg_ms": round(phase_ms[dom], 4),
                "hbm": hbm}
    else:
        roof = dict(bound="hbm", kernel=PHASE_KERNEL[dom], phase=dom, traffic=None,
                    avg_ms=round(phase_ms[dom], 4), **hbm)
    step_bytes = sum(algorithmic_bytes(p, n_mean, M) for p in PHASES)
    cnt = st.cnt()
    res = dict(
        metric=METRIC, value=round(total_ps / wall, 1), unit="particle-steps/s", n_gpus=1,
        steps=K, warmup=args.warmup, ms_per_step=round(wall / K * 1e3, 4),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config={"workload": f"cylinder_mach10_{prob.grid.nx}x{prob.grid.ny}",
                "particles_start": int(n0), "particles_mean": int(n_mean), "cells": M,
                "state": "f32", "accumulation": "f64", "dt_s": prob.dt,
                "first_timed_step": args.warmup, "sampling": bool(args.sample),
                "scheme": args.scheme, "parallelism": "single-gpu"},
        launch="one HIP graph of the K steps (per-phase times from an eager pass over the same "
               "steps from the same state)",
        eager_ms_per_step=round(wall_eager / K * 1e3, 4),
        graph_event_ms=round(ms_graph, 3),
        phase_ms=phase_ms,
        step_algorithmic_gbs=round(step_bytes / (wall / K) / 1e9, 1),
        hbm_copy_gbs=hbm_copy,
        roofline=roof,
        counters={k: v for k, v in cnt.items() if v},
    )
    return res, prob, parts


def run_gpu_adjoint(args):
    """The differentiable Poiseuille case: Kn = 0.05, 100 cells x 500
    particles (50,000), FP64, K steps from the initial state.  Times a plain
    forward (usp_step), the checkpointed forward with output sampling, and
    the reverse pass (re-run with tapes + usp_adjoint_step), every 32 steps
    a checkpoint; then checks the gradient against central differences of
    the outputs (h = 1e-4 relative, common random numbers: same seed)."""
    import numpy as np
    import torch

    import usp_workloads as W
    from paper_2508_05642_amd import adjoint as ADJ, usp

    torch.cuda.set_device(0)
    prob = W.poiseuille(kn=0.05, cells=100, ppc=500, f32=False, seed=7)
    parts = W.particles_for(prob)
    n, K, seg = int(parts["n"]), args.steps, 32
    log(f"workload ready: {n} particles, {prob.grid.ncells} cells, {K} steps")
    warm = usp.DeviceState(prob, parts)
    for k in range(args.warmup):
        warm.step(k, 1)
    wa = ADJ.PathwiseAdjoint(prob, parts, min(K, 4), 2)
    wa.forward(0)
    wa.backward()
    torch.cuda.synchronize()
    del warm, wa

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    st = usp.DeviceState(prob, parts)

    def plain():
        for k in range(K):
            st.step(k, 1)
    _, t_plain = timed(plain)
    adj = ADJ.PathwiseAdjoint(prob, parts, K, seg)
    J, t_fwd = timed(lambda: adj.forward(0))
    G, t_bwd = timed(lambda: adj.backward())
    J, G = J.cpu().numpy(), G.cpu().numpy()
    log(f"plain forward {t_plain:.3f} s, forward with checkpoints {t_fwd:.3f} s, "
        f"reverse {t_bwd:.3f} s; J = {J}")
    th0 = np.array([prob.gas.Z_rot, prob.gas.omega, prob.gas.mu_ref])
    fd = np.full((2, 3), np.nan)
    for p in range(3 if not args.no_fd else 0):
        h = 1e-4 * th0[p]
        Js = []
        for sgn in (1, -1):
            th = th0.copy()
            th[p] += sgn * h
            a = ADJ.PathwiseAdjoint(ADJ.with_theta(prob, th), parts, K, seg)
            Js.append(a.forward(0).cpu().numpy())
            del a
        fd[:, p] = (Js[0] - Js[1]) / (2 * h)
        log(f"  {ADJ.PathwiseAdjoint.__name__} d/d{('Z_rot', 'omega', 'mu_ref')[p]}: "
            f"adjoint {G[:, p]}, central differences {fd[:, p]}")
    rel = np.abs(G - fd) / np.maximum(np.abs(fd), 1e-300)
    # short horizon: 8 steps, h = 1e-7 relative, where few discrete outcomes flip
    Ks = 8
    a = ADJ.PathwiseAdjoint(prob, parts, Ks, seg)
    a.forward(0)
    Gs = a.backward().cpu().numpy()
    fds = np.full((2, 3), np.nan)
    for p in range(3 if not args.no_fd else 0):
        Js = []
        for sgn in (1, -1):
            th = th0.copy()
            th[p] += sgn * 1e-7 * th0[p]
            b = ADJ.PathwiseAdjoint(ADJ.with_theta(prob, th), parts, Ks, seg)
            Js.append(b.forward(0).cpu().numpy())
        fds[:, p] = (Js[0] - Js[1]) / (2e-7 * th0[p])
    rels = np.abs(Gs[0] - fds[0]) / np.maximum(np.abs(fds[0]), 1e-300)
    log(f"  8 steps, h = 1e-7: mdot gradient {Gs[0]}, central differences {fds[0]}")
    res = dict(
        metric=METRIC, value=round(n * K / t_bwd, 1), unit="particle-steps/s", n_gpus=1, steps=K,
        warmup=args.warmup, ms_per_step=round(t_bwd / K * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config={"workload": "poiseuille_kn0.05_100x500_adjoint", "particles": n, "cells": 100,
                "state": "f64", "checkpoint_every": seg, "outputs": ["mdot", "tau_w"],
                "parameters": ["Z_rot", "omega", "mu_ref"], "parallelism": "single-gpu"},
        value_kind="reverse pass (re-run with tapes + adjoint), particle-steps/s",
        adjoint_forward_ratio=round(t_bwd / t_plain, 3),
        forward_and_adjoint_ratio=round((t_fwd + t_bwd) / t_plain, 3),
        times_s={"plain_forward": round(t_plain, 4), "forward_checkpointed": round(t_fwd, 4),
                 "reverse": round(t_bwd, 4)},
        outputs={"mdot": float(J[0]), "tau_w": float(J[1])},
        gradient=G.tolist(),
        fd_check={"h_relative": 1e-4, "central_differences": fd.tolist(),
                  "relative_difference": rel.tolist(),
                  "note": "differences of full runs: cell switches, wall hits and level jumps "
                          "that the perturbation flips are outside the pathwise derivative, "
                          "which itself grows about 30x per 100 steps on this case"},
        fd_check_short={"steps": Ks, "h_relative": 1e-7, "mdot_gradient": Gs[0].tolist(),
                        "mdot_central_differences": fds[0].tolist(),
                        "relative_difference": rels.tolist()},
    )
    return res, prob, parts


def run_cpu_adjoint_baseline(prob, parts, K=4):
    """The oracle's gradient (PyTorch FP64 replay with autograd) over the
    first K steps of the same workload, on the host's cores."""
    import torch

    from oracle import adjoint as A
    t0 = time.perf_counter()
    path = A.Path(A.Record(prob, parts, 0, K))
    path.gradient()
    dt = time.perf_counter() - t0
    n = int(parts["n"])
    return {"value": round(n * K / dt, 1), "unit": "particle-steps/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"record + autograd gradient of the first {K} steps of the same case "
                      f"({n} particles), FP64, {dt:.1f} s"}


def _oracle_steps(prob, parts, nsteps, threads=0):
    import oracle
    sim = oracle.Sim(prob, parts, threads=threads)
    total = 0
    t0 = time.perf_counter()
    for s in range(nsteps):
        sim.bin()
        total += sim.n
        sim.do_moments()
        sim.do_cellstate()
        sim.collide(s)
        sim.conserve(s)
        sim.advect(s)
    return total, time.perf_counter() - t0


def run_cpu_baseline(prob, parts, nsteps, one_core_steps=1, what="cylinder"):
    """The oracle on all host threads for `nsteps` steps, and on one thread
    for `one_core_steps` steps, from the workload's initial state."""
    import oracle
    all_threads = oracle.threads()
    total, dt = _oracle_steps(prob, parts, nsteps)
    res = {"value": round(total / dt, 1), "unit": "particle-steps/s", "cores": all_threads,
           "kind": "oracle",
           "sample": f"{nsteps} full steps of the same {what} workload from its initial state "
                     f"({parts['n']} particles), FP64 oracle, {dt:.1f} s"}
    if one_core_steps > 0:
        t1, d1 = _oracle_steps(prob, parts, one_core_steps, threads=1)
        res["value_1core"] = round(t1 / d1, 1)
        res["sample_1core"] = f"{one_core_steps} step(s) on 1 thread, {d1:.1f} s"
        oracle.lib().orc_set_threads(all_threads)
    return res


def run_gpu_c2(args):
    """The batched 0D workload (4096 uneven cells, ~3.0M particles, FP32):
    one usp_step bins it, the warmup runs eagerly on the default schedule,
    the autotuner then picks the usp_batch schedule on the warmed state, and
    the timed steps are one usp_batch call captured in a HIP graph and
    replayed once."""
    import torch

    import usp_workloads as W
    from paper_2508_05642_amd import autotune, usp

    torch.cuda.set_device(0)
    prob, parts = W.batch_c2()
    n = parts["n"]
    log(f"workload ready: {n} particles, {prob.grid.ncells} cells")
    st = usp.DeviceState(prob, parts, device="cuda:0")
    st.step(0, 1)
    step = 1
    # warmup on the library's default schedule, then the schedule is chosen
    # on the state the timed steps start from (the cells relax over the
    # first steps, and with them the cost of each candidate)
    if args.warmup:
        st.batch(step, args.warmup, 0, 0)
        step += args.warmup
    if args.schedule:
        tile, spl = (int(x) for x in args.schedule.split(","))
        log(f"schedule (given): tile {tile}, steps per launch {spl or 'all'}")
    else:
        tune = autotune.tune_batch(st, step=step, nsteps=24, reps=3)
        tile, spl = tune["tile"], tune["steps_per_launch"]
        log(f"schedule: tile {tile}, steps per launch {spl or 'all'} "
            f"({ {f'{k[0]}/{k[1]}': round(v, 4) for k, v in tune['ms_per_step'].items()} } ms/step)")
    torch.cuda.synchronize()
    K = args.steps
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        st.batch(step, K, tile, spl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_ev = e0.elapsed_time(e1)
    ctr = stored_counters("k_batch")
    t_step = ms_ev * 1e-3 / K
    if ctr:
        ach = ctr["valu_per_particle"] * n / t_step
        roof = {"bound": "alu", "kernel": "k_batch", "achieved": round(ach / 1e9, 2),
                "peak": round(VALU_PEAK / 1e9, 1), "unit": "G VALU wave-instr/s",
                "frac": round(ach / VALU_PEAK, 4),
                "traffic": int((ctr["fetch_bytes"] + ctr["write_bytes"])),
                "valu_per_particle": ctr["valu_per_particle"], "avg_ms": round(ms_ev, 3)}
    else:
        roof = {"bound": "alu", "kernel": "k_batch", "achieved": None, "peak": round(VALU_PEAK / 1e9, 1),
                "unit": "G VALU wave-instr/s", "frac": None, "traffic": None,
                "avg_ms": round(ms_ev, 3)}
    res = dict(
        metric=METRIC, value=round(n * K / wall, 1), unit="particle-steps/s", n_gpus=1, steps=K,
        warmup=args.warmup, ms_per_step=round(wall / K * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config={"workload": "batch0d_4096_uneven_cells", "particles": int(n), "cells": 4096,
                "state": "f32", "accumulation": "f64", "schedule": {"tile": tile,
                "steps_per_launch": spl}, "hip_graph": True, "parallelism": "single-gpu"},
        roofline=roof, counters={k: v for k, v in st.cnt().items() if v},
    )
    return res, prob, parts


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("cylinder", "c2", "adjoint"), default="cylinder",
                    help="cylinder (the headline case) or c2 (4096 independent 0D cells)")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (cylinder 100, c2 500)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="grid scale of the cylinder workload (1.0 = full size)")
    ap.add_argument("--schedule", default=None, metavar="TILE,SPL",
                    help="c2: fixed usp_batch schedule (tile, steps per launch; 0 = all) "
                         "instead of the autotuner's choice")
    ap.add_argument("--sample", type=int, default=0, metavar="NBODY",
                    help="cylinder: sample fields every step and wall fluxes with NBODY "
                         "angular elements on the cylinder (0 = no sampling)")
    ap.add_argument("--no-fd", action="store_true",
                    help="adjoint: skip the finite-difference runs (profiling)")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", choices=("usp", "fpm"), default="usp",
                    help="cylinder: the USP-FPM scheme (default) or the first-order FPM scheme")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU (the multi-GPU split is not implemented); "
              f"--gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
    if args.steps is None:
        args.steps = {"c2": 500, "adjoint": 2000}.get(args.workload, 100)
    if args.workload == "adjoint":
        res, prob, parts = run_gpu_adjoint(args)
        log(f"GPU reverse: {res['value']:.4g} particle-steps/s, adjoint/forward "
            f"{res['adjoint_forward_ratio']}")
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = run_cpu_adjoint_baseline(prob, parts)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "c2":
        res, prob, parts = run_gpu_c2(args)
    else:
        res, prob, parts = run_gpu(args)
    log(f"GPU: {res['value']:.4g} particle-steps/s, {res['ms_per_step']} ms/step")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = run_cpu_baseline(
            prob, parts, args.cpu_steps, one_core_steps=1,
            what="cylinder" if args.workload == "cylinder" else "batched 0D")
        log(f"CPU oracle: {res['cpu_baseline']['value']:.4g} particle-steps/s "
            f"({res['cpu_baseline'].get('value_1core', 0):.4g} on 1 thread)")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
