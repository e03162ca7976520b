#!/usr/bin/env python3
"""Throughput of the full USP-FPM step on one MI355X.

Workload: Mach-10 N2 over a cylinder (half body), 600 x 300 cells of 1 mm,
~36.1M particles at start (FP32 particle state, FP64 cell accumulators),
VHS gas with Parker / Millikan-White collision numbers, dt = 1.25e-7 s.
A step is bin -> moments -> cell state -> the fused particle phase
(collide + conserve + advect with injection, one pass), each a call of the
C ABI on torch's current stream so HIP events bracket every phase.  `value`
is particle-steps/s over exactly --steps timed steps (inputs resident in
HBM), after --warmup steps, replayed from one HIP graph; an eager pass over
the same steps from the same state gives the per-phase and k_update times.

Also reported on the same line:
  roofline      the HBM roofline of the dominant kernel (k_update): the
                algorithmic bytes of one launch over its average duration,
                timed with HIP events recorded by the library around that
                kernel alone, against the 8 TB/s peak; the step's own HBM
                fraction beside it;
  oracle_error  the first step on the GPU against the FP64 oracle's first
                step from the same initial state;
  developed     particle-steps/s after --developed steps (the flow has
                formed its shock layer);
  adjoint       the pathwise adjoint's reverse/forward time ratio on the
                differentiable channel;
  c2            the batched 0D solve's throughput;
  c0            the single-cell 0D relaxation (100,000 particles, FP64), whose
                cell is split over the chip (c0 and c2 also give an effective
                cache-resident rate: the bytes a 0D step would stream per
                particle times the throughput);
  gamma_scope   the headline window with the coefficient chain per particle
                and once per cell (the two readings), eager, side by side;
  cpu_baseline  the oracle timed on the host's cores on a bounded sample.
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


# algorithmic bytes per particle-step of the whole step and of the fused
# particle kernel (FP32 cylinder layout of 33 B per particle): moments read
# 17, fused collide+conserve+advect read 29 and write 29, rebin scatter read
# and write 66, per-cell traffic about 2; the fused kernel's per-cell bytes
# are its cell record (128) and the conservation planes (9 x 8) with the
# offsets (8)
STEP_BYTES_PER_PARTICLE = 17 + 29 + 29 + 66
STEP_BYTES_PER_CELL = 400
UPDATE_BYTES_PER_PARTICLE = 29 + 29
UPDATE_BYTES_PER_CELL = 128 + 9 * 8 + 8


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


def _roctx():
    """roctxProfilerResume/Pause of the ROCTx library (no-ops unless the
    process runs under `rocprofv3 --selected-regions`), or None."""
    import ctypes
    for nm in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
        try:
            L = ctypes.CDLL(nm)
        except OSError:
            continue
        for f in (L.roctxProfilerResume, L.roctxProfilerPause):
            f.argtypes = [ctypes.c_uint64]
            f.restype = ctypes.c_int
        return L
    return None


def _raw_event(torch):
    """A timing torch.cuda.Event with its HIP event created (recorded once),
    so that its handle can be given to the library."""
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def _mom_scales(prob, om, names):
    """The natural scale of each moment plane of each cell: the count 1, the
    mean level max(1, I), velocities sqrt(R T) + |U|, second moments
    R T + e_rot, heat fluxes (R T + e_rot) sqrt(R T), <C I> sqrt(R T) I."""
    import numpy as np
    T = np.maximum((om[names.index("PXX")] + om[names.index("PYY")] + om[names.index("PZZ")]) / 3,
                   1.0)
    c = np.sqrt(T)
    Ib = np.maximum(1.0, om[names.index("IBAR")])
    U = np.abs(om[1:4]).max(axis=0)
    E = T + np.abs(om[names.index("EROT")])
    sc = {}
    for k in names:
        sc[k] = {"N": np.ones_like(T), "IBAR": Ib}.get(k)
        if k in ("UX", "UY", "UZ"):
            sc[k] = c + U
        elif k in ("PXX", "PYY", "PZZ", "PXY", "PXZ", "PYZ", "EROT"):
            sc[k] = E
        elif k.startswith("QTR") or k.startswith("QROT"):
            sc[k] = E * c
        elif k.startswith("QI"):
            sc[k] = c * Ib
    return sc


def oracle_error(prob, g, o):
    """The GPU's first step against the oracle's first step from the same
    initial state.  g, o: {"mom", "cs", "state", "cnt"}.  Moments: the
    largest difference over each cell's natural scale; cell state: the
    largest relative difference (floored at 1e-6 of the plane's largest
    value); particles (same slot order on both sides): the largest difference
    of each array over the velocity scale (max sqrt(R T_tr) + |U| over the
    cells), its square for e_rot, the domain length for x and y; the
    fractions of equal levels and cells; whether the event counters agree."""
    import numpy as np

    import oracle
    mn, cn = oracle.MOM_NAMES, oracle.CS_NAMES
    om, gm = o["mom"], g["mom"]
    sc = _mom_scales(prob, om, mn)
    mom_err = max(float((np.abs(gm[k] - om[k]) / sc[nm]).max()) for k, nm in enumerate(mn))
    oc, gc = o["cs"], g["cs"]
    cs_err = 0.0
    for k in range(len(cn)):
        fs = np.max(np.abs(oc[k])) + 1e-300
        cs_err = max(cs_err, float((np.abs(gc[k] - oc[k]) / (np.abs(oc[k]) + 1e-6 * fs)).max()))
    T = oc[cn.index("TTR")]
    U = np.abs(oc[cn.index("UX"):cn.index("UZ") + 1]).max(axis=0)
    vs = float(np.max(np.sqrt(prob.gas.R * np.maximum(T, 1.0)) + U))
    a, b = g["state"], o["state"]
    res = {"particles": int(a["n"]), "same_count": bool(a["n"] == b["n"]),
           "moments_vs_natural_scale": mom_err, "cell_state_relative": cs_err}
    if a["n"] == b["n"]:
        res["same_order"] = bool(np.array_equal(a["pid"], b["pid"]))
        gr = prob.grid
        scale = {"cx": vs, "cy": vs, "cz": vs, "erot": vs * vs, "x": gr.nx * gr.dx,
                 "y": gr.ny * gr.dy}
        res["particle_max_scaled_diff"] = {
            k: float((np.abs(a[k] - b[k]) / scale[k]).max()) for k in scale if a.get(k) is not None}
        res["vib_level_agreement"] = float(np.mean(a["vib"] == b["vib"]))
        res["cell_agreement"] = float(np.mean(a["cell"] == b["cell"]))
    res["counters_equal"] = bool(g["cnt"] == o["cnt"])
    return res


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
    rtx = _roctx()
    first = {}

    def one_step(s, ev=None, nlog=None, k=None, kev=None, keep=None):
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
        if keep is not None:
            keep["mom"], keep["cs"] = st.moments(), st.cellstate()
        if ev: ev[3].record()
        st.update(s, events=kev)
        if ev: ev[4].record()
        if keep is not None:
            keep["state"], keep["cnt"] = st.state(), st.cnt()

    for _ in range(args.warmup):
        # the first step from the initial state is kept for the comparison
        # with the oracle's first step
        one_step(step, keep=first if (step == 0 and args.oracle_error) else None)
        step += 1
    torch.cuda.synchronize()
    log(f"{args.warmup} warmup steps done")
    K = args.steps
    step0 = step
    snap = _snapshot(st)
    # eager pass: per-phase times (events between the phases) and the
    # particle kernel alone (events the library records around it)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(PHASES) + 1)] for _ in range(K)]
    kevs = [(_raw_event(torch), _raw_event(torch)) for _ in range(K)]
    nlog = torch.zeros(K, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    if rtx:
        rtx.roctxProfilerResume(0)
    t0 = time.perf_counter()
    for k in range(K):
        one_step(step0 + k, evs[k], nlog, k,
                 kev=(kevs[k][0].cuda_event, kevs[k][1].cuda_event))
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    if rtx:
        rtx.roctxProfilerPause(0)
    # timed pass: the same K steps from the same state, captured in one HIP
    # graph and replayed once
    _restore(st, snap)
    del snap
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
    del graph
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
    kms = [kevs[k][0].elapsed_time(kevs[k][1]) for k in range(K)]
    k_ms = float(np.mean(kms))
    total_ps = float(ns.sum())
    n_mean = float(ns.mean())
    ms_step = wall / K * 1e3
    # the dominant kernel: bytes of one launch at the mean particle count
    upd_bytes = UPDATE_BYTES_PER_PARTICLE * n_mean + UPDATE_BYTES_PER_CELL * M
    ach = upd_bytes / (k_ms * 1e-3) / 1e9
    step_bytes = STEP_BYTES_PER_PARTICLE * n_mean + STEP_BYTES_PER_CELL * M
    step_gbs = step_bytes / (ms_step * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_update", "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": None, "avg_ms": round(k_ms, 4),
            "min_ms": round(float(np.min(kms)), 4), "max_ms": round(float(np.max(kms)), 4),
            "window": f"steps {step0}..{step0 + K - 1} (eager pass; HIP events around each "
                      f"k_update launch, on its stream)",
            "bytes_per_particle": UPDATE_BYTES_PER_PARTICLE,
            "bytes_per_cell": UPDATE_BYTES_PER_CELL,
            "algorithmic_bytes_per_launch": int(upd_bytes),
            "step": {"achieved": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_particle": STEP_BYTES_PER_PARTICLE,
                     "bytes_per_cell": STEP_BYTES_PER_CELL, "ms_per_step": round(ms_step, 4)}}
    # counters of the same sources and flags (PMC), when they are on record
    ctr = stored_counters("k_update") if args.scheme == "usp" else None
    if ctr:
        roof["traffic"] = int(ctr["fetch_bytes"] + ctr["write_bytes"])
        roof["traffic_per_particle"] = round(roof["traffic"] / n_mean, 1)
        valu = ctr["valu_per_particle"] * n_mean / (k_ms * 1e-3)
        roof["valu"] = {"achieved": round(valu / 1e9, 2), "peak": round(VALU_PEAK / 1e9, 1),
                        "unit": "G VALU wave-instr/s", "frac": round(valu / VALU_PEAK, 4),
                        "valu_per_particle": ctr["valu_per_particle"]}
    cnt = st.cnt()
    res = dict(
        metric=METRIC, value=round(total_ps / wall, 1), unit="particle-steps/s", n_gpus=1,
        steps=K, warmup=args.warmup, ms_per_step=round(ms_step, 4),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config={"workload": f"cylinder_mach10_{prob.grid.nx}x{prob.grid.ny}",
                "particles_start": int(n0), "particles_mean": int(n_mean), "cells": M,
                "state": "f32", "accumulation": "f64", "dt_s": prob.dt,
                "first_timed_step": args.warmup, "sampling": bool(args.sample),
                "scheme": args.scheme, "parallelism": "single-gpu"},
        launch="one HIP graph of the K steps (per-phase and k_update times from an eager pass "
               "over the same steps from the same state)",
        eager_ms_per_step=round(wall_eager / K * 1e3, 4),
        graph_event_ms=round(ms_graph, 3),
        phase_ms=phase_ms,
        step_algorithmic_gbs=round(step_gbs, 1),
        hbm_copy_gbs=hbm_copy,
        roofline=roof,
        counters={k: v for k, v in cnt.items() if v},
    )
    if args.developed and args.developed > step0 + K:
        # keep stepping (eagerly, with the run's own step indices) until the
        # shock layer has formed, then time K more steps
        s = step0 + K
        while s < args.developed:
            one_step(s)
            s += 1
        torch.cuda.synchronize()
        kd = [(_raw_event(torch), _raw_event(torch)) for _ in range(K)]
        nd = torch.zeros(K, dtype=torch.int64, device=dev)
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        d0.record()
        for k in range(K):
            one_step(s + k, None, nd, k, kev=(kd[k][0].cuda_event, kd[k][1].cuda_event))
        d1.record()
        torch.cuda.synchronize()
        dms = d0.elapsed_time(d1)
        ndm = nd.cpu().numpy()
        kdm = float(np.mean([kd[k][0].elapsed_time(kd[k][1]) for k in range(K)]))
        nmd = float(ndm.mean())
        ub = UPDATE_BYTES_PER_PARTICLE * nmd + UPDATE_BYTES_PER_CELL * M
        res["developed"] = {
            "first_step": s, "steps": K, "value": round(float(ndm.sum()) / (dms * 1e-3), 1),
            "unit": "particle-steps/s", "ms_per_step": round(dms / K, 4),
            "particles_mean": int(nmd), "k_update_ms": round(kdm, 4),
            "k_update_hbm_frac": round(ub / (kdm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch": "eager (events around the K steps)",
            "counters_since_start": {k: v for k, v in st.cnt().items() if v}}
        log(f"developed flow (steps {s}..{s + K - 1}): {res['developed']['value']:.4g} "
            f"particle-steps/s, {dms / K:.4f} ms/step")
    del st
    torch.cuda.empty_cache()
    return res, prob, parts, first


def eager_window(prob, parts, warmup, K):
    """K eager steps of the gather pipeline after `warmup` steps from the
    initial state: HIP events around the K steps and around each k_update
    launch.  Returns (particle-steps/s, ms/step, k_update ms, mean
    particles, counters)."""
    import numpy as np
    import torch

    from paper_2508_05642_amd import usp

    st = usp.DeviceState(prob, parts, device="cuda:0")

    def one(s, nlog=None, k=None, kev=None):
        st.bin(gather=True)
        if nlog is not None:
            nlog[k].copy_(st.bufs[1 - st.cur]["count"][0])
        st.do_moments()
        st.do_reconstruct()
        st.update(s, events=kev)

    for s in range(warmup):
        one(s)
    kd = [(_raw_event(torch), _raw_event(torch)) for _ in range(K)]
    nd = torch.zeros(K, dtype=torch.int64, device="cuda:0")
    d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    d0.record()
    for k in range(K):
        one(warmup + k, nd, k, (kd[k][0].cuda_event, kd[k][1].cuda_event))
    d1.record()
    torch.cuda.synchronize()
    dms = d0.elapsed_time(d1)
    ndm = nd.cpu().numpy()
    kdm = float(np.mean([kd[k][0].elapsed_time(kd[k][1]) for k in range(K)]))
    cnt = {k: v for k, v in st.cnt().items() if v}
    del st
    torch.cuda.empty_cache()
    return float(ndm.sum()) / (dms * 1e-3), dms / K, kdm, float(ndm.mean()), cnt


def gamma_cell_window(prob, parts, warmup, K):
    """The headline window with the coefficient chain taken once per cell
    (gamma_scope = cell), next to the per-particle chain, both eager."""
    import dataclasses

    import usp_workloads as W

    M = prob.grid.ncells
    out = {}
    for name, scope in (("particle", W.GAMMA_PARTICLE), ("cell", W.GAMMA_CELL)):
        pr = dataclasses.replace(prob, gas=dataclasses.replace(prob.gas, gamma_scope=scope))
        v, ms, kms, nm, _ = eager_window(pr, parts, warmup, K)
        ub = UPDATE_BYTES_PER_PARTICLE * nm + UPDATE_BYTES_PER_CELL * M
        out[name] = {"value": round(v, 1), "ms_per_step": round(ms, 4),
                     "k_update_ms": round(kms, 4),
                     "k_update_hbm_frac": round(ub / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["unit"] = "particle-steps/s"
    out["window"] = f"steps {warmup}..{warmup + K - 1}, eager, events around the K steps"
    return out


# Bytes per particle-step of a 0D step if its passes streamed the state
# (moments read c, e_rot, I; update read c, e_rot, I, id; update write c,
# e_rot, I): 17 + 21 + 17 B for an FP32 state, 33 + 37 + 33 B for FP64.
# The 0D workloads fit the Infinity Cache (and the batched kernel keeps a
# tile's particles in LDS for all its steps), so the product of this figure
# and the throughput is an effective, cache-resident rate, not HBM traffic.
ZERO_D_BYTES = {"f32": 55, "f64": 103}


def effective_0d(value, state):
    return {"effective_gbs_cache_resident": round(value * ZERO_D_BYTES[state] / 1e9, 1),
            "bytes_per_particle_step": ZERO_D_BYTES[state]}


def relax0d_timing(K=200, warmup=20):
    """The 0D relaxation at full size (one cell, 100,000 particles, FP64):
    usp_step, K steps after `warmup`, events around them."""
    import torch

    import usp_workloads as W
    from paper_2508_05642_amd import usp

    prob = W.relax0d()
    parts = W.particles_for(prob)
    st = usp.DeviceState(prob, parts, device="cuda:0")
    st.step(0, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    st.step(warmup, K)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    n = int(parts["n"])
    del st
    torch.cuda.empty_cache()
    value = round(n / (ms * 1e-3), 1)
    return {"workload": "relax0d (1 cell, 100,000 particles, FP64)", "steps": K,
            "ms_per_step": round(ms, 4), "value": value,
            "unit": "particle-steps/s", "launch": "one usp_step call of K steps",
            **effective_0d(value, "f64")}


def adjoint_timing(K, warmup=20, seg=32):
    """The differentiable Poiseuille case: Kn = 0.05, 100 cells x 500
    particles (50,000), FP64, K steps from the initial state.  Times a plain
    forward (usp_step), the checkpointed forward with output sampling, and
    the reverse pass (re-run with tapes + usp_adjoint_step), a checkpoint
    every `seg` steps.  Returns (times, outputs J, gradient G, prob, parts)."""
    import torch

    import usp_workloads as W
    from paper_2508_05642_amd import adjoint as ADJ, usp

    torch.cuda.set_device(0)
    prob = W.poiseuille(kn=0.05, cells=100, ppc=500, f32=False, seed=7)
    parts = W.particles_for(prob)
    n = int(parts["n"])
    log(f"adjoint workload ready: {n} particles, {prob.grid.ncells} cells, {K} steps")
    warm = usp.DeviceState(prob, parts)
    for k in range(warmup):
        warm.step(k, 1)
    wa = ADJ.PathwiseAdjoint(prob, parts, min(K, 4), 2, allow_long=True)
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
    adj = ADJ.PathwiseAdjoint(prob, parts, K, seg, allow_long=True)
    J, t_fwd = timed(lambda: adj.forward(0))
    G, t_bwd = timed(lambda: adj.backward())
    J, G = J.cpu().numpy(), G.cpu().numpy()
    del st, adj
    torch.cuda.empty_cache()
    log(f"plain forward {t_plain:.3f} s, forward with checkpoints {t_fwd:.3f} s, "
        f"reverse {t_bwd:.3f} s; J = {J}")
    times = {"plain_forward": round(t_plain, 4), "forward_checkpointed": round(t_fwd, 4),
             "reverse": round(t_bwd, 4)}
    return times, J, G, prob, parts


def run_gpu_adjoint(args):
    """adjoint_timing over --steps steps, then the gradient against central
    differences of the outputs (h = 1e-4 relative, common random numbers:
    same seed)."""
    import numpy as np

    from paper_2508_05642_amd import adjoint as ADJ
    K, seg = args.steps, 32
    times, J, G, prob, parts = adjoint_timing(K, args.warmup, seg)
    n = int(parts["n"])
    t_plain, t_fwd, t_bwd = times["plain_forward"], times["forward_checkpointed"], times["reverse"]
    th0 = np.array([prob.gas.Z_rot, prob.gas.omega, prob.gas.mu_ref])
    # finite-difference check within the validated horizon: the mass-flow
    # gradient over Kf steps against central differences of complete runs
    # (h = 1e-8 relative: no discrete outcome of the run changes)
    Kf, hf = min(32, ADJ.VALID_HORIZON), 1e-8
    a = ADJ.PathwiseAdjoint(prob, parts, Kf, seg)
    a.forward(0)
    Gs = a.backward().cpu().numpy()
    fds = np.full(3, np.nan)
    for p in range(3 if not args.no_fd else 0):
        Js = []
        for sgn in (1, -1):
            th = th0.copy()
            th[p] += sgn * hf * th0[p]
            b = ADJ.PathwiseAdjoint(ADJ.with_theta(prob, th), parts, Kf, seg)
            Js.append(b.forward(0).cpu().numpy()[0])
        fds[p] = (Js[0] - Js[1]) / (2 * hf * th0[p])
    rels = np.abs(Gs[0] - fds) / np.maximum(np.abs(fds), 1e-300)
    log(f"  {Kf} steps, h = {hf:g}: mdot gradient {Gs[0]}, central differences {fds}, rel {rels}")
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
        fd_check={"steps": Kf, "h_relative": hf, "output": "mdot",
                  "gradient": Gs[0].tolist(), "central_differences": fds.tolist(),
                  "relative_difference": rels.tolist(),
                  "note": f"within the validated horizon ({ADJ.VALID_HORIZON} steps); the "
                          "wall shear's differences are checked against FP64 oracle runs in "
                          "tests/test_gpu_adjoint.py (the device wall sums are fixed point)"},
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


def _oracle_step(sim, s, keep=None):
    sim.bin()
    n = sim.n
    sim.do_moments()
    sim.do_cellstate()
    if keep is not None:
        keep["mom"], keep["cs"] = sim.moments().copy(), sim.cellstate().copy()
    sim.collide(s)
    sim.conserve(s)
    sim.advect(s)
    if keep is not None:
        keep["state"], keep["cnt"] = sim.state(), sim.cnt()
    return n


def run_cpu_baseline(prob, parts, warm, timed, one_core_steps=1, what="cylinder", keep=None):
    """The oracle on all host threads: `warm` steps from the workload's
    initial state (the first kept in `keep` when given), then `timed` steps
    timed; and `one_core_steps` steps on one thread from the initial
    state."""
    import oracle
    all_threads = oracle.threads()
    sim = oracle.Sim(prob, parts)
    for s in range(warm):
        _oracle_step(sim, s, keep if s == 0 else None)
    total = 0
    t0 = time.perf_counter()
    for s in range(warm, warm + timed):
        total += _oracle_step(sim, s)
    dt = time.perf_counter() - t0
    del sim
    res = {"value": round(total / dt, 1), "unit": "particle-steps/s", "cores": all_threads,
           "kind": "oracle",
           "sample": f"steps {warm}..{warm + timed - 1} of the same {what} workload "
                     f"({parts['n']} particles at start), timed after {warm} warm-up steps "
                     f"from its initial state, FP64 oracle, {dt:.1f} s"}
    if one_core_steps > 0:
        oracle.lib().orc_set_threads(1)
        sim = oracle.Sim(prob, parts, threads=1)
        t1 = 0
        t0 = time.perf_counter()
        for s in range(one_core_steps):
            t1 += _oracle_step(sim, s)
        d1 = time.perf_counter() - t0
        del sim
        res["value_1core"] = round(t1 / d1, 1)
        res["sample_1core"] = f"step(s) 0..{one_core_steps - 1} on 1 thread, {d1:.1f} s"
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
        **effective_0d(n * K / wall, "f32"),
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
    ap.add_argument("--developed", type=int, default=2000, metavar="STEP",
                    help="cylinder: also time --steps steps from this step on (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="cylinder: skip the adjoint, batched-0D, single-cell and "
                         "gamma-scope figures")
    ap.add_argument("--no-oracle-error", dest="oracle_error", action="store_false",
                    help="cylinder: skip the first-step comparison with the oracle")
    ap.add_argument("--cpu-warmup", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=20)
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
        log(f"GPU: {res['value']:.4g} particle-steps/s, {res['ms_per_step']} ms/step")
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = run_cpu_baseline(prob, parts, args.cpu_warmup, args.cpu_steps,
                                                   what="batched 0D")
        print(json.dumps(res), flush=True)
        return
    res, prob, parts, first = run_gpu(args)
    log(f"GPU: {res['value']:.4g} particle-steps/s, {res['ms_per_step']} ms/step")
    if not args.no_extras:
        times, _, _, _, _ = adjoint_timing(2000)
        res["adjoint"] = {
            "workload": "poiseuille_kn0.05_100x500_adjoint (FP64, 2000 steps, checkpoint every 32)",
            "adjoint_forward_ratio": round(times["reverse"] / times["plain_forward"], 3),
            "forward_and_adjoint_ratio": round(
                (times["forward_checkpointed"] + times["reverse"]) / times["plain_forward"], 3),
            "times_s": times}
        c2args = argparse.Namespace(steps=500, warmup=20, schedule=None)
        c2, _, _ = run_gpu_c2(c2args)
        res["c2"] = {"workload": c2["config"]["workload"], "value": c2["value"],
                     "unit": c2["unit"], "ms_per_step": c2["ms_per_step"], "steps": 500,
                     "schedule": c2["config"]["schedule"], "launch": "one HIP graph of 500 steps",
                     **effective_0d(c2["value"], "f32")}
        log(f"adjoint/forward {res['adjoint']['adjoint_forward_ratio']}, "
            f"c2 {c2['value']:.4g} particle-steps/s")
        res["c0"] = relax0d_timing()
        log(f"c0 {res['c0']['ms_per_step']} ms/step")
        res["gamma_scope"] = gamma_cell_window(prob, parts, args.warmup, args.steps)
        log(f"gamma scope per particle / per cell: "
            f"{res['gamma_scope']['particle']['k_update_ms']} / "
            f"{res['gamma_scope']['cell']['k_update_ms']} ms k_update")
    if not args.no_cpu_baseline:
        keep = {} if first else None
        res["cpu_baseline"] = run_cpu_baseline(prob, parts, args.cpu_warmup, args.cpu_steps,
                                               what="cylinder", keep=keep)
        log(f"CPU oracle: {res['cpu_baseline']['value']:.4g} particle-steps/s "
            f"({res['cpu_baseline'].get('value_1core', 0):.4g} on 1 thread)")
        if keep:
            res["oracle_error"] = oracle_error(prob, first, keep)
            res["oracle_error"]["step"] = 0
            log(f"oracle error of the first step: {res['oracle_error']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
