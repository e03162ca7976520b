"""Schedule autotuner for the batched 0D solve (usp_batch).

Each candidate schedule (tile window in particle slots, steps per launch)
is timed on the caller's own state for a few steps with HIP events; the
state is restored after every trial, so tuning does not advance the
simulation.  The fastest choice is cached per problem signature (cells,
capacity, precision) for the life of the process.
"""
import torch

from . import usp

CANDIDATES_F32 = ((512, 0), (1024, 0), (2048, 0), (512, 1), (1024, 1), (2048, 1))
CANDIDATES_F64 = ((512, 0), (512, 1))

_cache = {}


def _signature(st):
    return (st.M, st.cap, st.prec, st.dim)


def _snapshot(st):
    keep = [{k: v.clone() for k, v in B.items() if k != "struct" and torch.is_tensor(v)}
            for B in st.bufs]
    extra = {k: getattr(st, k).clone() for k in ("offsets", "mom", "cs", "counters")}
    return keep, extra


def _restore(st, snap):
    keep, extra = snap
    for B, S in zip(st.bufs, keep):
        for k, v in S.items():
            B[k].copy_(v)
    for k, v in extra.items():
        getattr(st, k).copy_(v)


def tune_batch(st, step=0, nsteps=8, candidates=None, reps=2, stream=None):
    """Best (tile, steps_per_launch) for usp_batch on the binned 0D state
    `st` (a usp.DeviceState), and the measured ms per step of every
    candidate.  Cached per signature; the state is left unchanged."""
    key = _signature(st)
    if key in _cache:
        return _cache[key]
    if candidates is None:
        candidates = CANDIDATES_F32 if st.prec == usp.USP_F32 else CANDIDATES_F64
    snap = _snapshot(st)
    times = {}
    for tile, spl in candidates:
        best = float("inf")
        for _ in range(reps):
            _restore(st, snap)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st.batch(step, nsteps, tile, spl, stream)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / nsteps)
        times[(tile, spl)] = best
    _restore(st, snap)
    torch.cuda.synchronize()
    choice = min(times, key=times.get)
    _cache[key] = {"tile": choice[0], "steps_per_launch": choice[1], "ms_per_step": times}
    return _cache[key]
