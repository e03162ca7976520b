"""usp_update_noalloc (the fused particle phase with its scratch in the
library's fixed device array) through the C ABI against usp_update (the same
phase with a caller workspace): bit-identical states and counters on two
calls in a row, the second with a smaller input; sizes beyond the fixed
array are rejected on the host."""
import ctypes
import sys

import numpy as np
import pytest

import usp_workloads as W

torch = pytest.importorskip("torch")

ESCRATCH = -6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _snap(st):
    B = st.bufs[st.cur]
    return ({k: v.clone() for k, v in B.items() if k != "struct" and v is not None},
            st.counters.clone())


def _put(st, snap):
    B = st.bufs[st.cur]
    for k, v in snap[0].items():
        B[k].copy_(v)
    st.counters.copy_(snap[1])


def _host(st):
    torch.cuda.synchronize()
    B = st.bufs[st.cur]
    return ({k: v.cpu().numpy().copy() for k, v in B.items() if k != "struct" and v is not None},
            st.counters.cpu().numpy().copy())


def _fn():
    from paper_2508_05642_amd import usp
    f = usp.lib().usp_update_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                  ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int32
    return f


def _noalloc(st, step):
    bc = ctypes.byref(st.bc) if st.dim >= 1 else None
    return _fn()(ctypes.byref(st.grid), ctypes.byref(st.gas), bc, st.prob.dt, st.cs.data_ptr(),
                 st.offsets.data_ptr(), ctypes.byref(st.p), st.prob.seed, step,
                 st.counters.data_ptr(), torch.cuda.current_stream().cuda_stream)


def _case(prob, parts, step):
    from paper_2508_05642_amd import usp
    st = usp.DeviceState(prob, parts)
    st.step(0, 2)           # a developed, binned state with injected particles
    st.bin()
    st.do_moments()
    st.do_reconstruct()
    snap = _snap(st)
    st.update(step)         # usp_update with the caller workspace
    ref = _host(st)
    _put(st, snap)
    status = _noalloc(st, step)
    assert status == 0, status
    got = _host(st)
    for k, v in ref[0].items():
        assert np.array_equal(v.view(np.uint8), got[0][k].view(np.uint8)), k
    assert np.array_equal(ref[1], got[1])
    return int(ref[0]["count"][0])


@pytest.mark.gpu
def test_noalloc_update_matches_update_twice():
    """Two calls in a row on one GPU, the second on a smaller input: every
    array of the resulting state and every counter equals usp_update's."""
    sizes = []
    for scale, step in ((0.05, 5), (0.03, 9)):
        prob = W.cylinder(scale=scale, f32=True)
        parts = W.particles_for(prob)
        _say(f"[noalloc] cylinder scale {scale}, n={parts['n']}, step {step}")
        sizes.append(_case(prob, parts, step))
    assert sizes[1] < sizes[0]


@pytest.mark.gpu
def test_noalloc_update_fp64_channel():
    """The FP64 state of the 1D channel (no injection; FP64 stage)."""
    prob = W.poiseuille(kn=0.05, cells=40, ppc=100, f32=False)
    parts = W.particles_for(prob)
    _say(f"[noalloc] channel FP64 n={parts['n']}")
    _case(prob, parts, 3)


def test_noalloc_rejects_capacity_beyond_scratch():
    """A capacity whose tile index does not fit the fixed array is rejected
    with USP_ESCRATCH in the host-side checks (the struct's arrays are
    stand-in addresses: nothing reaches a device)."""
    from paper_2508_05642_amd import usp
    L = usp.lib()
    f = _fn()
    prob = W.poiseuille(kn=0.05, cells=10, ppc=10, f32=True)
    g = usp.UspGrid(1, 1, 10, 0.0, 0.0, 1e-4, 1e-4, 1.0, 0x10, None)
    gas, bc = usp.make_gas(prob.gas), usp.make_bc(prob.bc)
    a = [0x1000_0000 + 0x1000 * k for k in range(10)]
    p = usp.UspParticles(usp.USP_F32, 4_000_000_000, *a)
    assert f(ctypes.byref(g), ctypes.byref(gas), ctypes.byref(bc), 1e-8, 0x10, 0x10,
             ctypes.byref(p), 1, 0, None, None) == ESCRATCH
    assert L.usp_status_str(ESCRATCH).startswith(b"problem too large")
