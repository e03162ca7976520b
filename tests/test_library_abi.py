"""The C-ABI library loads and exports every function include/usp.h
declares (no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "usp.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(usp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_seven_entry_points():
    d = declared()
    for nm in ("usp_bin", "usp_moments", "usp_reconstruct", "usp_collide", "usp_conserve",
               "usp_advect", "usp_step"):
        assert nm in d


def test_library_exports_every_declared_symbol():
    from paper_2508_05642_amd import build as B
    if not os.path.exists(B.LIB):
        B.build(force=True)
    L = ctypes.CDLL(B.LIB)
    for nm in declared():
        assert hasattr(L, nm), nm


def test_host_side_queries_and_validation():
    from paper_2508_05642_amd import usp
    L = usp.lib()
    assert usp.names("cs")[0] == "NP" and len(usp.names("cs")) == usp.NCS
    assert usp.names("mom")[-1] == "QIZ"
    assert usp.names("cnt")[10] == "INJECTED"
    assert L.usp_status_str(-1) == b"invalid argument"
    g = usp.UspGrid(2, 10, 5, 0.0, 0.0, 0.1, 0.1, 1.0, 1, None)
    assert L.usp_workspace_bytes(ctypes.byref(g), 1000) > 0
    bad = usp.UspGrid(2, 0, 5, 0.0, 0.0, 0.1, 0.1, 1.0, 1, None)
    assert L.usp_workspace_bytes(ctypes.byref(bad), 1000) == 0
    # host-side checks fire before any device work: null structs
    assert L.usp_bin(None, None, None, None, None, None, 0, None, None) == -1
    assert L.usp_step(None, None, None, 1.0, None, None, None, None, None, None, None, None, 0, 0,
                      0, 1, None, None) == -1
    assert L.usp_sample_fields(None, None, None, None) == -1
    assert L.usp_sample_fields(ctypes.byref(g), None, None, None) == -1


def test_surface_element_count():
    """2 nx + 2 ny wall elements plus the requested cylinder elements; a
    negative element count or a bad grid gives 0."""
    from paper_2508_05642_amd import usp
    import usp_workloads as W
    g = usp.UspGrid(2, 10, 5, 0.0, 0.0, 0.1, 0.1, 1.0, 1, None)
    b = usp.make_bc(W.BC(), None, 36)
    assert usp.usp_surf_elements(g, b) == 2 * 10 + 2 * 5 + 36
    b.surf_nbody = -1
    assert usp.usp_surf_elements(g, b) == 0
    bad = usp.UspGrid(2, 0, 5, 0.0, 0.0, 0.1, 0.1, 1.0, 1, None)
    assert usp.usp_surf_elements(bad, usp.make_bc(W.BC())) == 0


def test_binding_rejects_host_tensors_before_any_call():
    """The Python wrappers check every array argument (a contiguous GPU
    tensor of the declared dtype and length) and raise ValueError before
    anything is enqueued; host tensors never reach the library."""
    import torch
    from paper_2508_05642_amd import usp
    g = usp.UspGrid(2, 10, 5, 0.0, 0.0, 0.1, 0.1, 1.0, None, None)
    M = 50
    p = usp.UspParticles()
    host = dict(offsets=torch.zeros(M + 1, dtype=torch.int64),
                mom=torch.zeros(usp.NMOM * M, dtype=torch.float64))
    with pytest.raises(ValueError, match="offsets: expected a tensor on a GPU"):
        usp.usp_moments(g, p, host["offsets"], host["mom"])
    with pytest.raises(ValueError, match="a tensor is required"):
        usp.usp_moments(g, p, None, host["mom"])
    with pytest.raises(ValueError, match="ws: expected a tensor on a GPU"):
        usp.usp_advect(g, usp.UspGas(), usp.UspBC(), 1e-6, p, 0, 0,
                       torch.zeros(16, dtype=torch.uint8), None)


def _fake_parts(usp, cap, base):
    """A particle struct whose arrays are non-null stand-in addresses: only
    for calls that must fail in the host-side checks, before any enqueue."""
    a = [base + 0x1000 * k for k in range(10)]
    return usp.UspParticles(usp.USP_F32, cap, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7],
                            a[8], a[9])


def test_step_rejects_unequal_buffer_capacities():
    """usp_step moves the state between its two buffers every step, so the
    buffers must hold the same number of slots: a larger second buffer
    would let the injection fill slots the first cannot take on the next
    bin.  Unequal capacities, and buffers that share arrays or the count,
    are rejected with USP_EINVAL on the host."""
    from paper_2508_05642_amd import usp
    import usp_workloads as W
    L = usp.lib()
    prob = W.poiseuille(kn=0.05, cells=10, ppc=10, f32=True)
    g = usp.UspGrid(1, 1, 10, 0.0, 0.0, 1e-4, 1e-4, 1.0, 0x10, None)
    gas, bc = usp.make_gas(prob.gas), usp.make_bc(prob.bc)
    fake = 0x7000_0000

    def step(p, q):
        return L.usp_step(ctypes.byref(g), ctypes.byref(gas), ctypes.byref(bc), 1e-8, None,
                          ctypes.byref(p), ctypes.byref(q), fake, None, fake, fake, fake,
                          1 << 40, 1, 0, 1, None, None)
    assert step(_fake_parts(usp, 100, 0x1000_0000), _fake_parts(usp, 200, 0x2000_0000)) == -1
    assert step(_fake_parts(usp, 200, 0x1000_0000), _fake_parts(usp, 100, 0x2000_0000)) == -1
    # shared count
    p, q = _fake_parts(usp, 100, 0x1000_0000), _fake_parts(usp, 100, 0x2000_0000)
    q.count = p.count
    assert step(p, q) == -1


def test_check_statuses_and_host_validation():
    """usp_check reports USP_ENUMERIC and USP_ECAPACITY by name and
    rejects a missing counters array on the host."""
    from paper_2508_05642_amd import usp
    L = usp.lib()
    assert L.usp_status_str(-4) == b"NaN or infinite value in the state"
    assert b"capacity" in L.usp_status_str(-3)
    assert usp.names("cnt")[16] == "NONFINITE" and usp.NCOUNTERS == 17
    g = usp.UspGrid(1, 1, 10, 0.0, 0.0, 1e-4, 1e-4, 1.0, 0x10, None)
    p = _fake_parts(usp, 100, 0x1000_0000)
    assert L.usp_check(ctypes.byref(g), ctypes.byref(p), None, None, None, None, None) == -1
    assert L.usp_check(None, ctypes.byref(p), None, None, 0x10, None, None) == -1
