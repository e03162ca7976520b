"""Python binding of libusp (the C ABI declared in include/usp.h).

Argument marshalling only: every step of the particle update runs in the
HIP kernels of libusp.so.  Tensors are PyTorch device tensors (PyTorch is
used for device memory and streams).  The functions keep the C names:
usp_bin, usp_moments, usp_reconstruct, usp_collide, usp_conserve,
usp_advect, usp_step.  If libusp.so is missing the import of this module
fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libusp.so")

USP_F32, USP_F64 = 0, 1
NMOM, NCS, NCOUNTERS = 21, 39, 17
NSAMP, SURF_NQ = 21, 9
SURF_HITS, SURF_PX, SURF_PY, SURF_PZ, SURF_PN, SURF_PT, SURF_ETR, SURF_EROT, SURF_QVIB = range(9)
SURF_P_SCALE, SURF_E_SCALE = 65536.0, 16.0


class UspGas(C.Structure):
    _fields_ = [("m", C.c_double), ("theta_vib", C.c_double), ("T_ref", C.c_double),
                ("mu_ref", C.c_double), ("omega", C.c_double), ("alpha_vss", C.c_double),
                ("zrot_model", C.c_int32), ("Z_rot", C.c_double), ("Z_rot_inf", C.c_double),
                ("T_star", C.c_double), ("zvib_model", C.c_int32), ("Z_vib", C.c_double),
                ("C1", C.c_double), ("C2", C.c_double), ("sigma_vib", C.c_double),
                ("d_ref", C.c_double), ("pr_model", C.c_int32), ("Pr_const", C.c_double),
                ("scheme", C.c_int32), ("gamma_scope", C.c_int32), ("alpha_sign", C.c_int32)]


class UspGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("fnum", C.c_double), ("volume", C.c_void_p), ("flags", C.c_void_p)]


class UspBC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 4), ("Tw", C.c_double * 4), ("fs_n", C.c_double),
                ("fs_T", C.c_double), ("fs_U", C.c_double * 3), ("depth", C.c_double),
                ("cyl", C.c_int32), ("cyl_xc", C.c_double), ("cyl_yc", C.c_double),
                ("cyl_r", C.c_double), ("cyl_Tw", C.c_double), ("g", C.c_double * 3),
                ("surf", C.c_void_p), ("surf_nbody", C.c_int32)]


class UspParticles(C.Structure):
    _fields_ = [("prec", C.c_int32), ("capacity", C.c_int64), ("x", C.c_void_p),
                ("y", C.c_void_p), ("cx", C.c_void_p), ("cy", C.c_void_p), ("cz", C.c_void_p),
                ("erot", C.c_void_p), ("vib", C.c_void_p), ("cell", C.c_void_p),
                ("pid", C.c_void_p), ("count", C.c_void_p)]


_lib = None


def lib():
    """The loaded libusp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2508_05642_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, d, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double,
                                    C.c_size_t)
        L.usp_status_str.argtypes = [i32]
        L.usp_status_str.restype = C.c_char_p
        for nm in ("usp_mom_name", "usp_cs_name", "usp_counter_name"):
            getattr(L, nm).argtypes = [i32]
            getattr(L, nm).restype = C.c_char_p
        L.usp_version.restype = C.c_char_p
        L.usp_workspace_bytes.argtypes = [vp, i64]
        L.usp_workspace_bytes.restype = sz
        L.usp_cellstate_bytes.argtypes = [vp]
        L.usp_cellstate_bytes.restype = sz
        L.usp_surf_elements.argtypes = [vp, vp]
        L.usp_surf_elements.restype = i64
        L.usp_sample_fields.argtypes = [vp, vp, vp, vp]
        L.usp_bin_gather.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp, vp]
        L.usp_moments_gather.argtypes = [vp, vp, vp, vp, vp, vp]
        L.usp_update_gather.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, vp, vp, sz, u64, u64, vp, vp,
                                        vp, vp]
        L.usp_check.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.usp_bin.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, vp]
        L.usp_moments.argtypes = [vp, vp, vp, vp, vp]
        L.usp_reconstruct.argtypes = [vp, vp, vp, d, vp, vp, vp, vp]
        L.usp_collide.argtypes = [vp, vp, vp, vp, vp, u64, u64, vp, vp]
        L.usp_conserve.argtypes = [vp, vp, vp, vp, vp, u64, u64, vp, vp]
        L.usp_advect.argtypes = [vp, vp, vp, d, vp, u64, u64, vp, sz, vp, vp]
        L.usp_update.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, sz, u64, u64, vp, vp]
        L.usp_batch.argtypes = [vp, vp, d, vp, vp, vp, vp, vp, vp, sz, i32, i32, u64, u64, i32, vp,
                                vp]
        L.usp_step.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, vp, vp, vp, vp, sz, u64, u64, i32, vp,
                               vp]
        L.usp_tape_bytes.argtypes = [vp, i64]
        L.usp_tape_bytes.restype = sz
        L.usp_adjoint_ws_bytes.argtypes = [vp, i64]
        L.usp_adjoint_ws_bytes.restype = sz
        L.usp_step_taped.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, vp, vp, vp, sz, u64, u64, vp,
                                     sz, vp, sz, vp, vp]
        L.usp_adjoint_step.argtypes = [vp, vp, vp, d, vp, sz, i64, u64, u64, vp, vp, d, d, vp, vp,
                                       sz, vp]
        for nm in ("usp_bin", "usp_bin_gather", "usp_moments_gather", "usp_update_gather",
                   "usp_moments", "usp_sample_fields", "usp_reconstruct", "usp_collide",
                   "usp_conserve", "usp_advect", "usp_update", "usp_batch", "usp_step",
                   "usp_step_taped", "usp_adjoint_step", "usp_check"):
            getattr(L, nm).restype = i32
        _lib = L
    return _lib


EXPORTED = ["usp_status_str", "usp_mom_name", "usp_cs_name", "usp_counter_name", "usp_version",
            "usp_workspace_bytes", "usp_cellstate_bytes", "usp_surf_elements", "usp_bin",
            "usp_bin_gather", "usp_moments_gather", "usp_update_gather",
            "usp_moments", "usp_sample_fields", "usp_reconstruct", "usp_collide", "usp_conserve",
            "usp_advect", "usp_update", "usp_batch", "usp_step", "usp_tape_bytes",
            "usp_adjoint_ws_bytes", "usp_step_taped", "usp_adjoint_step", "usp_check"]


def names(kind):
    fn = {"mom": lib().usp_mom_name, "cs": lib().usp_cs_name, "cnt": lib().usp_counter_name}[kind]
    n = {"mom": NMOM, "cs": NCS, "cnt": NCOUNTERS}[kind]
    return [fn(k).decode() for k in range(n)]


class UspError(RuntimeError):
    pass


def _check(st, what):
    if st != 0:
        raise UspError(f"{what}: {lib().usp_status_str(st).decode()} ({st})")


def _ptr(t):
    return None if t is None else t.data_ptr()


def _dev(t, dtype, n, what, optional=False):
    """Device pointer of tensor t after checking that it is a contiguous
    tensor on a GPU with the given dtype and at least n elements; raises
    ValueError before anything is enqueued."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: a tensor is required")
    if not torch.is_tensor(t) or not t.is_cuda:
        raise ValueError(f"{what}: expected a tensor on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} elements, at least {n} needed")
    return t.data_ptr()


def _ncells(grid):
    return int(grid.nx) * int(grid.ny)


def _offsets(grid, t, what="offsets", optional=False):
    return _dev(t, torch.int64, _ncells(grid) + 1, what, optional)


def _planes(grid, t, k, what):
    return _dev(t, torch.float64, k * _ncells(grid), what)


def _cs(grid, t):
    return _dev(t, torch.float64, lib().usp_cellstate_bytes(C.byref(grid)) // 8, "cs")


def _ws(t, what="ws"):
    _dev(t, torch.uint8, 0, what)
    return t.data_ptr(), t.numel()


def _cnt(t):
    return _dev(t, torch.int64, NCOUNTERS, "counters", optional=True)


def _perm(t, p):
    return _dev(t, torch.int32, int(p.capacity), "perm")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---- struct builders (duck-typed descriptions with the C field names) ----
def make_gas(g):
    return UspGas(g.m, g.theta_vib, g.T_ref, g.mu_ref, g.omega, g.alpha_vss, g.zrot_model,
                  g.Z_rot, g.Z_rot_inf, g.T_star, g.zvib_model, g.Z_vib, g.C1, g.C2,
                  g.sigma_vib, g.d_ref, g.pr_model, g.Pr_const, getattr(g, "scheme", 0),
                  getattr(g, "gamma_scope", 0), getattr(g, "alpha_sign", 0))


def make_bc(b, surf=None, surf_nbody=0):
    return UspBC((C.c_int32 * 4)(*b.kind), (C.c_double * 4)(*b.Tw), b.fs_n, b.fs_T,
                 (C.c_double * 3)(*b.fs_U), b.depth, b.cyl, b.cyl_xc, b.cyl_yc, b.cyl_r,
                 b.cyl_Tw, (C.c_double * 3)(*b.g), _ptr(surf), int(surf_nbody))


# ---- the seven entry points -------------------------------------------------
def usp_bin(grid, pin, pout, offsets, ws, counters, stream=None, in_offsets=None):
    _check(lib().usp_bin(C.byref(grid), C.byref(pin), C.byref(pout), _offsets(grid, offsets),
                         _offsets(grid, in_offsets, "in_offsets", True), *_ws(ws), _cnt(counters),
                         _stream(stream)), "usp_bin")


def usp_bin_gather(grid, pin, pout, offsets, perm, ws, counters, stream=None, in_offsets=None):
    _check(lib().usp_bin_gather(C.byref(grid), C.byref(pin), C.byref(pout), _offsets(grid, offsets),
                                _offsets(grid, in_offsets, "in_offsets", True), _perm(perm, pout),
                                *_ws(ws), _cnt(counters), _stream(stream)), "usp_bin_gather")


def usp_moments_gather(grid, pin, perm, offsets, mom, stream=None):
    _check(lib().usp_moments_gather(C.byref(grid), C.byref(pin), _perm(perm, pin),
                                    _offsets(grid, offsets), _planes(grid, mom, NMOM, "mom"),
                                    _stream(stream)), "usp_moments_gather")


def usp_update_gather(grid, gas, bc, dt, cs, offsets, pin, perm, pout, seed, step, ws, counters,
                      stream=None, events=None):
    """events: optional pair of raw hipEvent_t handles (ints) recorded just
    before and after the particle kernel itself."""
    ev0, ev1 = (None, None) if events is None else (C.c_void_p(events[0]), C.c_void_p(events[1]))
    _check(lib().usp_update_gather(C.byref(grid), C.byref(gas), None if bc is None else C.byref(bc),
                                   dt, _cs(grid, cs), _offsets(grid, offsets), C.byref(pin),
                                   _perm(perm, pin), C.byref(pout), *_ws(ws), seed, step,
                                   _cnt(counters), ev0, ev1, _stream(stream)), "usp_update_gather")


def usp_check(grid, p, mom, cs, counters, stream=None):
    """Scan p (and mom, cs when given) for NaN/Inf; waits for the stream.
    Returns (status, nonfinite values found by this scan); the status is
    USP_OK (0), USP_ENUMERIC (-4) or USP_ECAPACITY (-3); other statuses
    raise."""
    found = C.c_int64(0)
    st = lib().usp_check(C.byref(grid), C.byref(p),
                         None if mom is None else _planes(grid, mom, NMOM, "mom"),
                         None if cs is None else _cs(grid, cs),
                         _dev(counters, torch.int64, NCOUNTERS, "counters"), C.byref(found),
                         _stream(stream))
    if st not in (0, -3, -4):
        _check(st, "usp_check")
    return int(st), int(found.value)


def usp_moments(grid, p, offsets, mom, stream=None):
    _check(lib().usp_moments(C.byref(grid), C.byref(p), _offsets(grid, offsets),
                             _planes(grid, mom, NMOM, "mom"), _stream(stream)), "usp_moments")


def usp_sample_fields(grid, mom, acc, stream=None):
    _check(lib().usp_sample_fields(C.byref(grid), _planes(grid, mom, NMOM, "mom"),
                                   _planes(grid, acc, NSAMP, "acc"), _stream(stream)),
           "usp_sample_fields")


def usp_surf_elements(grid, bc):
    return int(lib().usp_surf_elements(C.byref(grid), C.byref(bc)))


def usp_reconstruct(grid, gas, mom, dt, dt_cell, cs, counters, stream=None):
    _check(lib().usp_reconstruct(C.byref(grid), C.byref(gas), _planes(grid, mom, NMOM, "mom"), dt,
                                 _dev(dt_cell, torch.float64, _ncells(grid), "dt_cell", True),
                                 _cs(grid, cs), _cnt(counters), _stream(stream)), "usp_reconstruct")


def usp_collide(grid, gas, cs, offsets, p, seed, step, counters, stream=None):
    _check(lib().usp_collide(C.byref(grid), C.byref(gas), _cs(grid, cs), _offsets(grid, offsets),
                             C.byref(p), seed, step, _cnt(counters), _stream(stream)), "usp_collide")


def usp_conserve(grid, gas, cs, offsets, p, seed, step, counters, stream=None):
    _check(lib().usp_conserve(C.byref(grid), C.byref(gas), _cs(grid, cs), _offsets(grid, offsets),
                              C.byref(p), seed, step, _cnt(counters), _stream(stream)), "usp_conserve")


def usp_batch(grid, gas, dt, dt_cell, p, offsets, mom, cs, ws, tile, steps_per_launch, seed, step,
              nsteps, counters, stream=None):
    _check(lib().usp_batch(C.byref(grid), C.byref(gas), dt,
                           _dev(dt_cell, torch.float64, _ncells(grid), "dt_cell", True), C.byref(p),
                           _offsets(grid, offsets), _planes(grid, mom, NMOM, "mom"), _cs(grid, cs),
                           *_ws(ws), tile, steps_per_launch, seed, step, nsteps, _cnt(counters),
                           _stream(stream)), "usp_batch")


def usp_update(grid, gas, bc, dt, cs, offsets, p, seed, step, ws, counters, stream=None):
    _check(lib().usp_update(C.byref(grid), C.byref(gas), None if bc is None else C.byref(bc), dt,
                            _cs(grid, cs), _offsets(grid, offsets), C.byref(p), *_ws(ws), seed,
                            step, _cnt(counters), _stream(stream)), "usp_update")


def usp_advect(grid, gas, bc, dt, p, seed, step, ws, counters, stream=None):
    _check(lib().usp_advect(C.byref(grid), C.byref(gas), C.byref(bc), dt, C.byref(p), seed, step,
                            *_ws(ws), _cnt(counters), _stream(stream)), "usp_advect")


def usp_step(grid, gas, bc, dt, dt_cell, p, p_alt, offsets, mom, cs, ws, seed, step, nsteps,
             counters, stream=None, in_offsets=None):
    """nsteps full steps; p and p_alt (UspParticles) are swapped in place as
    the library swaps them, so p describes the current state afterwards.
    in_offsets: the segments of an already binned input (usp_bin's)."""
    _check(lib().usp_step(C.byref(grid), C.byref(gas), C.byref(bc) if bc is not None else None,
                          dt, _dev(dt_cell, torch.float64, _ncells(grid), "dt_cell", True),
                          C.byref(p), C.byref(p_alt), _offsets(grid, offsets),
                          _offsets(grid, in_offsets, "in_offsets", True),
                          _planes(grid, mom, NMOM, "mom"), _cs(grid, cs), *_ws(ws), seed, step,
                          nsteps, _cnt(counters), _stream(stream)), "usp_step")


def usp_step_taped(grid, gas, bc, dt, p, p_alt, offsets, mom, cs, ws, seed, step, tape, aws,
                   counters, stream=None, in_offsets=None):
    """One step with its tape; p and p_alt are swapped in place as the
    library swaps them."""
    _check(lib().usp_step_taped(C.byref(grid), C.byref(gas), C.byref(bc), dt, C.byref(p),
                                C.byref(p_alt), _offsets(grid, offsets),
                                _offsets(grid, in_offsets, "in_offsets", True),
                                _planes(grid, mom, NMOM, "mom"), _cs(grid, cs), *_ws(ws), seed,
                                step, *_ws(tape, "tape"), *_ws(aws, "aws"), _cnt(counters),
                                _stream(stream)), "usp_step_taped")


def usp_adjoint_step(grid, gas, bc, dt, tape, capacity, seed, step, lam_in, lam_out, w_mdot,
                     w_tau, grad, aws, stream=None):
    nl = 2 * 5 * int(capacity)
    _check(lib().usp_adjoint_step(C.byref(grid), C.byref(gas), C.byref(bc), dt,
                                  *_ws(tape, "tape"), capacity, seed, step,
                                  _dev(lam_in, torch.float64, nl, "lam_in"),
                                  _dev(lam_out, torch.float64, nl, "lam_out"), w_mdot, w_tau,
                                  _dev(grad, torch.float64, 6, "grad"), *_ws(aws, "aws"),
                                  _stream(stream)), "usp_adjoint_step")


# ---- device-resident state for one problem ---------------------------------
class DeviceState:
    """Device buffers for one problem: two particle buffers, offsets,
    moments, cell state, workspace and counters.  `prob` carries gas, grid,
    bc, dt, dt_cell, seed and f32 (field names as in the C structs)."""

    FIELDS = ("x", "y", "cx", "cy", "cz", "erot")

    def __init__(self, prob, parts, device="cuda", capacity=None):
        self.prob = prob
        self.dev = torch.device(device)
        g = prob.grid
        self.M = g.nx * g.ny
        self.dim = g.dim
        self.prec = USP_F32 if prob.f32 else USP_F64
        self.fdt = torch.float32 if prob.f32 else torch.float64
        cap = int(capacity or parts["cap"])
        self.cap = cap
        self.volume = torch.as_tensor(np.ascontiguousarray(g.volume, np.float64), device=self.dev)
        flags = g.flags if g.flags is not None else np.zeros(self.M, np.uint8)
        self.flags = torch.as_tensor(np.ascontiguousarray(flags, np.uint8), device=self.dev)
        self.grid = UspGrid(g.dim, g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.fnum,
                            self.volume.data_ptr(), self.flags.data_ptr())
        self.gas = make_gas(prob.gas)
        self.bc = make_bc(prob.bc)
        self.dt_cell = (None if prob.dt_cell is None else
                        torch.as_tensor(np.asarray(prob.dt_cell, np.float64), device=self.dev))
        self.bufs = [self._alloc(), self._alloc()]
        self.load(parts)
        self.offsets = torch.zeros(self.M + 1, dtype=torch.int64, device=self.dev)
        self.mom = torch.zeros(NMOM * self.M, dtype=torch.float64, device=self.dev)
        csb = lib().usp_cellstate_bytes(C.byref(self.grid))
        self.cs = torch.zeros(csb // 8, dtype=torch.float64, device=self.dev)
        wsb = lib().usp_workspace_bytes(C.byref(self.grid), cap)
        if wsb == 0:
            raise UspError("usp_workspace_bytes rejected the grid/capacity")
        self.ws = torch.zeros(wsb, dtype=torch.uint8, device=self.dev)
        self.counters = torch.zeros(NCOUNTERS, dtype=torch.int64, device=self.dev)
        self.fields = None
        self.surf = None
        self.perm = torch.zeros(cap, dtype=torch.int32, device=self.dev)  # uint32 bits
        self.gathered = False

    def enable_sampling(self, nbody=0):
        """Zeroed field sums (double[NSAMP, M]) and surface sums (int64
        [usp_surf_elements, SURF_NQ]); from now on every diffuse re-emission
        is sampled, and sample_fields() adds the current moments."""
        self.bc = make_bc(self.prob.bc, None, nbody)
        ne = usp_surf_elements(self.grid, self.bc)
        if ne <= 0:
            raise UspError("usp_surf_elements rejected the grid/bc")
        self.surf = torch.zeros(ne * SURF_NQ, dtype=torch.int64, device=self.dev)
        self.fields = torch.zeros(NSAMP * self.M, dtype=torch.float64, device=self.dev)
        self.bc = make_bc(self.prob.bc, self.surf, nbody)

    def sample_fields(self, stream=None):
        """Add the moments in `mom` (the last step's pre-collision state) to
        the field sums."""
        usp_sample_fields(self.grid, self.mom, self.fields, stream)

    def field_sums(self):
        return self.fields.view(NSAMP, self.M).cpu().numpy()

    def surface_sums(self):
        return self.surf.view(-1, SURF_NQ).cpu().numpy()

    def _alloc(self):
        cap, dev, f = self.cap, self.dev, self.fdt
        b = {k: torch.zeros(cap, dtype=f, device=dev) for k in ("cx", "cy", "cz", "erot")}
        b["x"] = torch.zeros(cap, dtype=f, device=dev) if self.dim == 2 else None
        b["y"] = torch.zeros(cap, dtype=f, device=dev) if self.dim >= 1 else None
        b["vib"] = torch.zeros(cap, dtype=torch.uint8, device=dev)
        b["cell"] = torch.full((cap,), -1, dtype=torch.int32, device=dev)
        b["pid"] = torch.zeros(cap, dtype=torch.int32, device=dev)  # uint32 bits
        b["count"] = torch.zeros(2, dtype=torch.int64, device=dev)
        b["struct"] = UspParticles(self.prec, cap, _ptr(b["x"]), _ptr(b["y"]), _ptr(b["cx"]),
                                   _ptr(b["cy"]), _ptr(b["cz"]), _ptr(b["erot"]), _ptr(b["vib"]),
                                   _ptr(b["cell"]), _ptr(b["pid"]), _ptr(b["count"]))
        return b

    def load(self, parts):
        """Copy a host particle dict into buffer 0 (the current one)."""
        n = int(parts["n"])
        if n > self.cap:
            raise ValueError("more particles than capacity")
        B = self.bufs[0]
        for k in self.FIELDS:
            if B[k] is not None:
                src = parts.get(k)
                if src is None:
                    raise ValueError(f"particle array {k} required for dim {self.dim}")
                B[k][:n] = torch.as_tensor(np.asarray(src[:n]), dtype=self.fdt)
        vib = np.asarray(parts["vib"][:n])
        if vib.size and (vib.min() < 0 or vib.max() > 255):
            raise ValueError("vibrational levels must be in [0, 255]")
        B["vib"][:n] = torch.as_tensor(vib.astype(np.uint8))
        B["cell"][:n] = torch.as_tensor(np.asarray(parts["cell"][:n], np.int32))
        B["pid"][:n] = torch.as_tensor(np.asarray(parts["pid"][:n]).astype(np.uint32).view(np.int32))
        B["count"][:] = torch.tensor([n, int(parts["next_pid"])], dtype=torch.int64)
        self.cur = 0
        self.binned = False

    @property
    def p(self):
        return self.bufs[self.cur]["struct"]

    @property
    def p_alt(self):
        return self.bufs[1 - self.cur]["struct"]

    def state(self):
        """Host copy of the current particle state (numpy, first n entries)."""
        torch.cuda.synchronize()
        B = self.bufs[self.cur]
        n, nxt = (int(v) for v in B["count"].cpu())
        out = {"n": n, "next_pid": nxt}
        for k in self.FIELDS:
            out[k] = None if B[k] is None else B[k][:n].cpu().numpy().astype(np.float64)
        out["vib"] = B["vib"][:n].cpu().numpy().astype(np.int32)
        out["cell"] = B["cell"][:n].cpu().numpy()
        out["pid"] = B["pid"][:n].cpu().numpy().view(np.uint32)
        return out

    def moments(self):
        return self.mom.view(NMOM, self.M).cpu().numpy()

    def cellstate(self):
        return self.cs[: NCS * self.M].view(NCS, self.M).cpu().numpy()

    def cnt(self):
        return dict(zip(names("cnt"), self.counters.cpu().tolist()))

    # -- phases (the C entry points on this state) ------------------------
    def bin(self, stream=None, use_offsets=True, gather=False):
        """Rebin the current state.  Once this state has been binned, the
        previous offsets describe its prefix (the phases keep the order) and
        are passed on, unless use_offsets is False.  With gather the order
        is only recorded (usp_bin_gather): do_moments and update then read
        through it, and update writes the new state to the other buffer."""
        prev = self.offsets if (use_offsets and self.binned) else None
        if gather:
            usp_bin_gather(self.grid, self.p, self.p_alt, self.offsets, self.perm, self.ws,
                           self.counters, stream, in_offsets=prev)
            self.gathered = True
        else:
            usp_bin(self.grid, self.p, self.p_alt, self.offsets, self.ws, self.counters, stream,
                    in_offsets=prev)
            self.cur = 1 - self.cur
        self.binned = True

    def do_moments(self, stream=None):
        if self.gathered:
            usp_moments_gather(self.grid, self.p, self.perm, self.offsets, self.mom, stream)
        else:
            usp_moments(self.grid, self.p, self.offsets, self.mom, stream)

    def do_reconstruct(self, stream=None):
        usp_reconstruct(self.grid, self.gas, self.mom, self.prob.dt, self.dt_cell, self.cs,
                        self.counters, stream)

    def collide(self, step, stream=None):
        self._not_gathered("collide")
        usp_collide(self.grid, self.gas, self.cs, self.offsets, self.p, self.prob.seed, step,
                    self.counters, stream)

    def conserve(self, step, stream=None):
        self._not_gathered("conserve")
        usp_conserve(self.grid, self.gas, self.cs, self.offsets, self.p, self.prob.seed, step,
                     self.counters, stream)

    def advect(self, step, stream=None):
        self._not_gathered("advect")
        usp_advect(self.grid, self.gas, self.bc, self.prob.dt, self.p, self.prob.seed, step,
                   self.ws, self.counters, stream)

    def update(self, step, stream=None, events=None):
        """collide + conserve + advect in one fused pass (binned state, or
        the recorded order of a gathering bin; `events` as for
        usp_update_gather)."""
        bc = self.bc if self.dim >= 1 else None
        if self.gathered:
            usp_update_gather(self.grid, self.gas, bc, self.prob.dt, self.cs, self.offsets, self.p,
                              self.perm, self.p_alt, self.prob.seed, step, self.ws, self.counters,
                              stream, events)
            self.cur = 1 - self.cur
            self.gathered = False
            return
        usp_update(self.grid, self.gas, bc, self.prob.dt, self.cs, self.offsets, self.p,
                   self.prob.seed, step, self.ws, self.counters, stream)

    def _not_gathered(self, what):
        if self.gathered:
            raise UspError(f"{what}: the state is between a gathering bin and its update")

    def step(self, step, nsteps=1, stream=None):
        self._not_gathered("step")
        a, b = self.bufs[self.cur]["struct"], self.bufs[1 - self.cur]["struct"]
        usp_step(self.grid, self.gas, self.bc if self.dim >= 1 else None, self.prob.dt,
                 self.dt_cell, a, b, self.offsets, self.mom, self.cs, self.ws, self.prob.seed,
                 step, nsteps, self.counters, stream,
                 in_offsets=self.offsets if self.binned else None)
        if nsteps > 0:
            self.binned = True
        # the library swapped the struct contents once per rebin: a now
        # describes the buffer that holds the state
        if a.cx != self.bufs[self.cur]["cx"].data_ptr():
            B0, B1 = self.bufs[self.cur], self.bufs[1 - self.cur]
            B0["struct"], B1["struct"] = B1["struct"], B0["struct"]
            self.cur = 1 - self.cur

    def check(self, stream=None):
        """usp_check of the current state, its moments and cell state:
        (status, non-finite values found)."""
        return usp_check(self.grid, self.p, self.mom, self.cs, self.counters, stream)

    def step_taped(self, step, tape, aws, stream=None):
        """One step (the bits of step()) that also writes its tape."""
        a, b = self.bufs[self.cur]["struct"], self.bufs[1 - self.cur]["struct"]
        usp_step_taped(self.grid, self.gas, self.bc, self.prob.dt, a, b, self.offsets, self.mom,
                       self.cs, self.ws, self.prob.seed, step, tape, aws, self.counters, stream,
                       in_offsets=self.offsets if self.binned else None)
        self.binned = True
        if a.cx != self.bufs[self.cur]["cx"].data_ptr():
            B0, B1 = self.bufs[self.cur], self.bufs[1 - self.cur]
            B0["struct"], B1["struct"] = B1["struct"], B0["struct"]
            self.cur = 1 - self.cur

    def batch(self, step, nsteps, tile=0, steps_per_launch=0, stream=None):
        """nsteps steps of a binned 0D state with usp_batch (same bits as
        step())."""
        usp_batch(self.grid, self.gas, self.prob.dt, self.dt_cell, self.p, self.offsets, self.mom,
                  self.cs, self.ws, tile, steps_per_launch, self.prob.seed, step, nsteps,
                  self.counters, stream)
