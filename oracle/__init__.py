"""Python access to the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the oracle is the plain FP64 reference of the
USP-FPM step that the GPU library is checked against.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg import this package.
It shares no code with the GPU library; inputs come from ``usp_workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "usp_oracle.c")

MOM_NAMES = ["N", "UX", "UY", "UZ", "PXX", "PYY", "PZZ", "PXY", "PXZ", "PYZ", "EROT", "IBAR",
             "QTRX", "QTRY", "QTRZ", "QROTX", "QROTY", "QROTZ", "QIX", "QIY", "QIZ"]
CS_NAMES = ["NP", "NDENS", "UX", "UY", "UZ", "TTR", "TROT", "TVIB",
            "PXX", "PYY", "PZZ", "PXY", "PXZ", "PYZ", "ETR", "EROT", "EVIB",
            "MU", "MUP", "TAUC", "ZROT", "ZVIB", "PR", "DT", "A", "B", "R2", "R3",
            "ALPHA", "OMA2", "NU", "EROT_NEW", "EVIB_NEW", "COLLIDE", "NBR_OK",
            "FPM_TAU", "FPM_TTR_REL", "FPM_TROT_REL", "FPM_MREL"]
CNT_NAMES = ["PB_CLAMP", "CHOL_FALLBACK", "NU_ZERO", "TREL_SKIP", "TREL_CLAMP", "VIB_SAT",
             "INTERP_CLAMP", "CONS_SKIP", "PICK_FAIL", "CELL_SKIP", "INJECTED", "DELETED",
             "WALL_HITS", "BOUNCE_LIMIT", "CAPACITY", "SOLID_DROP", "NONFINITE"]
NMOM, NCS, NCNT = len(MOM_NAMES), len(CS_NAMES), len(CNT_NAMES)
SAMP_NAMES = ["N", "CX", "CY", "CZ", "CXX", "CYY", "CZZ", "CXY", "CXZ", "CYZ", "EROT", "I",
              "HC2CX", "HC2CY", "HC2CZ", "CXEROT", "CYEROT", "CZEROT", "CXI", "CYI", "CZI"]
SURF_NAMES = ["HITS", "PX", "PY", "PZ", "PN", "PT", "ETR", "EROT", "QVIB"]
NSAMP, SURF_NQ = len(SAMP_NAMES), len(SURF_NAMES)
SURF_P_SCALE, SURF_E_SCALE = 65536.0, 16.0

PD = C.POINTER(C.c_double)


class OrcGas(C.Structure):
    _fields_ = [("m", C.c_double), ("theta_vib", C.c_double), ("T_ref", C.c_double),
                ("mu_ref", C.c_double), ("omega", C.c_double), ("alpha_vss", C.c_double),
                ("zrot_model", C.c_int32), ("Z_rot", C.c_double), ("Z_rot_inf", C.c_double),
                ("T_star", C.c_double), ("zvib_model", C.c_int32), ("Z_vib", C.c_double),
                ("C1", C.c_double), ("C2", C.c_double), ("sigma_vib", C.c_double),
                ("d_ref", C.c_double), ("pr_model", C.c_int32), ("Pr_const", C.c_double),
                ("scheme", C.c_int32), ("gamma_scope", C.c_int32), ("alpha_sign", C.c_int32)]


class OrcGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("fnum", C.c_double), ("volume", C.c_void_p), ("flags", C.c_void_p)]


class OrcBC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 4), ("Tw", C.c_double * 4), ("fs_n", C.c_double),
                ("fs_T", C.c_double), ("fs_U", C.c_double * 3), ("depth", C.c_double),
                ("cyl", C.c_int32), ("cyl_xc", C.c_double), ("cyl_yc", C.c_double),
                ("cyl_r", C.c_double), ("cyl_Tw", C.c_double), ("g", C.c_double * 3),
                ("surf", C.c_void_p), ("surf_nbody", C.c_int32)]


class OrcParts(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("cx", C.c_void_p), ("cy", C.c_void_p),
                ("cz", C.c_void_p), ("erot", C.c_void_p), ("vib", C.c_void_p),
                ("cell", C.c_void_p), ("pid", C.c_void_p), ("next_pid", C.c_uint64)]


# With ORACLE_SANITIZE=1 in the environment the oracle is built and loaded
# as liboracle_san.so, instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (every finding aborts).  The Python process
# must then preload the ASan runtime, e.g.
#   ORACLE_SANITIZE=1 LD_PRELOAD=$(gcc -print-file-name=libasan.so) \
#   ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu"
SANITIZE = os.environ.get("ORACLE_SANITIZE", "") not in ("", "0")
if SANITIZE:
    _LIB = os.path.join(_HERE, "liboracle_san.so")


def build(force=False):
    """Compile liboracle.so with gcc (plain C11, FP64, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-o", _LIB, _SRC, "-lm"]
    if SANITIZE:
        cmd[1:1] = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        vp, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        for nm in ["orc_R", "orc_tau_c_factor"]:
            getattr(L, nm).argtypes = [vp]
            getattr(L, nm).restype = d
        for nm in ["orc_e_vib", "orc_cv_vib", "orc_viscosity", "orc_zrot", "orc_zvib", "orc_prandtl"]:
            getattr(L, nm).argtypes = [vp, d]
            getattr(L, nm).restype = d
        L.orc_tcheck.argtypes = [vp, d, d, d, d, d]
        L.orc_tcheck.restype = d
        L.orc_gammas.argtypes = [vp, d, d, d, d, d, vp, vp]
        L.orc_eigvals_sym3.argtypes = [vp, vp]
        L.orc_particle_coef.argtypes = [vp, d, d, d, vp] + [d] * 9 + [vp]
        L.orc_bin.argtypes = [vp, vp, vp, vp, i32, vp]
        L.orc_moments.argtypes = [vp, vp, vp, vp, vp]
        L.orc_cellstate.argtypes = [vp, vp, vp, d, vp, vp]
        L.orc_interp.argtypes = [vp, vp, C.c_int, i32, d, d]
        L.orc_interp.restype = d
        L.orc_collide.argtypes = [vp, vp, vp, vp, vp, u64, u64, i32, vp]
        L.orc_conserve.argtypes = [vp, vp, vp, vp, vp, u64, u64, i32, vp]
        L.orc_advect.argtypes = [vp, vp, vp, d, vp, u64, u64, i32, vp]
        L.orc_sample_fields.argtypes = [vp, vp, vp, vp]
        L.orc_collide_normals.argtypes = [u64, u64, i64, vp, vp]
        L.orc_step.argtypes = [vp, vp, vp, d, vp, vp, vp, vp, vp, vp, u64, u64, i32, i32, vp]
        L.orc_sample_nb.argtypes = [d, i32, d]
        L.orc_sample_nb.restype = i32
        L.orc_sample_b.argtypes = [d, i32, d]
        L.orc_sample_b.restype = i32
        L.orc_inflow_speed.argtypes = [u64, u64, C.c_uint32, d]
        L.orc_inflow_speed.restype = d
        L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32).copy()
    k = np.asarray(key, np.uint32).copy()
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def make_gas(g):
    return OrcGas(g.m, g.theta_vib, g.T_ref, g.mu_ref, g.omega, g.alpha_vss, g.zrot_model,
                  g.Z_rot, g.Z_rot_inf, g.T_star, g.zvib_model, g.Z_vib, g.C1, g.C2,
                  g.sigma_vib, g.d_ref, g.pr_model, g.Pr_const, getattr(g, "scheme", 0),
                  getattr(g, "gamma_scope", 0), getattr(g, "alpha_sign", 0))


class Gas:
    """Scalar gas-model functions of the oracle."""

    def __init__(self, gas):
        self.s = make_gas(gas)
        self.ref = C.byref(self.s)

    def R(self): return lib().orc_R(self.ref)
    def e_vib(self, T): return lib().orc_e_vib(self.ref, T)
    def cv_vib(self, T): return lib().orc_cv_vib(self.ref, T)
    def viscosity(self, T): return lib().orc_viscosity(self.ref, T)
    def tau_c_factor(self): return lib().orc_tau_c_factor(self.ref)
    def zrot(self, T): return lib().orc_zrot(self.ref, T)
    def zvib(self, T): return lib().orc_zvib(self.ref, T)
    def prandtl(self, T): return lib().orc_prandtl(self.ref, T)

    def tau_c(self, T, n):
        return self.tau_c_factor() * self.viscosity(T) / (n * 1.380649e-23 * T)

    def tcheck(self, Ttr, Trot, Tvib, a, b):
        return lib().orc_tcheck(self.ref, Ttr, Trot, Tvib, a, b)

    def gammas(self, Ttr, Trot, Tvib, a, b):
        out = np.zeros(3)
        tc = C.c_double(0.0)
        lib().orc_gammas(self.ref, Ttr, Trot, Tvib, a, b, _p(out), C.byref(tc))
        return out, tc.value


class OrcPCoef(C.Structure):
    _fields_ = [("L", C.c_double * 6), ("al", C.c_double), ("oma2", C.c_double),
                ("nu", C.c_double), ("nu_bound", C.c_double), ("Ttr_rel", C.c_double),
                ("Trot_rel", C.c_double), ("mstar", C.c_double), ("fallback", C.c_int32),
                ("nu_zero", C.c_int32), ("skip", C.c_int32)]


def particle_coef(gas, Ttr, Trot, Tvib, P, a, b, al, oma2, nu, r2, A2, Pr, dt):
    """orc_particle_coef (Secs. III.A.1-III.A.3) for one particle: its
    interpolated temperatures and Pi (xx, yy, zz, xy, xz, yz), and the cell
    coefficients; returns the fields of orc_pcoef as a dict."""
    g = gas if isinstance(gas, Gas) else Gas(gas)
    P = np.ascontiguousarray(P, np.float64)
    out = OrcPCoef()
    lib().orc_particle_coef(g.ref, Ttr, Trot, Tvib, _p(P), a, b, al, oma2, nu, r2, A2, Pr, dt,
                            C.byref(out))
    r = {k: getattr(out, k) for k, _ in OrcPCoef._fields_ if k != "L"}
    r["L"] = np.array(out.L[:])
    return r


def eigvals_sym3(P):
    P = np.asarray(P, np.float64).copy()
    out = np.zeros(3)
    lib().orc_eigvals_sym3(_p(P), _p(out))
    return out


class Sim:
    """Oracle state for one problem: FP64 particle buffers (double-buffered),
    offsets, moments, cell state and event counters."""

    def __init__(self, prob, parts, threads=0):
        L = lib()
        if threads:
            L.orc_set_threads(threads)
        self.prob = prob
        self.f32 = 1 if prob.f32 else 0
        g = prob.grid
        self.M = g.ncells
        self._vol = np.ascontiguousarray(g.volume, np.float64)
        self._flags = np.ascontiguousarray(g.flags if g.flags is not None else np.zeros(self.M), np.uint8)
        self.grid = OrcGrid(g.dim, g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.fnum,
                            self._vol.ctypes.data, self._flags.ctypes.data)
        self.gas = make_gas(prob.gas)
        b = prob.bc
        self.bc = OrcBC((C.c_int32 * 4)(*b.kind), (C.c_double * 4)(*b.Tw), b.fs_n, b.fs_T,
                        (C.c_double * 3)(*b.fs_U), b.depth, b.cyl, b.cyl_xc, b.cyl_yc, b.cyl_r,
                        b.cyl_Tw, (C.c_double * 3)(*b.g), None, 0)
        self.surf = None
        self.fields = None
        self.dt_cell = None if prob.dt_cell is None else np.ascontiguousarray(prob.dt_cell, np.float64)
        cap = parts["cap"]
        self.cap = cap
        self.bufs = [self._alloc(cap, g.dim), self._alloc(cap, g.dim)]
        n = parts["n"]
        A = self.bufs[0]
        for k in ("x", "y", "cx", "cy", "cz", "erot"):
            if A[k] is not None and parts.get(k) is not None:
                A[k][:n] = parts[k][:n]
        A["vib"][:n] = parts["vib"][:n]
        A["cell"][:n] = parts["cell"][:n]
        A["pid"][:n] = parts["pid"][:n]
        self.structs = [self._struct(self.bufs[0], n, parts["next_pid"]),
                        self._struct(self.bufs[1], 0, parts["next_pid"])]
        self.cur = 0
        self.offsets = np.zeros(self.M + 1, np.int64)
        self.mom = np.zeros(NMOM * self.M)
        self.cs = np.zeros(NCS * self.M)
        self.counters = np.zeros(NCNT, np.int64)
        self.sorted = False

    @staticmethod
    def _alloc(cap, dim):
        f = lambda: np.zeros(cap, np.float64)
        return dict(x=f() if dim == 2 else None, y=f() if dim >= 1 else None, cx=f(), cy=f(),
                    cz=f(), erot=f(), vib=np.zeros(cap, np.int32),
                    cell=np.full(cap, -1, np.int32), pid=np.zeros(cap, np.uint32))

    def _struct(self, A, n, next_pid):
        return OrcParts(n, self.cap, _p(A["x"]), _p(A["y"]), _p(A["cx"]), _p(A["cy"]),
                        _p(A["cz"]), _p(A["erot"]), _p(A["vib"]), _p(A["cell"]), _p(A["pid"]),
                        next_pid)

    # -- accessors ---------------------------------------------------------
    @property
    def n(self):
        return self.structs[self.cur].n

    @property
    def next_pid(self):
        return self.structs[self.cur].next_pid

    def state(self):
        A, n = self.bufs[self.cur], self.n
        out = {k: (None if v is None else v[:n].copy()) for k, v in A.items()}
        out["n"] = n
        out["next_pid"] = self.next_pid
        return out

    def moments(self):
        return self.mom.reshape(NMOM, self.M)

    def cellstate(self):
        return self.cs.reshape(NCS, self.M)

    def cnt(self):
        return dict(zip(CNT_NAMES, self.counters.tolist()))

    # -- phases ------------------------------------------------------------
    def bin(self):
        L = lib()
        src, dst = self.cur, 1 - self.cur
        r = L.orc_bin(C.byref(self.grid), C.byref(self.structs[src]), C.byref(self.structs[dst]),
                      _p(self.offsets), self.f32, _p(self.counters))
        if r != 0:
            raise RuntimeError("orc_bin failed")
        self.cur = dst
        self.sorted = True

    def do_moments(self):
        lib().orc_moments(C.byref(self.grid), C.byref(self.gas), C.byref(self.structs[self.cur]),
                          _p(self.offsets), _p(self.mom))

    def do_cellstate(self):
        lib().orc_cellstate(C.byref(self.grid), C.byref(self.gas), _p(self.mom), self.prob.dt,
                            _p(self.dt_cell), _p(self.cs))

    def collide(self, step):
        lib().orc_collide(C.byref(self.grid), C.byref(self.gas), _p(self.cs), _p(self.offsets),
                          C.byref(self.structs[self.cur]), self.prob.seed, step, self.f32,
                          _p(self.counters))

    def conserve(self, step):
        lib().orc_conserve(C.byref(self.grid), C.byref(self.gas), _p(self.cs), _p(self.offsets),
                           C.byref(self.structs[self.cur]), self.prob.seed, step, self.f32,
                           _p(self.counters))

    def advect(self, step):
        lib().orc_advect(C.byref(self.grid), C.byref(self.gas), C.byref(self.bc), self.prob.dt,
                         C.byref(self.structs[self.cur]), self.prob.seed, step, self.f32,
                         _p(self.counters))

    def enable_sampling(self, nbody=0):
        """Zeroed field sums [NSAMP, M] and surface sums [elements, SURF_NQ]
        (int64 fixed point); from now on every diffuse re-emission is
        sampled, and :meth:`sample_fields` adds the current binned state."""
        g = self.prob.grid
        ne = 2 * g.nx + 2 * g.ny + int(nbody)
        self.surf = np.zeros((ne, SURF_NQ), np.int64)
        self.fields = np.zeros((NSAMP, self.M))
        self.bc.surf = self.surf.ctypes.data
        self.bc.surf_nbody = int(nbody)

    def sample_fields(self):
        """Add the per-cell particle sums of the current binned state."""
        if not self.sorted:
            raise RuntimeError("sample_fields needs a binned state")
        lib().orc_sample_fields(C.byref(self.grid), C.byref(self.structs[self.cur]),
                                _p(self.offsets), _p(self.fields))

    def interp(self, field, cell, x, y):
        return lib().orc_interp(C.byref(self.grid), _p(self.cs), CS_NAMES.index(field), cell, x, y)

    def step(self, step, nsteps=1):
        """Full steps: bin, moments, cell state, collide, conserve, advect."""
        for s in range(nsteps):
            st = step + s
            self.bin()
            self.do_moments()
            self.do_cellstate()
            self.collide(st)
            self.conserve(st)
            self.advect(st)

    def step_native(self, step, nsteps=1):
        """Same as :meth:`step`, in one call into the library."""
        L = lib()
        a, b = C.byref(self.structs[self.cur]), C.byref(self.structs[1 - self.cur])
        r = L.orc_step(C.byref(self.grid), C.byref(self.gas), C.byref(self.bc), self.prob.dt,
                       _p(self.dt_cell), a, b, _p(self.offsets), _p(self.mom), _p(self.cs),
                       self.prob.seed, step, nsteps, self.f32, _p(self.counters))
        if r != 0:
            raise RuntimeError("orc_step failed")
        # orc_step swaps the contents of the two structs once per step;
        # re-pair structs with buffers so structs[k] describes bufs[k]
        if nsteps % 2 == 1:
            self.structs = [self.structs[1], self.structs[0]]
            self.cur = 1 - self.cur
        self.sorted = False


def threads():
    return lib().orc_get_threads()


def sample_nb(u, r, p):
    return lib().orc_sample_nb(u, r, p)


def sample_b(u, n, p):
    return lib().orc_sample_b(u, n, p)


def inflow_speed(seed, step, pid, s):
    return lib().orc_inflow_speed(seed, step, pid, s)
