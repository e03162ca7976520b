"""Pathwise gradient of the oracle's steps (TEST INFRASTRUCTURE ONLY).

The gradient checked here is that of time-averaged outputs of a 1D run
(FP64, USP-FPM scheme) with respect to the collision-model parameters
(Z_rot, omega, mu_ref), along the path of one run with every discrete
outcome held fixed at the values the run took:

- the cell of every particle and the order of the binned state;
- the vibrational levels after the collision (Sec. III.A.2 jumps) and after
  the conservation picks (Sec. IV.C);
- every boundary event of the free flight: a particle whose flight meets a
  wall keeps its re-emitted velocity, energy and level as constants, and
  its position after the flight follows the time of its first wall hit
  (the flights between walls after it keep their recorded durations);
- every branch: the stencil of each particle (Sec. III.B), the 5% floor of
  the interpolated temperatures, the Cholesky test (a particle whose test
  fails keeps its post-collision state as a constant, Sec. III.A.3), the
  clamp of T_rot^rel, and the skips of the conservation scalings.

The random normals of the update (eq. update_ci, eq. update_erot) are the
oracle's own draws.  Everything continuous is evaluated with plain PyTorch
FP64 operations on the CPU in the order of the paper's algorithm, and the
gradient comes from torch.autograd.  `replay()` evaluates the same path at
other parameter values with the recorded outcomes, so central finite
differences of it give the same derivative (the pin of the tests).

Outputs (a run of K steps, area = cell volume / dy):
  mdot = m fnum / (area K) * sum over steps of sum_i c_x,i at the start of
         the step (mass flow per unit depth through the channel);
  tau_w = m fnum / (2 area K dt) * sum over steps of sum over the particles
         whose flight meets a wall of (c_x before - c_x after) (the wall
         shear averaged over the two walls; a particle's successive
         re-emissions telescope to its first incident and last re-emitted
         velocity).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import CS_NAMES, Sim, lib, _p

KB = 1.380649e-23

DT = torch.float64
PARAMS = ("Z_rot", "omega", "mu_ref")


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=DT)


class Record:
    """The oracle's K steps from the initial state, with everything the
    replay needs per step (arrays over the binned particles of the step)."""

    def __init__(self, prob, parts, step0, K):
        g = prob.grid
        if g.dim != 1 or prob.f32 or getattr(prob.gas, "scheme", 0) != 0:
            raise ValueError("the pathwise gradient is defined for 1D FP64 USP-FPM runs")
        self.prob, self.step0, self.K = prob, step0, K
        sim = Sim(prob, parts)
        self.init = sim.state()
        self.steps = []
        L = lib()
        for s in range(K):
            st = step0 + s
            pre = sim.state()
            pos = {int(p): i for i, p in enumerate(pre["pid"])}
            sim.bin()
            b = sim.state()
            perm = np.array([pos[int(p)] for p in b["pid"]], np.int64)
            offsets = sim.offsets.copy()
            sim.do_moments()
            sim.do_cellstate()
            cs = sim.cellstate().copy()
            sim.collide(st)
            co = sim.state()
            sim.conserve(st)
            cn = sim.state()
            sim.advect(st)
            fl = sim.state()
            n = b["n"]
            G = np.zeros(4 * n)
            pid = np.ascontiguousarray(b["pid"], np.uint32)
            L.orc_collide_normals(prob.seed, st, n, pid.ctypes.data, _p(G))
            self.steps.append(dict(perm=perm, offsets=offsets, cs=cs, binned=b, coll=co, cons=cn,
                                   flight=fl, G=G.reshape(n, 4)))
        self.final = sim.state()


def _segsum(cell, M, v):
    out = torch.zeros((M,) + tuple(v.shape[1:]), dtype=DT)
    return out.index_add_(0, cell, v)


def _evib_R(theta, T):
    """e_vib / R = theta / (e^{theta/T} - 1) (0 for T <= 0)."""
    x = theta / torch.where(T > 0, T, torch.ones_like(T))
    safe = torch.where(x > 700, torch.full_like(x, 700.0), x)
    v = theta / torch.expm1(safe)
    return torch.where((T > 0) & (x <= 700), v, torch.zeros_like(v))


def _cv_R(theta, T):
    """c_v,vib / R = x^2 / sinh(x)^2 / ... with x = theta/(2T)."""
    x = theta / (2 * torch.where(T > 0, T, torch.ones_like(T)))
    safe = torch.where(x > 300, torch.full_like(x, 300.0), x)
    s = torch.sinh(safe)
    v = safe * safe / (s * s)
    return torch.where((T > 0) & (x <= 300), v, torch.zeros_like(v))


def _tcheck(theta, Ttr, Trot, Tvib, a, b):
    """Rescaled temperature (Sec. III.A.1): the root of
    (3/2 + a) T + b e_vib(T)/R = 3/2 T_tr + a T_rot + b e_vib(T_vib)/R,
    by Newton without gradient, then one Newton step from the root with
    gradient (its derivative is that of the root: implicit function)."""
    with torch.no_grad():
        rhs = 1.5 * Ttr + a * Trot + b * _evib_R(theta, Tvib)
        hi = rhs / (1.5 + a)
        lo = torch.zeros_like(hi)
        T = hi.clone()
        for _ in range(200):
            f = (1.5 + a) * T + b * _evib_R(theta, T) - rhs
            hi = torch.where(f > 0, T, hi)
            lo = torch.where(f > 0, lo, T)
            fp = (1.5 + a) + b * _cv_R(theta, T)
            Tn = T - f / fp
            bad = ~((Tn > lo) & (Tn < hi))
            Tn = torch.where(bad, 0.5 * (lo + hi), Tn)
            done = (Tn - T).abs() <= 1e-15 * T
            T = Tn
            if bool(done.all()):
                break
        T0 = torch.where(hi > 0, T, torch.zeros_like(T))
    rhs = 1.5 * Ttr + a * Trot + b * _evib_R(theta, Tvib)
    f = (1.5 + a) * T0 + b * _evib_R(theta, T0) - rhs
    fp = (1.5 + a) + b * _cv_R(theta, T0)
    return T0 - f / fp


def _gammas(theta, Ttr, Trot, Tvib, a, b):
    """(g_tr-rot, g_tr-vib, g_rot-vib) / R of Sec. III.A.1 with the secant
    c_v,vib between T-check and T_vib (midpoint c_v within 3e-6)."""
    Tc = _tcheck(theta, Ttr, Trot, Tvib, a, b)
    near = (Tc - Tvib).abs() <= 3e-6 * torch.maximum(Tc, Tvib)
    den = torch.where(near, torch.ones_like(Tc), Tc - Tvib)
    sec = (_evib_R(theta, Tc) - _evib_R(theta, Tvib)) / den
    cbar = torch.where(near, _cv_R(theta, 0.5 * (Tc + Tvib)), sec)
    D = 1.5 + a + b * cbar
    return 3.0 * a / D, 3.0 * b * cbar / D, 2.0 * a * b * cbar / D


def _chol(S):
    l11 = torch.sqrt(S[0])
    l21, l31 = S[3] / l11, S[4] / l11
    d2 = S[1] - l21 * l21
    l22 = torch.sqrt(d2)
    l32 = (S[5] - l31 * l21) / l22
    d3 = S[2] - l31 * l31 - l32 * l32
    ok = (S[0] > 0) & (d2 > 0) & (d3 > 0)
    return (l11, l21, l22, l31, l32, torch.sqrt(d3)), ok


class Path:
    """The run of a Record as a function of theta = (Z_rot, omega, mu_ref)."""

    def __init__(self, rec):
        self.rec = rec
        self.dec = None   # branch outcomes of the base evaluation

    def run(self, theta, check=False):
        """J = (mdot, tau_w) along the recorded path.  The first call fixes
        the branch outcomes (at the recorded parameters); later calls replay
        them.  With check, the continuous values of every phase are compared
        with the oracle's (largest relative difference returned)."""
        rec, prob = self.rec, self.rec.prob
        gas, g, bc = prob.gas, prob.grid, prob.bc
        record = self.dec is None
        if record:
            self.dec = []
        Zr, om, mur = theta[0], theta[1], theta[2]
        R = KB / gas.m
        Th = gas.theta_vib
        av = gas.alpha_vss
        Kf = av * (5 - 2 * om) * (7 - 2 * om) / (5 * (av + 1) * (av + 2))
        M = g.ny
        vol = _t(g.volume)
        area = float(g.volume[0]) / g.dy
        fnum, dt = g.fnum, prob.dt
        ylo, yhi = g.y0, g.y0 + g.ny * g.dy
        gvec = _t(bc.g)
        st0 = rec.init
        y = _t(st0["y"])
        c = torch.stack([_t(st0["cx"]), _t(st0["cy"]), _t(st0["cz"])], 1)
        e = _t(st0["erot"])
        mdot = torch.zeros((), dtype=DT)
        tau = torch.zeros((), dtype=DT)
        worst = 0.0

        def cmp(name, a, ref):
            nonlocal worst
            a = a.detach().numpy()
            ref = ref.detach().numpy() if torch.is_tensor(ref) else np.asarray(ref)
            sc = max(np.abs(ref).max(), 1e-300)
            worst = max(worst, float(np.abs(a - ref).max() / sc))

        for k, S in enumerate(rec.steps):
            dk = {} if record else self.dec[k]
            mdot = mdot + c[:, 0].sum()
            perm = torch.as_tensor(S["perm"])
            y, c, e = y[perm], c[perm], e[perm]
            b = S["binned"]
            if check:
                cmp("bin y", y, b["y"]); cmp("bin c", c, np.stack([b["cx"], b["cy"], b["cz"]], 1))
            off = S["offsets"]
            cnt = np.diff(off)
            cell = torch.as_tensor(np.repeat(np.arange(M), cnt))
            Nc = _t(cnt)
            Np = Nc.clamp(min=1.0)
            lev0 = _t(b["vib"])
            # moments (Sec. II.A)
            U = _segsum(cell, M, c) / Np[:, None]
            d = c - U[cell]
            pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
            P = torch.stack([_segsum(cell, M, d[:, i] * d[:, j]) for i, j in pairs], 1) / Np[:, None]
            er = _segsum(cell, M, e) / Np
            Ib = _segsum(cell, M, lev0) / Np
            # cell state
            trP = P[:, 0] + P[:, 1] + P[:, 2]
            Ttr = trP / (3 * R)
            Trot = er / R
            Tvib = torch.where(Ib > 0, Th / torch.log1p(1 / torch.where(Ib > 0, Ib, torch.ones_like(Ib))),
                               torch.zeros_like(Ib))
            coll = (Nc >= 2) & (Ttr > 0) & (vol > 0)
            if record:
                dk["coll"] = coll.clone()
            else:
                coll = dk["coll"]
            Tsafe = torch.where(coll, Ttr, torch.ones_like(Ttr))
            mu = mur * (Tsafe / gas.T_ref) ** om
            nd = Nc * fnum / vol
            mup = mu / (torch.where(coll, nd, torch.ones_like(nd)) * KB * Tsafe)
            # cells that do not collide: harmless stand-ins (no value or
            # gradient of theirs is used, but none may be singular)
            mup = torch.where(coll, mup, torch.full_like(mup, prob.dt))
            tauc = Kf * mup
            x = Th / Tsafe
            xi = torch.where(x > 700, torch.zeros_like(x), x / torch.expm1(torch.clamp(x, max=700.0)))
            Pr = (14 + 2 * xi) / (19 + 2 * xi)
            A = 2 * mup
            dtc = dt
            r3 = (A - Pr * dtc) / (A + Pr * dtc)
            r2 = (A - dtc) / (A + dtc)
            al = torch.sign(r3) * torch.abs(r3) ** (1.0 / 3.0)
            oma2 = 1 - al * al
            nu = (r2 - al * al) / oma2
            ac = dtc / (dtc + 2 * Zr * tauc)
            bcf = dtc / (dtc + 2 * gas.Z_vib * tauc)
            g0, g1, g2 = _gammas(Th, Tsafe, Trot, Tvib, ac, bcf)
            erot_new = er + R * (g0 * (Ttr - Trot) - g2 * (Trot - Tvib))
            E0 = 0.5 * trP + er + Ib * R * Th
            if check:
                cs = S["cs"]
                ci = lambda nm: CS_NAMES.index(nm)
                m = coll.numpy()
                for nm, v in (("ALPHA", al), ("NU", nu), ("A", ac), ("EROT_NEW", erot_new),
                              ("TTR", Ttr), ("UX", U[:, 0])):
                    cmp(nm, v[m], cs[ci(nm)][m])
            # reconstruction (Sec. III.B): stencil toward the particle's half
            j = cell
            dyv = y - (g.y0 + (j.to(DT) + 0.5) * g.dy)
            if record:
                sy = torch.where(dyv >= 0, 1, -1)
                okc = coll.numpy()

                def ok(jj):
                    jn = jj.numpy()
                    inside = (jn >= 0) & (jn < M)
                    res = np.zeros_like(inside)
                    res[inside] = okc[jn[inside]]
                    return torch.as_tensor(res)
                ty = torch.where(ok(j + sy), sy, torch.where(ok(j - sy), -sy, torch.zeros_like(sy)))
                dk["ty"] = ty
            ty = dk["ty"]
            has = ty != 0
            jn = torch.where(has, j + ty, j)
            w = torch.where(has, dyv / (torch.where(has, ty, torch.ones_like(ty)).to(DT) * g.dy),
                            torch.zeros_like(dyv))

            def interp(F):
                f0, f1 = F[j], F[jn]
                return f0 + (f1 - f0) * (w[:, None] if F.dim() == 2 else w)
            Ui, Pi = interp(U), interp(P)
            Ti = [interp(Ttr), interp(Trot), interp(Tvib)]
            Tcell = [Ttr[j], Trot[j], Tvib[j]]
            if record:
                dk["floor"] = [Ti[q] < 0.05 * Tcell[q] for q in range(3)]
            for q in range(3):
                Ti[q] = torch.where(dk["floor"][q], 0.05 * Tcell[q], Ti[q])
            a_p, b_p, al_p, om_p, nu_p = ac[j], bcf[j], al[j], oma2[j], nu[j]
            h0, h1, h2 = _gammas(Th, Ti[0], Ti[1], Ti[2], a_p, b_p)
            Xtr = h0 * (Ti[0] - Ti[1]) + h1 * (Ti[0] - Ti[2])
            Xrot = h0 * (Ti[0] - Ti[1]) - h2 * (Ti[1] - Ti[2])
            Ttr_rel = Ti[0] - Xtr / (om_p * 1.5)
            Trot_rel = Ti[1] + Xrot / om_p
            RT = R * Ti[0]
            Lam = [R * Ttr_rel + nu_p * (Pi[:, q] - RT) for q in range(3)] + \
                  [nu_p * Pi[:, q] for q in range(3, 6)]
            Lc, chol_ok = _chol(Lam)
            inc = coll[j]
            if record:
                dk["fixed"] = inc & ~chol_ok
                dk["rclamp"] = Trot_rel < 0
            fixed = dk["fixed"]
            Trot_rel = torch.where(dk["rclamp"], torch.zeros_like(Trot_rel), Trot_rel)
            G = _t(S["G"])
            sq = torch.sqrt(om_p)
            v = torch.stack([Lc[0] * G[:, 0], Lc[1] * G[:, 0] + Lc[2] * G[:, 1],
                             Lc[3] * G[:, 0] + Lc[4] * G[:, 1] + Lc[5] * G[:, 2]], 1)
            cn = Ui + al_p[:, None] * (c - Ui) + sq[:, None] * v
            half = 0.5 * R * Trot_rel * om_p
            root = torch.sqrt(e) * al_p + torch.sqrt(half) * G[:, 3]
            en = half + root * root
            co = S["coll"]
            cfix = _t(np.stack([co["cx"], co["cy"], co["cz"]], 1))
            upd = inc & ~fixed
            c1 = torch.where(upd[:, None], cn, torch.where(fixed[:, None], cfix, c))
            e1 = torch.where(upd, en, torch.where(fixed, _t(co["erot"]), e))
            if check:
                cmp("collide c", c1, cfix); cmp("collide e", e1, co["erot"])
            # conservation (Sec. IV.C)
            cs_ = S["cons"]
            lev2 = _t(cs_["vib"])
            Un = U
            dd = c1 - Un[j]
            s = _segsum(j, M, dd)
            s3 = _segsum(j, M, (dd * dd).sum(1))
            s4 = _segsum(j, M, e1)
            SI = _segsum(j, M, lev2)
            m1 = s / Np[:, None]
            etr_s = 0.5 * (s3 / Np - (m1 * m1).sum(1))
            erot_s = s4 / Np
            if record:
                dk["rot"] = coll & (erot_s > 0) & (erot_new > 0)
            rot = dk["rot"]
            frot = torch.where(rot, erot_new / torch.where(rot, erot_s, torch.ones_like(erot_s)),
                               torch.ones_like(erot_s))
            erot_a = torch.where(rot, erot_new, erot_s)
            evib_a = SI * R * Th / Np
            s2 = (E0 - erot_a - evib_a) / torch.where(etr_s != 0, etr_s, torch.ones_like(etr_s))
            if record:
                dk["vel"] = coll & (etr_s > 0) & (s2 > 0)
            vel = dk["vel"]
            sc = torch.sqrt(torch.where(vel, s2, torch.ones_like(s2)))
            Us = Un + m1
            c2 = torch.where(vel[j][:, None], Un[j] + sc[j][:, None] * (c1 - Us[j]), c1)
            e2 = torch.where(rot[j], e1 * frot[j], e1)
            if check:
                cmp("conserve c", c2, np.stack([cs_["cx"], cs_["cy"], cs_["cz"]], 1))
                cmp("conserve e", e2, cs_["erot"])
            # free flight (Sec. II.C) and walls
            ck = c2 + gvec * dt
            fl = S["flight"]
            if record:
                yy = y + ck[:, 1] * dt
                dk["event"] = ((ck[:, 1] < 0) & (yy < ylo)) | ((ck[:, 1] > 0) & (yy >= yhi))
            ev = dk["event"]
            cf = _t(np.stack([fl["cx"], fl["cy"], fl["cz"]], 1))
            tau = tau + torch.where(ev, ck[:, 0] - cf[:, 0], torch.zeros_like(ck[:, 0])).sum()
            # a particle whose flight meets a wall leaves with the re-emitted
            # velocity, energy and level (constants of the path); its position
            # after the flight follows the first hit time t1 = (y_wall,1 - y)/c_y:
            # y_f = y_wall,last + c_y,f (dt - t_between - t1), with t_between
            # (the flights between the walls) fixed at its recorded value
            cfy = cf[:, 1]
            yw1 = torch.where(ck[:, 1] < 0, torch.full_like(y, ylo), torch.full_like(y, yhi))
            ywl = torch.where(cfy > 0, torch.full_like(y, ylo), torch.full_like(y, yhi))
            cky = torch.where(ev, ck[:, 1], torch.ones_like(y))
            if record:
                with torch.no_grad():
                    t1r = (yw1 - y) / cky
                    tlr = dt - (_t(fl["y"]) - ywl) / torch.where(ev, cfy, torch.ones_like(cfy))
                    dk["t_between"] = torch.where(ev, tlr - t1r, torch.zeros_like(t1r))
            yhit = ywl + cfy * (dt - dk["t_between"] - (yw1 - y) / cky)
            y = torch.where(ev, yhit, y + ck[:, 1] * dt)
            c = torch.where(ev[:, None], cf, ck)
            e = torch.where(ev, _t(fl["erot"]), e2)
            if check:
                cmp("flight y", y, fl["y"]); cmp("flight c", c, cf)
            if record:
                self.dec.append(dk)
        Kst = len(rec.steps)
        w_m = gas.m * fnum / (area * Kst)
        w_t = gas.m * fnum / (2 * area * Kst * dt)
        J = torch.stack([w_m * mdot, w_t * tau])
        return (J, worst) if check else J

    def theta0(self):
        gas = self.rec.prob.gas
        return torch.tensor([gas.Z_rot, gas.omega, gas.mu_ref], dtype=DT)

    def gradient(self):
        """J and dJ/dtheta (2 x 3) at the recorded parameters."""
        th = self.theta0().requires_grad_(True)
        J = self.run(th)
        rows = [torch.autograd.grad(J[o], th, retain_graph=o == 0)[0] for o in range(2)]
        return J.detach().numpy(), torch.stack(rows).numpy()

    def replay(self, theta):
        """J at other parameters along the recorded outcomes (no gradient)."""
        if self.dec is None:
            self.run(self.theta0())
        with torch.no_grad():
            return self.run(torch.as_tensor(theta, dtype=DT)).numpy()
