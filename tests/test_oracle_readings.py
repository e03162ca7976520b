"""Pins of the oracle's two reading switches of the USP-FPM particle update.

gamma_scope: the coefficient chain of Secs. III.A.1-III.A.3 (gammas,
relaxation temperatures, diffusion tensor and its refit) runs at the
temperatures and Pi interpolated to each particle (the flow chart of Sec.
IV.D) or at the cell's own values; the mean velocity U is interpolated in
both.  alpha_sign: after a positivity refit, the root of eq.
alpha_USP_positivity_2 whose Prandtl number (eq. alpha_USP_positivity_3)
is closer to the cell's, or the root with the sign of the cell's alpha.

Pins: in 0D there is nothing to interpolate, so the two scopes give the
same bits; with the cell scope a particle's new rotational energy and level
cannot depend on where in its cell it sits, and its new velocity depends on
it only through (1 - alpha) U (eq. update_ci); the sign switch changes only
the sign of alpha, never alpha^2, nu, T^rel or the Cholesky factor."""
import math

import numpy as np
import pytest

import oracle
import usp_workloads as W

from test_oracle_collide import ANISO, _coef_cell, _refit_cases


def _run_collide(prob, parts, step=3):
    sim = oracle.Sim(prob, parts)
    sim.bin(); sim.do_moments(); sim.do_cellstate()
    sim.collide(step)
    return sim


def test_gamma_scope_0d_is_identical():
    """0D cells (no neighbours): the interpolated temperatures and Pi are
    the cell's own, so the two readings give the same bits (several cells
    of different temperatures, anisotropic Pi)."""
    rng = np.random.default_rng(5)
    counts = [40, 300, 2000]
    M = len(counts)
    U = [(rng.normal() * 300, 0.0, 0.0) for _ in range(M)]
    out = []
    for scope in (W.GAMMA_PARTICLE, W.GAMMA_CELL):
        prob, parts = W.batch0d(counts, T_tr=[3000.0, 9000.0, 20000.0], T_rot=[300.0, 800.0, 2000.0],
                                T_vib=[300.0, 1500.0, 4000.0], dens=[1e22, 1e23, 1e24], dt=2e-8,
                                f32=False, seed=9,
                                U=U, anis=[(1.0, 2.0, 0.5)] * M)
        prob.gas = W.replace(prob.gas, gamma_scope=scope)
        sim = _run_collide(prob, parts)
        out.append((sim.state(), sim.cnt()))
    (a, ca), (b, cb) = out
    for k in ("cx", "cy", "cz", "erot", "vib"):
        assert np.array_equal(a[k], b[k]), k
    assert ca == cb


def _shear_problem(scope):
    """1D channel (16 cells) with a sheared, non-isothermal state: U_x and
    the temperature vary across each cell, so interpolation matters."""
    prob = W.poiseuille(kn=0.05, cells=16, ppc=300, f32=False)
    prob.gas = W.replace(prob.gas, gamma_scope=scope)
    parts = W.particles_for(prob)
    n = parts["n"]
    gap = prob.notes["gap"]
    frac = parts["y"][:n] / gap
    heat = np.sqrt(0.4 + 1.2 * frac)
    for k in ("cx", "cy", "cz"):
        parts[k][:n] *= heat
    parts["erot"][:n] *= heat ** 2
    parts["cx"][:n] += 400.0 * np.sin(np.pi * frac)
    return prob, parts


def _jittered(prob, parts, seed=17):
    """The same particles, each moved to a random point of its own cell
    (kept 1% away from the cell's edges)."""
    out = W.copy_parts(parts)
    n, g = parts["n"], prob.grid
    y = parts["y"][:n]
    cell = np.floor((y - g.y0) / g.dy)
    u = np.random.default_rng(seed).uniform(0.01, 0.99, n)
    out["y"][:n] = g.y0 + (cell + u) * g.dy
    assert np.array_equal(np.floor((out["y"][:n] - g.y0) / g.dy), cell)
    return out


def test_gamma_scope_cell_ignores_position_in_cell():
    """Cell scope: moving every particle inside its own cell leaves its new
    rotational energy and level bit-identical and changes its new velocity
    by exactly (1 - alpha)(U(x_a) - U(x_b)) (eq. update_ci with the same
    draws and the same Cholesky factor), alpha the cell's (no refit in this
    near-equilibrium state).  The per-particle scope, on the same pair of
    states, changes the rotational energies: the pin tells the two apart."""
    prob, parts = _shear_problem(W.GAMMA_CELL)
    moved = _jittered(prob, parts)
    a = _run_collide(prob, parts)
    b = _run_collide(prob, moved)
    assert a.cnt()["CHOL_FALLBACK"] == 0 and b.cnt()["CHOL_FALLBACK"] == 0
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["pid"], sb["pid"]) and np.array_equal(sa["cell"], sb["cell"])
    assert np.array_equal(sa["erot"], sb["erot"])
    assert np.array_equal(sa["vib"], sb["vib"])
    cs = a.cellstate()
    al = cs[oracle.CS_NAMES.index("ALPHA")]
    vs = math.sqrt(prob.gas.R * 300.0)
    worst = 0.0
    for i in range(sa["n"]):
        c = int(sa["cell"][i])
        for k, f in (("cx", "UX"), ("cy", "UY"), ("cz", "UZ")):
            ua = a.interp(f, c, 0.0, float(sa["y"][i]))
            ub = b.interp(f, c, 0.0, float(sb["y"][i]))
            d = (sa[k][i] - sb[k][i]) - (1.0 - al[c]) * (ua - ub)
            worst = max(worst, abs(d) / vs)
    assert worst < 1e-11, worst
    # the per-particle scope on the same two states
    prob_p = W.replace(prob, gas=W.replace(prob.gas, gamma_scope=W.GAMMA_PARTICLE))
    pa, pb = _run_collide(prob_p, parts).state(), _run_collide(prob_p, moved).state()
    assert np.mean(pa["erot"] != pb["erot"]) > 0.5


def test_gamma_scope_cell_particles_of_a_cell_share_coefficients():
    """Cell scope: every particle of a cell is updated with the chain taken
    at the cell's own temperatures and Pi.  From each particle's velocity
    change, eq. update_ci with the cell's alpha and Cholesky factor L gives
    back three standard normals; they must be the particle's own Box-Muller
    draws (counter (pid, step, collide, 0)), and eq. update_erot with the
    cell's T_rot^rel and the fourth normal must give its new rotational
    energy.  A chain evaluated anywhere else (an interpolated value, a
    neighbour's) gives other L and T_rot^rel and fails."""
    prob, parts = _shear_problem(W.GAMMA_CELL)
    sim = _run_collide(prob, parts)
    cs = sim.cellstate()
    names = oracle.CS_NAMES
    pre = oracle.Sim(prob, parts)
    pre.bin()
    s0, s1 = pre.state(), sim.state()
    R = prob.gas.R
    checked = 0
    for c in range(prob.grid.ncells):
        v = {k: cs[names.index(k), c] for k in names}
        if v["COLLIDE"] == 0.0:
            continue
        P = np.array([v["PXX"], v["PYY"], v["PZZ"], v["PXY"], v["PXZ"], v["PYZ"]])
        r = oracle.particle_coef(prob.gas, v["TTR"], v["TROT"], v["TVIB"], P, v["A"], v["B"],
                                 v["ALPHA"], v["OMA2"], v["NU"], v["R2"], 2.0 * v["MUP"], v["PR"],
                                 v["DT"])
        idx = np.nonzero(s1["cell"] == c)[0]
        al, sq, L = r["al"], math.sqrt(r["oma2"]), r["L"]
        for i in idx[:20]:
            U = [sim.interp(f, c, 0.0, float(s1["y"][i])) for f in ("UX", "UY", "UZ")]
            # velocity rows of eq. update_ci give G1, G2, G3 from the x, y, z rows
            G1 = (s1["cx"][i] - U[0] - al * (s0["cx"][i] - U[0])) / (sq * L[0])
            G2 = (s1["cy"][i] - U[1] - al * (s0["cy"][i] - U[1]) - sq * L[1] * G1) / (sq * L[2])
            G3 = (s1["cz"][i] - U[2] - al * (s0["cz"][i] - U[2]) - sq * (L[3] * G1 + L[4] * G2)) / (
                sq * L[5])
            # the Gaussians are those of the particle's own Box-Muller pair
            w = oracle.philox([int(s1["pid"][i]), 3, 0, 0],
                              [prob.seed & 0xFFFFFFFF, prob.seed >> 32])
            u = (w.astype(np.float64) + 0.5) / 4294967296.0
            r0 = math.sqrt(-2.0 * math.log(u[0]))
            r1 = math.sqrt(-2.0 * math.log(u[2]))
            assert G1 == pytest.approx(r0 * math.cos(2 * math.pi * u[1]), abs=1e-9)
            assert G2 == pytest.approx(r0 * math.sin(2 * math.pi * u[1]), abs=1e-9)
            assert G3 == pytest.approx(r1 * math.cos(2 * math.pi * u[3]), abs=1e-9)
            G4 = r1 * math.sin(2 * math.pi * u[3])
            half = 0.5 * R * r["Trot_rel"] * r["oma2"]
            root = math.sqrt(s0["erot"][i]) * al + math.sqrt(half) * G4
            assert s1["erot"][i] == pytest.approx(half + root * root, rel=1e-12)
            checked += 1
    assert checked > 100


def _pair_cases(gas, dto, seed, Ts, aniso):
    g_keep = W.replace(gas, alpha_sign=W.ALPHA_SIGN_KEEP)
    cc = _coef_cell(gas, 3000.0, 3000.0, dto, seed)
    a = _refit_cases(gas, cc, Ts, aniso, seed)
    b = _refit_cases(g_keep, cc, Ts, aniso, seed)
    return cc, a, b


def _compare_rules(cc, A, B):
    """Per case: every field but alpha equal, |alpha| equal, KEEP's sign the
    cell's.  Returns (refits, flips, [|alpha|, flipped] per refit)."""
    refits, flips, seen = 0, 0, []
    for (_, _, _, _, r, _), (_, _, _, _, q, _) in zip(A, B):
        for k in ("fallback", "nu_zero", "skip", "oma2", "nu", "nu_bound", "Ttr_rel",
                  "Trot_rel", "mstar"):
            assert r[k] == q[k], k
        assert np.array_equal(r["L"], q["L"])
        assert abs(r["al"]) == abs(q["al"])
        if r["fallback"] and not r["skip"]:
            refits += 1
            if q["al"] != 0.0:
                assert math.copysign(1.0, q["al"]) == (-1.0 if cc["ALPHA"] < 0 else 1.0)
            flips += r["al"] != q["al"]
            seen.append((abs(r["al"]), r["al"] != q["al"]))
        else:
            assert r["al"] == q["al"]
    return refits, flips, seen


def test_alpha_sign_keep_changes_only_the_sign():
    """The two sign rules on the same hand-made anisotropic Pi: every field
    but alpha is the same bits, |alpha| is the same, and with KEEP the sign
    is the cell's alpha = cbrt(r3) (0 counts +).

    When the rules differ follows from eq. alpha_USP_positivity_3: with s =
    alpha^3, Pr(s) is proportional to f(s) = (1 - s)/(1 + s), decreasing, and
    the target is f(s_c), s_c the cell's.  For s_c >= 0 the + root is always
    closer (f(a^3) + f(-a^3) >= 2 > 2 f(s_c)); for s_c < 0 the - root is
    closer iff f(a^3) + f(-a^3) < 2 f(s_c), i.e. iff a^6 < |s_c|: the Prandtl
    rule leaves the cell's sign exactly when |alpha| > sqrt(|alpha_c|).  With
    the Eucken Prandtl number (nu < 0) the clamp only shrinks |alpha| below
    |alpha_c|, so the rules never differ; with a constant Pr = 2.5 (nu > 0)
    and dt just above A/Pr (alpha_c slightly negative) a strong refit grows
    |alpha| past sqrt(|alpha_c|) and they do."""
    Ts = [(3000.0, 3000.0, 3000.0), (3000.0, 300.0, 300.0), (3000.0, 12000.0, 3000.0),
          (3000.0, 30000.0, 5000.0), (1000.0, 60000.0, 1000.0)]
    neg_cell, refits = 0, 0
    for dto, seed in ((0.3, 1), (1.0, 2), (3.0, 3), (10.0, 4), (30.0, 5)):
        cc, A, B = _pair_cases(W.Gas(), dto, seed, Ts, ANISO)
        assert cc["NU"] < 0
        neg_cell += cc["ALPHA"] < 0
        n, flips, _ = _compare_rules(cc, A, B)
        refits += n
        assert flips == 0
    assert neg_cell >= 1 and refits >= 10, (neg_cell, refits)
    gas = W.Gas(pr_model=W.PR_CONST, Pr_const=2.5, Z_rot=0.2)
    Ts = [(3000.0, 10.0, 10.0), (3000.0, 300.0, 10.0), (3000.0, 1000.0, 300.0)]
    aniso = ANISO + [(1, 1e-3, 1e-3), (1, 1e-2, 1e-2), (1, 0.1, 0.1)]
    total = 0
    for dto in (1.21, 1.22, 1.3):
        cc, A, B = _pair_cases(gas, dto, 5, Ts, aniso)
        assert cc["NU"] > 0 and cc["ALPHA"] < 0
        _, flips, seen = _compare_rules(cc, A, B)
        total += flips
        thr = math.sqrt(abs(cc["ALPHA"]))
        for a, flipped in seen:
            assert flipped == (a > thr), (dto, a, thr)
    assert total >= 1
