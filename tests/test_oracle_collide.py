"""Pins of the oracle's particle update and conservation scheme against the
relaxation rates the paper derives (Sec. III.A) and exact invariants.

The statistical tests compare one-step changes with their conditional
expectations given the pre-collision sample, so the only noise is that of
the fresh Gaussian/uniform draws."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import usp_workloads as W

KB = 1.380649e-23


def _cell_problem(cx, cy, cz, erot, vib, n_dens=1e23, dt=None, dt_over_tauc=1.0, gas=None,
                  cells=None, f32=False, seed=11):
    gas = gas or W.Gas()
    N = len(cx)
    cells = np.zeros(N, np.int32) if cells is None else cells
    M = int(cells.max()) + 1
    counts = np.bincount(cells, minlength=M)
    fnum = 1e9
    vol = counts * fnum / n_dens
    grid = W.Grid(dim=0, nx=M, ny=1, fnum=fnum, volume=vol, flags=np.zeros(M, np.uint8))
    R = gas.R
    if dt is None:
        Ttr = np.mean((cx - cx.mean()) ** 2 + (cy - cy.mean()) ** 2 + (cz - cz.mean()) ** 2) / (3 * R)
        dt = dt_over_tauc * oracle.Gas(gas).tau_c(Ttr, n_dens)
    prob = W.Problem("cell", gas, grid, W.BC(), dt=dt, seed=seed, f32=f32)
    parts = dict(n=N, cap=N, x=None, y=None, cx=cx, cy=cy, cz=cz, erot=erot,
                 vib=vib.astype(np.int32), cell=cells, pid=np.arange(N, dtype=np.uint32),
                 next_pid=N)
    sim = oracle.Sim(prob, parts)
    sim.bin(); sim.do_moments(); sim.do_cellstate()
    return prob, sim


def _cs(sim, name, c=0):
    return sim.cellstate()[oracle.CS_NAMES.index(name), c]


def _mom(sim, name, c=0):
    return sim.moments()[oracle.MOM_NAMES.index(name), c]


def test_viscous_stress_decay_factor():
    """sigma^{n+1} = sigma^n (2mu/p - dt)/(2mu/p + dt) in expectation
    (eq. sigma_relax reproduced through alpha and nu, Sec. III.A.2)."""
    rng = np.random.default_rng(21)
    gas = W.Gas()
    N = 1_000_000
    T = 3000.0
    s = math.sqrt(gas.R * T)
    cx = 1.5 * s * rng.standard_normal(N); cy = s * rng.standard_normal(N)
    cz = 0.8 * s * rng.standard_normal(N)
    cx += 0.3 * cy   # off-diagonal stress too
    erot = rng.exponential(gas.R * T, N)
    vib = rng.geometric(1 - math.exp(-gas.theta_vib / T), N) - 1
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, dt_over_tauc=1.0, gas=gas)
    A, dt = 2 * _cs(sim, "MUP"), _cs(sim, "DT")
    factor = (A - dt) / (A + dt)
    P0 = {k: _mom(sim, k) for k in ("PXX", "PYY", "PZZ", "PXY")}
    sim.collide(0)
    sim.do_moments()
    P1 = {k: _mom(sim, k) for k in ("PXX", "PYY", "PZZ", "PXY")}
    d0, d1 = P0["PXX"] - P0["PYY"], P1["PXX"] - P1["PYY"]
    RT = gas.R * _cs(sim, "TTR")
    assert abs(d1 - factor * d0) < 0.01 * RT, (d1 / d0, factor)
    assert abs(P1["PXY"] - factor * P0["PXY"]) < 0.01 * RT
    # a first-order (FPM-like) or nu-free factor would miss by far more
    assert abs(factor - _cs(sim, "ALPHA") ** 2) > 0.1


def test_heat_flux_decay_factor_all_modes():
    """q_tr, q_rot, q_vib each decay by alpha^3 = (2mu/p - Pr dt)/(2mu/p +
    Pr dt) per step (eqs. q*_relax; Sec. III.A.2)."""
    rng = np.random.default_rng(22)
    gas = W.Gas()
    N = 2_000_000
    T = 3000.0
    s = math.sqrt(gas.R * T)
    G = rng.standard_normal(N)
    cx = s * (G + 0.25 * (G * G - 1.0))
    cy = s * rng.standard_normal(N); cz = s * rng.standard_normal(N)
    erot = rng.exponential(gas.R * T, N) * (1.0 + 0.5 * np.tanh(G))
    Tv = np.where(G > 0, 3500.0, 2500.0)
    vib = rng.geometric(1 - np.exp(-gas.theta_vib / Tv)) - 1
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, dt_over_tauc=1.0, gas=gas)
    A, dt, Pr = 2 * _cs(sim, "MUP"), _cs(sim, "DT"), _cs(sim, "PR")
    factor = (A - Pr * dt) / (A + Pr * dt)
    assert abs(_cs(sim, "ALPHA") ** 3 - factor) < 1e-12
    q0 = {k: _mom(sim, k) for k in ("QTRX", "QROTX", "QIX")}
    sim.collide(0)
    sim.do_moments()
    q1 = {k: _mom(sim, k) for k in ("QTRX", "QROTX", "QIX")}
    for k in q0:
        assert abs(q1[k] / q0[k] - factor) < 0.03, (k, q1[k] / q0[k], factor)


def test_rotational_update_variance_closed_form():
    """Modified Milstein step (eq. update_erot) with T_rot^rel = T: the mean
    is kept and Var(eps') = a^4 Var(eps) + 4a^2 b^2 <eps> + 2 b^4, b^2 =
    R T (1-a^2)/2 -- for exponential eps, (RT)^2 [1 - (1-a^2)^2/2]."""
    rng = np.random.default_rng(23)
    gas = W.Gas()
    N = 2_000_000
    T = 2000.0
    s = math.sqrt(gas.R * T)
    cx, cy, cz = (s * rng.standard_normal(N) for _ in range(3))
    erot = rng.exponential(gas.R * T, N)
    vib = rng.geometric(1 - math.exp(-gas.theta_vib / T), N) - 1
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, dt_over_tauc=2.0, gas=gas)
    a = _cs(sim, "ALPHA")
    Trot = _cs(sim, "TROT")
    e0 = sim.state()["erot"]
    sim.collide(0)
    e1 = sim.state()["erot"]
    b2 = gas.R * Trot * (1 - a * a) / 2   # T_rot^rel ~ T_rot at equilibrium
    want_mean = 2 * b2 + a * a * e0.mean()
    want_var = a ** 4 * e0.var() + 4 * a * a * b2 * e0.mean() + 2 * b2 * b2
    th = gas.R * Trot
    assert abs(e1.mean() - want_mean) < 3e-3 * th
    assert abs(e1.var() / want_var - 1) < 0.01
    assert abs(want_var / (th * th * (1 - (1 - a * a) ** 2 / 2)) - 1) < 0.01


def test_maxwellian_velocities_stay_maxwellian():
    """With T_tr^rel = T and an isotropic Maxwellian, the velocity update is
    an exact Ornstein-Uhlenbeck step: the kurtosis stays Gaussian."""
    rng = np.random.default_rng(24)
    gas = W.Gas()
    N = 400_000
    T = 2500.0
    s = math.sqrt(gas.R * T)
    cx, cy, cz = (s * rng.standard_normal(N) for _ in range(3))
    erot = rng.exponential(gas.R * T, N)
    vib = rng.geometric(1 - math.exp(-gas.theta_vib / T), N) - 1
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, dt_over_tauc=1.0, gas=gas)
    for st in range(10):
        if st:
            sim.bin(); sim.do_moments(); sim.do_cellstate()
        sim.collide(st); sim.conserve(st)
    v = sim.state()
    for k in ("cx", "cy", "cz"):
        c = v[k] - v[k].mean()
        kurt = np.mean(c ** 4) / np.mean(c ** 2) ** 2
        assert abs(kurt - 3.0) < 0.04, (k, kurt)


def _pmf_nb(r, p, kmax):
    return stats.nbinom.pmf(np.arange(kmax), r, p)


def test_vibrational_jump_keeps_boltzmann_levels():
    """NB(I+1, p_NB) - B(I, p_B) with the printed parameters (eq.
    update_evib) leaves (1-q) q^I, q = exp(-Theta/T), invariant when T_vib^rel
    = T; the oracle's simplified forms p_NB = 1/(1+m*(1-a^2)), p_B =
    (1+m*)(1-a^2) equal the printed ones.  Exact pmf convolution."""
    th = W.THETA_VIB_N2
    for T, a2 in ((3371.0, 0.85), (1000.0, 0.5), (10000.0, 0.9)):
        x = th / T
        q = math.exp(-x)
        m = 1.0 / math.expm1(x)
        pNB = 1.0 / (1.0 + (1 - a2) / (math.exp(x) - 1))
        pB = math.exp(x) / (math.exp(x) - 1) * (1 - a2)
        assert abs(pNB - 1 / (1 + m * (1 - a2))) < 1e-14
        assert abs(pB - (1 + m) * (1 - a2)) < 1e-14
        K = 400
        P = (1 - q) * q ** np.arange(K)
        out = np.zeros(2 * K)
        for I in range(K):
            if P[I] < 1e-300:
                break
            nb = _pmf_nb(I + 1, pNB, K)
            b = stats.binom.pmf(np.arange(I + 1), I, pB)
            jump = np.convolve(nb, b[::-1])  # index j -> NB - B = j - I
            lo = 0  # I + (j - I) = j
            out[lo:lo + len(jump)] += P[I] * jump[:2 * K - lo]
        assert np.max(np.abs(out[:60] - P[:60])) < 1e-13
        # mean identity E[I'] = a^2 I + (1-a^2) m (Sec. III.A.2)
        for I in (0, 3, 17):
            mean = (I + 1) * (1 - pNB) / pNB - I * pB
            assert abs(I + mean - (a2 * I + (1 - a2) * m)) < 1e-12


def test_nb_and_b_inversion_match_library_quantiles():
    """The oracle's sequential CDF inversion returns the library quantile
    (smallest k with CDF(k) > u) away from exact CDF ties."""
    rng = np.random.default_rng(25)
    us = rng.random(4000)
    for r, p in ((1, 0.9), (4, 0.6), (12, 0.35)):
        cdf = stats.nbinom.cdf(np.arange(400), r, p)
        for u in us:
            want = int(np.searchsorted(cdf, u, side="right"))
            if np.min(np.abs(cdf - u)) < 1e-12:
                continue
            assert oracle.sample_nb(u, r, p) == want
    for n, p in ((1, 0.3), (7, 0.5), (20, 0.95)):
        cdf = stats.binom.cdf(np.arange(n + 1), n, p)
        for u in us:
            if np.min(np.abs(cdf - u)) < 1e-12:
                continue
            assert oracle.sample_b(u, n, p) == int(np.searchsorted(cdf, u, side="right"))
    assert oracle.sample_b(0.999, 5, 1.0) == 5 and oracle.sample_b(0.5, 0, 0.5) == 0


def test_conservation_to_round_off_and_targets():
    """After collide + conserve (Sec. IV.C) each cell keeps its momentum and
    total energy to rounding; rotational energy sits on its target, the
    vibrational energy within one quantum per cell."""
    rng = np.random.default_rng(26)
    gas = W.Gas()
    counts = np.array([2, 3, 50, 700, 4000])
    Ttr = [9000.0, 500.0, 6000.0, 12000.0, 3000.0]
    Trot = [300.0, 700.0, 4000.0, 800.0, 3000.0]
    Tv = [300.0, 2000.0, 2000.0, 600.0, 3000.0]
    cols = [[] for _ in range(5)]
    for c, N in enumerate(counts):
        s = math.sqrt(gas.R * Ttr[c])
        cols[0].append(300.0 * c + s * rng.standard_normal(N))
        cols[1].append(-50.0 + s * rng.standard_normal(N))
        cols[2].append(s * rng.standard_normal(N))
        cols[3].append(rng.exponential(gas.R * Trot[c], N))
        cols[4].append(rng.geometric(1 - math.exp(-gas.theta_vib / Tv[c]), N) - 1)
    cx, cy, cz, er, vb = (np.concatenate(v) for v in cols)
    cells = np.repeat(np.arange(len(counts)), counts).astype(np.int32)
    prob, sim = _cell_problem(cx, cy, cz, er, vb, cells=cells, n_dens=1e23, dt=2e-8, gas=gas)
    RTh = gas.R * gas.theta_vib
    st0 = sim.state()
    sim.collide(3)
    sim.conserve(3)
    st1 = sim.state()
    off = sim.offsets
    for c in range(len(counts)):
        sl = slice(off[c], off[c + 1])
        N = counts[c]
        scale = math.sqrt(gas.R * Ttr[c]) + 300.0 * c
        for k in ("cx", "cy", "cz"):
            assert abs(st1[k][sl].sum() - st0[k][sl].sum()) < 1e-11 * N * scale
        E = lambda s: (0.5 * (s["cx"][sl] ** 2 + s["cy"][sl] ** 2 + s["cz"][sl] ** 2).sum()
                       + s["erot"][sl].sum() + RTh * s["vib"][sl].sum())
        assert abs(E(st1) - E(st0)) < 1e-11 * abs(E(st0))
        assert abs(st1["erot"][sl].mean() - _cs(sim, "EROT_NEW", c)) < 1e-11 * abs(_cs(sim, "EROT_NEW", c))
        assert abs(st1["vib"][sl].mean() * RTh - _cs(sim, "EVIB_NEW", c)) <= RTh / N * (1 + 1e-9)


def test_positivity_fallback_keeps_update_finite():
    """A strongly anisotropic sampled cell fails the first Cholesky test for
    some of its particles; after the nu clamp and alpha refit of Sec.
    III.A.3 every update stays finite (the refit's own properties are
    pinned on hand-made Pi below)."""
    rng = np.random.default_rng(27)
    gas = W.Gas()
    N = 20000
    s = math.sqrt(gas.R * 300.0)
    cx = 12.0 * s * rng.standard_normal(N)
    cy = 0.3 * s * rng.standard_normal(N)
    cz = 0.3 * s * rng.standard_normal(N)
    erot = rng.exponential(gas.R * 8000.0, N)
    vib = np.zeros(N, np.int32)
    # nu ~ -0.88 at dt = 0.3 tau_c: R T_rel + nu (lambda_max - R T) < 0
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, dt_over_tauc=0.3, gas=gas)
    assert _cs(sim, "NU") < -0.8
    sim.collide(0)
    cnt = sim.cnt()
    assert cnt["CHOL_FALLBACK"] > 0
    st = sim.state()
    for k in ("cx", "cy", "cz", "erot"):
        assert np.all(np.isfinite(st[k]))
    assert np.all(st["erot"] >= 0)


# --------------------------------------------------------------------------
# The positivity fallback of Sec. III.A.3 on hand-made anisotropic Pi
# --------------------------------------------------------------------------
SHRINK = 1.0 - 2.0 ** -20


def _coef_cell(gas, T, Trot, dt_over_tauc, seed):
    """Cell coefficients (from the oracle's cell state of a sampled cell)."""
    rng = np.random.default_rng(seed)
    N = 4000
    s = math.sqrt(gas.R * T)
    cx, cy, cz = (s * rng.standard_normal(N) for _ in range(3))
    erot = rng.exponential(gas.R * Trot, N)
    prob, sim = _cell_problem(cx, cy, cz, erot, np.zeros(N, np.int32), gas=gas,
                              dt_over_tauc=dt_over_tauc)
    return {k: _cs(sim, k) for k in ("A", "B", "ALPHA", "OMA2", "NU", "R2", "MUP", "PR", "DT")}


def _sym(M):
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def _full(v):
    return np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])


def _refit_cases(gas, cc, Ts, aniso, seed):
    """Every combination of particle temperatures and Pi eigenvalue ratios
    (Pi = R T_tr Q diag(d) Q^T, trace 3 R T_tr, random rotation Q), with the
    oracle's coefficients and the same particle with an isotropic Pi (whose
    Lambda is R T_tr^rel I, so it gives the relaxation temperatures before
    any refit)."""
    rng = np.random.default_rng(seed)
    R = gas.R
    out = []
    for Ttr, Trot, Tvib in Ts:
        for d in aniso:
            d = np.asarray(d, float) * 3.0 / sum(d)
            Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
            Pm = R * Ttr * (Q @ np.diag(d) @ Q.T)
            args = (cc["A"], cc["B"], cc["ALPHA"], cc["OMA2"], cc["NU"], cc["R2"],
                    2.0 * cc["MUP"], cc["PR"], cc["DT"])
            r = oracle.particle_coef(gas, Ttr, Trot, Tvib, _sym(Pm), *args)
            iso = oracle.particle_coef(gas, Ttr, Trot, Tvib, _sym(R * Ttr * np.eye(3)), *args)
            # an isotropic Pi fails only through T_tr^rel <= 0, and then
            # before any refit: iso always holds the unrefitted values
            assert iso["fallback"] == (not iso["Ttr_rel"] > 0)
            out.append((Ttr, Trot, Tvib, Pm, r, iso))
    return out


def _check_refit(gas, cc, case):
    """The properties eqs. nu_USP_positivity and alpha_USP_positivity_1..4
    fix, evaluated independently of the oracle's arithmetic (eigenvalues by
    numpy, the bound from the pre-refit relaxation temperature).  Returns
    which branch the case took."""
    Ttr, Trot, Tvib, Pm, r, iso = case
    R = gas.R
    RT = R * Ttr
    if not r["fallback"]:
        # the first test passed: Lambda with the cell's nu is positive definite
        Lam = R * iso["Ttr_rel"] * np.eye(3) + cc["NU"] * (Pm - RT * np.eye(3))
        assert np.linalg.eigvalsh(Lam).min() > 0
        return "pass"
    Lam0 = R * iso["Ttr_rel"] * np.eye(3) + cc["NU"] * (Pm - RT * np.eye(3))
    assert np.linalg.eigvalsh(Lam0).min() <= 1e-12 * RT
    if not iso["Ttr_rel"] > 0:
        assert r["skip"]
        return "skip"
    lam = np.linalg.eigvalsh(Pm)
    RTr = R * iso["Ttr_rel"]
    nu0 = cc["NU"]
    # eq. nu_USP_positivity: the admissible interval (eigenvalues by numpy)
    lo = -RTr / (lam[2] - RT) if lam[2] > RT else -np.inf
    hi = RTr / (RT - lam[0]) if lam[0] < RT else np.inf
    # the oracle's bound on nu's side agrees with it (the closed-form
    # eigenvalues lose up to ~1e-8 relative where two eigenvalues coincide)
    bound = lo if nu0 <= 0 else hi
    if np.isfinite(bound):
        assert r["nu_bound"] == pytest.approx(bound, rel=1e-7)
        nu1 = max(nu0, r["nu_bound"] * SHRINK) if nu0 <= 0 else min(nu0, r["nu_bound"] * SHRINK)
    else:
        assert r["nu_bound"] == 0.0
        nu1 = nu0
    # the clamped nu lies strictly inside the interval
    assert lo < nu1 < hi
    # eq. alpha_USP_positivity_1: alpha^2 from the clamped nu and r2
    a2 = min(1.0, max(0.0, (nu1 - cc["R2"]) / (nu1 - 1.0)))
    assert r["al"] ** 2 == pytest.approx(a2, rel=1e-12, abs=1e-15)
    assert r["oma2"] == pytest.approx(1.0 - a2, rel=1e-12, abs=1e-15)
    # eq. alpha_USP_positivity_3: of +-sqrt(alpha^2), the Pr closer to the cell's
    def prandtl(al):
        return 2.0 * cc["MUP"] * (1.0 - al ** 3) / (cc["DT"] * (1.0 + al ** 3))
    ap = math.sqrt(a2)
    dp, dm = abs(prandtl(ap) - cc["PR"]), abs(prandtl(-ap) - cc["PR"])
    if dp != dm:
        assert r["al"] == pytest.approx(ap if dp < dm else -ap, rel=1e-14, abs=1e-15)
    # the relaxation temperature with the new 1 - alpha^2 (eq. T_tr_USP):
    # T_tr - (T_tr - T_tr^rel,0) (1 - alpha_0^2)/(1 - alpha^2)
    Trel1 = Ttr - (Ttr - iso["Ttr_rel"]) * cc["OMA2"] / r["oma2"]
    assert r["Ttr_rel"] == pytest.approx(Trel1, rel=1e-11)
    Lam1 = R * Trel1 * np.eye(3) + nu1 * (Pm - RT * np.eye(3))
    pd = np.linalg.eigvalsh(Lam1).min() > 1e-9 * RT
    L = r["L"]
    Lm = np.array([[L[0], 0, 0], [L[1], L[2], 0], [L[3], L[4], L[5]]])
    if r["nu_zero"]:
        # the second fallback fires exactly when the re-test fails
        assert np.linalg.eigvalsh(Lam1).min() < 1e-9 * RT
        assert r["nu"] == 0.0
        if Trel1 > 0:
            assert np.allclose(Lm @ Lm.T, R * Trel1 * np.eye(3), rtol=1e-12)
        return "nu_zero"
    assert pd
    assert r["nu"] == pytest.approx(nu1, rel=1e-14)
    assert np.allclose(Lm @ Lm.T, Lam1, rtol=1e-10, atol=1e-10 * RT)
    return "refit"


ANISO = [(1, 1, 1), (2, 1, 0.5), (4, 1, 1), (8, 1, 1), (20, 1, 1), (1, 1, 0.05), (1, 0.02, 0.02),
         (50, 0.5, 0.1)]


def test_positivity_refit_negative_nu():
    """nu < 0 (the Eucken Prandtl number): a Pi with a large eigenvalue fails
    the first test; nu is clamped to just inside -R T_rel/(lambda_max - R T),
    alpha^2 refitted, the Pr-closer sign taken, and the re-test decides
    between the refitted tensor (positive definite) and nu = 0.  Energy
    flowing into translation (T_rot > T_tr) raises T_tr^rel with the new
    1 - alpha^2 the other way, which is where the re-test can fail."""
    gas = W.Gas()
    seen = set()
    for dto, seed in ((0.3, 1), (1.0, 2), (3.0, 3), (10.0, 4)):
        cc = _coef_cell(gas, 3000.0, 3000.0, dto, seed)
        assert cc["NU"] < 0
        Ts = [(3000.0, 3000.0, 3000.0), (3000.0, 300.0, 300.0), (3000.0, 12000.0, 3000.0),
              (3000.0, 30000.0, 5000.0), (1000.0, 60000.0, 1000.0)]
        for case in _refit_cases(gas, cc, Ts, ANISO, seed):
            seen.add(_check_refit(gas, cc, case))
    assert {"pass", "refit", "nu_zero"} <= seen, seen


def test_positivity_refit_positive_nu():
    """nu > 0 (a constant Prandtl number above 3/2): a Pi with a small
    eigenvalue fails the first test, which needs R T_tr^rel < nu (R T -
    lambda_min) < R T_tr, i.e. energy leaving translation.  nu is clamped to
    just inside R T_rel/(R T - lambda_min).  Lowering nu raises alpha^2
    (d alpha^2/d nu = (r2 - 1)/(nu - 1)^2 < 0), so 1 - alpha^2 falls and
    T_tr^rel falls below the value the bound was taken at: under this
    reading the re-test then fails and nu = 0 is used, in every case."""
    gas = W.Gas(pr_model=W.PR_CONST, Pr_const=2.5, Z_rot=0.5)
    seen = set()
    for dto, seed in ((0.1, 5), (0.3, 6), (0.6, 7)):
        cc = _coef_cell(gas, 3000.0, 3000.0, dto, seed)
        assert cc["NU"] > 0
        Ts = [(3000.0, 3000.0, 3000.0), (3000.0, 300.0, 300.0), (3000.0, 10.0, 10.0),
              (3000.0, 12000.0, 3000.0)]
        for case in _refit_cases(gas, cc, Ts, ANISO + [(1, 1e-3, 1e-3)], seed):
            seen.add(_check_refit(gas, cc, case))
    assert {"pass", "nu_zero"} <= seen and "refit" not in seen, seen
