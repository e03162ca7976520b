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
    """A strongly anisotropic cell fails the first
    Cholesky test; the nu clamp and alpha refit of Sec. III.A.3 restore a
    positive-definite diffusion tensor (parity of the refit itself is not
    pinned by the paper)."""
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
