"""Pins of the oracle's first-order FPM mode (Secs. II.B-II.C): one-step
moment decays that follow from the Langevin updates and the master
equation, the first-order Landau-Teller rates of the relaxation
temperatures, the conservation of momentum and energy, and the paper's
contrast of FPM and USP-FPM relaxations at a large time step."""
import math

import numpy as np
from scipy import stats

import oracle
import usp_workloads as W
from test_oracle_collide import _cell_problem, _cs, _mom
from test_oracle_targets import _lt_rk4


def _fpm_gas(**kw):
    return W.Gas(scheme=W.SCHEME_FPM, **kw)


def _sample(rng, N, T, gas, sx=1.0, sy=1.0, sz=1.0, Trot=None, Tvib=None):
    s = math.sqrt(gas.R * T)
    cx = sx * s * rng.standard_normal(N)
    cy = sy * s * rng.standard_normal(N)
    cz = sz * s * rng.standard_normal(N)
    erot = rng.exponential(gas.R * (Trot or T), N)
    q = math.exp(-gas.theta_vib / (Tvib or T))
    vib = rng.geometric(1 - q, N) - 1
    return cx, cy, cz, erot, vib


def test_fpm_cell_coefficients_are_the_fpm_ones():
    """nu = 1 - 3/(2 Pr) (the FPM Prandtl relation), tau = 2 mu (1-nu)/p and
    the update factor exp(-dt/tau): Pr = 3/(2(1-nu)) is recovered."""
    rng = np.random.default_rng(1)
    gas = _fpm_gas()
    prob, sim = _cell_problem(*_sample(rng, 2000, 3000.0, gas), gas=gas, dt_over_tauc=0.7)
    nu, Pr = _cs(sim, "NU"), _cs(sim, "PR")
    assert abs(3.0 / (2.0 * (1.0 - nu)) - Pr) < 1e-12
    tau = _cs(sim, "FPM_TAU")
    assert abs(tau - 2.0 * _cs(sim, "MU") * (1.0 - nu) / (_cs(sim, "NDENS") * 1.380649e-23 * _cs(sim, "TTR"))) < 1e-12 * tau
    assert abs(_cs(sim, "ALPHA") - math.exp(-_cs(sim, "DT") / tau)) < 1e-14
    assert abs(_cs(sim, "OMA2") - (1 - math.exp(-2 * _cs(sim, "DT") / tau))) < 1e-14


def test_fpm_stress_decay_factor():
    """One FPM velocity update multiplies the viscous stress by
    nu + (1 - nu) exp(-2 dt/tau) in expectation (from E[C'C'|C] =
    alpha^2 CC + (1-alpha^2) Lambda); its expansion is the paper's
    1 - 2(1-nu) dt/tau + 2(1-nu) dt^2/tau^2."""
    rng = np.random.default_rng(2)
    gas = _fpm_gas()
    N = 1_000_000
    cx, cy, cz, erot, vib = _sample(rng, N, 3000.0, gas, sx=1.5, sz=0.8)
    cx += 0.3 * cy
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, gas=gas, dt_over_tauc=1.0)
    nu, tau, dt = _cs(sim, "NU"), _cs(sim, "FPM_TAU"), _cs(sim, "DT")
    factor = nu + (1.0 - nu) * math.exp(-2.0 * dt / tau)
    x = dt / tau
    assert abs(factor - (1 - 2 * (1 - nu) * x + 2 * (1 - nu) * x * x)) < 2 * (1 - nu) * x ** 3
    P0 = {k: _mom(sim, k) for k in ("PXX", "PYY", "PXY")}
    sim.collide(0)
    sim.do_moments()
    P1 = {k: _mom(sim, k) for k in ("PXX", "PYY", "PXY")}
    RT = gas.R * _cs(sim, "TTR")
    assert abs((P1["PXX"] - P1["PYY"]) - factor * (P0["PXX"] - P0["PYY"])) < 0.01 * RT
    assert abs(P1["PXY"] - factor * P0["PXY"]) < 0.01 * RT
    # the USP-FPM factor (2mu/p - dt)/(2mu/p + dt) differs clearly here
    A = 2 * _cs(sim, "MUP")
    assert abs(factor - (A - dt) / (A + dt)) > 0.05


def test_fpm_heat_flux_decay_all_modes():
    """q_tr, q_rot and q_vib each decay by exp(-3 dt/tau) per step: the
    velocity keeps alpha C, and E[eps'|eps] and E[I'|I] are affine in eps
    and I with slope alpha^2."""
    rng = np.random.default_rng(3)
    gas = _fpm_gas()
    N = 2_000_000
    T = 2500.0
    s = math.sqrt(gas.R * T)
    cx = s * rng.standard_normal(N)
    cy = s * rng.standard_normal(N)
    cz = s * rng.standard_normal(N)
    # heat fluxes: skew the x velocity and correlate it with eps and I
    cx = cx + 0.3 * (cx ** 2 - s * s) / s
    erot = rng.exponential(gas.R * T, N) * np.exp(0.2 * cx / s)
    q0 = math.exp(-gas.theta_vib / T)
    vib = rng.geometric(1 - q0, N) - 1 + (cx > s).astype(int)
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, gas=gas, dt_over_tauc=1.0)
    a3 = math.exp(-3.0 * _cs(sim, "DT") / _cs(sim, "FPM_TAU"))
    Q0 = {k: _mom(sim, k) for k in ("QTRX", "QROTX", "QIX")}
    sim.collide(0)
    sim.do_moments()
    Q1 = {k: _mom(sim, k) for k in ("QTRX", "QROTX", "QIX")}
    for k in Q0:
        assert abs(Q1[k] / Q0[k] - a3) < 0.03, (k, Q1[k] / Q0[k], a3)


def test_fpm_gillespie_mean_level_and_equilibrium():
    """The master equation's rates are linear in I, so the mean level
    relaxes exactly as m_rel + (m - m_rel) exp(-2 dt/tau); at equilibrium the
    Boltzmann (geometric) levels are invariant."""
    rng = np.random.default_rng(4)
    gas = _fpm_gas(Z_vib=5.0)
    N = 1_000_000
    # out of equilibrium: T_vib below T_tr
    prob, sim = _cell_problem(*_sample(rng, N, 6000.0, gas, Tvib=2000.0), gas=gas,
                              dt_over_tauc=1.5)
    m0, mrel = _mom(sim, "IBAR"), _cs(sim, "FPM_MREL")
    e2 = math.exp(-2.0 * _cs(sim, "DT") / _cs(sim, "FPM_TAU"))
    I0 = sim.state()["vib"].copy()
    sim.collide(0)
    I1 = sim.state()["vib"]
    expect = mrel + (m0 - mrel) * e2
    se = np.std(I1 - I0) / math.sqrt(N)
    assert abs(I1.mean() - expect) < 5 * se + 1e-12, (I1.mean(), expect, se)
    assert mrel > m0 and I1.mean() > m0
    # equilibrium: levels stay geometric with q = exp(-Theta/T)
    T = 5000.0
    prob, sim = _cell_problem(*_sample(rng, N, T, gas), gas=gas, dt_over_tauc=2.0)
    sim.collide(0)
    I = sim.state()["vib"]
    q = math.exp(-gas.theta_vib / T)
    kmax = 12
    obs = np.bincount(np.minimum(I, kmax), minlength=kmax + 1)
    p = (1 - q) * q ** np.arange(kmax + 1)
    p[-1] = q ** kmax
    chi2 = ((obs - N * p) ** 2 / (N * p)).sum()
    assert stats.chi2.sf(chi2, kmax) > 1e-4, chi2


def test_fpm_relaxation_temperatures_first_order_landau_teller():
    """One FPM step moves e_rot by (1-alpha^2)(e_rot(T_rot^rel) - e_rot) and
    e_vib by (1-alpha^2)(e_vib(T_vib^rel) - e_vib) in expectation; per unit
    time this tends to the Landau-Teller rates (e(T_tr) - e)/tau_mode, and
    the error is first order in dt (it halves with dt): the paper's FPM
    accuracy statement."""
    rng = np.random.default_rng(5)
    gas = _fpm_gas(Z_rot=10.0, Z_vib=50.0)
    G = oracle.Gas(gas)
    R = gas.R
    cx, cy, cz, erot, vib = _sample(rng, 4000, 6000.0, gas, Trot=4000.0, Tvib=2000.0)
    errs = {"rot": [], "vib": [], "tr": []}
    for f in (0.4, 0.2, 0.1):
        prob, sim = _cell_problem(cx, cy, cz, erot, vib, gas=gas, dt_over_tauc=f)
        dt, oma2 = _cs(sim, "DT"), _cs(sim, "OMA2")
        Ttr, Trot, Tvib, tc = _cs(sim, "TTR"), _cs(sim, "TROT"), _cs(sim, "TVIB"), _cs(sim, "TAUC")
        tr, tv = _cs(sim, "ZROT") * tc, _cs(sim, "ZVIB") * tc
        lt_rot = R * (Ttr - Trot) / tr
        lt_vib = (G.e_vib(Ttr) - G.e_vib(Tvib)) / tv
        d_rot = oma2 * R * (_cs(sim, "FPM_TROT_REL") - Trot) / dt
        d_vib = oma2 * R * gas.theta_vib * (_cs(sim, "FPM_MREL") - _mom(sim, "IBAR")) / dt
        d_tr = oma2 * 1.5 * R * (_cs(sim, "FPM_TTR_REL") - Ttr) / dt
        errs["rot"].append(abs(d_rot / lt_rot - 1))
        errs["vib"].append(abs(d_vib / lt_vib - 1))
        errs["tr"].append(abs(d_tr / -(lt_rot + lt_vib) - 1))
    for k, e in errs.items():
        assert e[-1] < 0.1, (k, e)
        r1, r2 = e[0] / e[1], e[1] / e[2]
        assert 1.7 < r1 < 2.3 and 1.7 < r2 < 2.3, (k, e)


def test_fpm_conserve_momentum_energy_only():
    """FPM conservation: momentum and total energy per cell to round-off,
    levels and rotational energies as sampled."""
    rng = np.random.default_rng(6)
    gas = _fpm_gas()
    N = 50_000
    cells = np.repeat(np.arange(5, dtype=np.int32), N // 5)
    cx, cy, cz, erot, vib = _sample(rng, N, 4000.0, gas, Trot=2000.0, Tvib=1500.0)
    prob, sim = _cell_problem(cx, cy, cz, erot, vib, gas=gas, dt_over_tauc=1.0, cells=cells)
    mom0 = sim.moments()
    sim.collide(0)
    before = sim.state()
    sim.conserve(0)
    after = sim.state()
    assert np.array_equal(before["vib"], after["vib"])
    assert np.array_equal(before["erot"], after["erot"])
    sim.do_moments()
    mom1 = sim.moments()
    iN = oracle.MOM_NAMES.index
    R, Th = gas.R, gas.theta_vib
    for c in range(5):
        U0 = mom0[iN("UX"):iN("UZ") + 1, c]
        U1 = mom1[iN("UX"):iN("UZ") + 1, c]
        assert np.abs(U1 - U0).max() < 1e-9 * math.sqrt(R * 4000.0)
        E = lambda m: 0.5 * (m[iN("PXX"), c] + m[iN("PYY"), c] + m[iN("PZZ"), c]) + m[iN("EROT"), c] + R * Th * m[iN("IBAR"), c]
        assert abs(E(mom1) - E(mom0)) < 1e-10 * E(mom0)


def test_fpm_lags_usp_at_large_time_step():
    """The paper's relaxation to equilibrium (T_tr 6000, T_rot 4000,
    T_vib 2000 K, n = 1e24, Z_rot 10, Z_vib 50) at dt = 2 tau_c: the FPM
    temperatures deviate from the Landau-Teller solution far more than the
    USP-FPM ones (table tab:L2norm_temp: about 1% vs below 0.1%)."""
    rng = np.random.default_rng(7)
    N, nsteps = 100_000, 40
    res = {}
    for scheme in (W.SCHEME_USP, W.SCHEME_FPM):
        gas = W.Gas(scheme=scheme, Z_rot=10.0, Z_vib=50.0)
        G = oracle.Gas(gas)
        R = gas.R
        cx, cy, cz, erot, vib = _sample(rng, N, 6000.0, gas, Trot=4000.0, Tvib=2000.0)
        prob, sim = _cell_problem(cx, cy, cz, erot, vib, n_dens=1e24, gas=gas,
                                  dt_over_tauc=2.0, seed=17)
        hist = []
        for s in range(nsteps):
            sim.bin(); sim.do_moments(); sim.do_cellstate()
            cs = sim.cellstate()
            hist.append([cs[oracle.CS_NAMES.index(k), 0] for k in ("TTR", "TROT", "TVIB")])
            sim.collide(s); sim.conserve(s)
        hist = np.array(hist)

        def tau_of(Ttr):
            tc = G.tau_c(Ttr, 1e24)
            return gas.Z_rot * tc, gas.Z_vib * tc

        T0 = hist[0]
        y0 = [1.5 * R * T0[0], R * T0[1], G.e_vib(T0[2])]
        sub = 40
        ref = _lt_rk4(gas, y0, nsteps * prob.dt, tau_of, prob.dt / sub)[::sub][:nsteps]
        Tref = np.stack([ref[:, 0] / (1.5 * R), ref[:, 1] / R,
                         gas.theta_vib / np.log1p(R * gas.theta_vib / ref[:, 2])], 1)
        res[scheme] = np.sqrt(((hist - Tref) ** 2).mean(axis=0)) / np.sqrt((Tref ** 2).mean(axis=0))
    usp, fpm = res[W.SCHEME_USP], res[W.SCHEME_FPM]
    assert np.all(usp < 2e-3), usp
    assert fpm[0] > 3 * usp[0] and fpm[2] > 3 * usp[2], (fpm, usp)
    assert 3e-3 < fpm[0] < 3e-2, fpm
