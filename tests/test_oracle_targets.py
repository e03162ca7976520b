"""Pins of the oracle's second-order energy exchange (Sec. III.A.1) against
the Landau-Teller equations of Sec. II.A, integrated independently here."""
import math

import numpy as np
import pytest

import oracle
import usp_workloads as W


def _lt_rk4(gas, y0, t_end, tau_of, h):
    """RK4 for the Landau-Teller system in (e_tr, e_rot, e_vib) (Sec. II.A).
    tau_of(T_tr) -> (tau_rot, tau_vib)."""
    R, Th = gas.R, gas.theta_vib

    def ev(T):
        return R * Th / math.expm1(Th / T) if T > 0 else 0.0

    def inv_ev(e):
        return Th / math.log1p(R * Th / e) if e > 0 else 0.0

    def rhs(y):
        Ttr, Trot, Tv = y[0] / (1.5 * R), y[1] / R, inv_ev(y[2])
        tr, tv = tau_of(Ttr)
        fr = R * (Ttr - Trot) / tr
        fv = (ev(Ttr) - ev(Tv)) / tv
        return np.array([-fr - fv, fr, fv])

    y = np.array(y0, float)
    out = [y.copy()]
    n = int(round(t_end / h))
    for _ in range(n):
        k1 = rhs(y); k2 = rhs(y + h / 2 * k1); k3 = rhs(y + h / 2 * k2); k4 = rhs(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        out.append(y.copy())
    return np.array(out)


def _target_step(G, R, Ttr, Trot, Tv, a, b):
    g, _ = G.gammas(Ttr, Trot, Tv, a, b)
    etr = 1.5 * R * Ttr - g[0] * (Ttr - Trot) - g[1] * (Ttr - Tv)
    erot = R * Trot + g[0] * (Ttr - Trot) - g[2] * (Trot - Tv)
    evib = G.e_vib(Tv) + g[1] * (Ttr - Tv) + g[2] * (Trot - Tv)
    return etr, erot, evib


def test_crank_nicolson_two_mode_closed_form():
    """With vibration frozen (b = 0) the targets are the trapezoidal step of
    d(T_tr - T_rot)/dt = -(5/3)(T_tr - T_rot)/tau_rot, i.e. the ratio
    (1 - 5dt/(6tau))/(1 + 5dt/(6tau)) per step."""
    gas = W.Gas()
    G = oracle.Gas(gas)
    R = G.R()
    for dt_over_tau in (0.01, 0.3, 1.0, 4.0):
        tau = 1.0
        dt = dt_over_tau * tau
        a = dt / (dt + 2 * tau)
        Ttr, Trot = 7000.0, 1500.0
        etr, erot, _ = _target_step(G, R, Ttr, Trot, 800.0, a, 0.0)
        theta1 = etr / (1.5 * R) - erot / R
        ratio = (1 - 5 * dt / (6 * tau)) / (1 + 5 * dt / (6 * tau))
        assert abs(theta1 / (Ttr - Trot) - ratio) < 1e-12


def test_targets_second_order_in_dt():
    """Iterating the targets with constant tau's converges to the
    Landau-Teller solution at second order (error ratio ~4 per halving)."""
    gas = W.Gas()
    G = oracle.Gas(gas)
    R = G.R()
    tau_r, tau_v = 5.0, 50.0
    y0 = [1.5 * R * 10000.0, R * 300.0, G.e_vib(300.0)]
    t_end = 20.0
    ref = _lt_rk4(gas, y0, t_end, lambda T: (tau_r, tau_v), 1e-3)[-1]
    errs = []
    for dt in (2.0, 1.0, 0.5):
        a, b = dt / (dt + 2 * tau_r), dt / (dt + 2 * tau_v)
        Ttr, Trot, Tv = 10000.0, 300.0, 300.0
        for _ in range(int(round(t_end / dt))):
            etr, erot, evib = _target_step(G, R, Ttr, Trot, Tv, a, b)
            Ttr, Trot = etr / (1.5 * R), erot / R
            Tv = gas.theta_vib / math.log1p(R * gas.theta_vib / evib)
        y = np.array([1.5 * R * Ttr, R * Trot, G.e_vib(Tv)])
        errs.append(np.max(np.abs(y - ref)) / y0[0])
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
    assert errs[2] < 1e-5


def test_tcheck_solves_its_equation():
    """The rescaled temperature solves e_tr(T)+a e_rot(T)+b e_vib(T) =
    e_tr(T_tr)+a e_rot(T_rot)+b e_vib(T_vib) (App. C, rotational bracket
    with tau_rot)."""
    G = oracle.Gas(W.Gas())
    R = G.R()
    rng = np.random.default_rng(0)
    for _ in range(100):
        Ttr, Trot, Tv = rng.uniform(50, 30000, 3)
        a, b = rng.uniform(0, 1, 2)
        T = G.tcheck(Ttr, Trot, Tv, a, b)
        lhs = (1.5 + a) * R * T + b * G.e_vib(T)
        rhs = 1.5 * R * Ttr + a * R * Trot + b * G.e_vib(Tv)
        assert abs(lhs - rhs) <= 1e-12 * rhs


def test_no_exchange_at_equilibrium():
    G = oracle.Gas(W.Gas())
    g, tc = G.gammas(4000.0, 4000.0, 4000.0, 0.3, 0.05)
    assert abs(tc - 4000.0) < 1e-9
    R = G.R()
    etr, erot, evib = _target_step(G, R, 4000.0, 4000.0, 4000.0, 0.3, 0.05)
    assert abs(etr / (1.5 * R) - 4000.0) < 1e-9 and abs(erot / R - 4000.0) < 1e-9


def test_relax0d_histories_follow_landau_teller():
    """0D relaxation through the full particle step: the cell temperatures
    follow the Landau-Teller ODE (tau's evaluated at the current T_tr, as the
    cell coefficients are) and head to the energy-closure equilibrium."""
    prob = W.relax0d(n_particles=5000)
    parts = W.particles_for(prob)
    sim = oracle.Sim(prob, parts)
    gas = prob.gas
    G = oracle.Gas(gas)
    R = G.R()
    nsteps = 200
    hist = []
    for s in range(nsteps):
        sim.bin(); sim.do_moments(); sim.do_cellstate()
        cs = sim.cellstate()
        hist.append([cs[oracle.CS_NAMES.index(k), 0] for k in ("TTR", "TROT", "TVIB")])
        sim.collide(s); sim.conserve(s)
    hist = np.array(hist)
    n = prob.notes["n"]

    def tau_of(Ttr):
        tc = G.tau_c(Ttr, n)
        return gas.Z_rot * tc, gas.Z_vib * tc

    T0 = hist[0]
    y0 = [1.5 * R * T0[0], R * T0[1], G.e_vib(T0[2])]
    sub = 20
    ref = _lt_rk4(gas, y0, nsteps * prob.dt, tau_of, prob.dt / sub)[::sub][:nsteps]
    Tref = np.stack([ref[:, 0] / (1.5 * R), ref[:, 1] / R,
                     gas.theta_vib / np.log1p(R * gas.theta_vib / np.maximum(ref[:, 2], 1e-300))], 1)
    err = np.abs(hist - Tref).max(axis=0)
    # within 1% of the initial T_tr (tau varies with T_tr inside a step)
    assert np.all(err < 0.01 * T0[0]), err
    # energy closure: E/N stays at its initial value, T's approach T_eq
    E0 = 1.5 * R * T0[0] + R * T0[1] + G.e_vib(T0[2])
    lo, hi = 100.0, 20000.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 2.5 * R * mid + G.e_vib(mid) > E0: hi = mid
        else: lo = mid
    Teq = 0.5 * (lo + hi)
    assert abs(Teq - 4797.0) < 5.0
    assert hist[-1, 2] < Teq < hist[-1, 0]
