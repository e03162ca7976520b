"""Pin of the oracle's full step against the near-continuum Poiseuille
flow (the force-driven channel of Sec. V.B): after the transient, the
time-averaged velocity profile is a parabola whose curvature is
g / (2 nu) with nu = mu(T)/rho from the gas model (the method reproduces
the viscosity it is built from), plus a wall slip of the size of the
first-order Maxwell slip lambda du/dy at Kn = 0.05.  The parabola is fitted
over the cells more than two mean free paths from either wall: the
Knudsen layers next to the walls follow no Navier-Stokes profile.  No GPU."""
import numpy as np
import pytest

import oracle
import usp_workloads as W


def bulk_fit(y, U, L, mfp, walls=2.0):
    """Least-squares U = curv y (L - y) + slip over the cells farther than
    `walls` mean free paths from both walls; returns (curv, slip) and the
    standard error of curv from the residuals."""
    m = (y > walls * mfp) & (y < L - walls * mfp)
    A = np.stack([y[m] * (L - y[m]), np.ones(m.sum())], 1)
    coef, *_ = np.linalg.lstsq(A, U[m], rcond=None)
    r = U[m] - A @ coef
    cov = (r @ r) / (m.sum() - 2) * np.linalg.inv(A.T @ A)
    return coef, float(np.sqrt(cov[0, 0]))


def test_poiseuille_profile_curvature_and_slip():
    prob = W.poiseuille(kn=0.05, cells=40, ppc=150, f32=False, seed=7)
    parts = W.particles_for(prob)
    sim = oracle.Sim(prob, parts)
    g = prob.grid
    M, L = g.ny, g.ny * g.dy
    transient, sampled = 1500, 3000   # the slowest mode decays in ~360 steps
    sN, sU, sT = np.zeros(M), np.zeros(M), np.zeros(M)
    for s in range(transient + sampled):
        sim.step_native(s, 1)
        if s >= transient:
            m = sim.moments()
            sN += m[0]
            sU += m[0] * m[1]
            sT += m[0] * (m[4] + m[5] + m[6])
    U = sU / sN
    gas = prob.gas
    T = (sT / sN).mean() / (3 * gas.R)
    assert abs(T - 300.0) < 5.0          # Ma ~ 0.1: little viscous heating
    mu = gas.mu_ref * (T / gas.T_ref) ** gas.omega
    nu = mu / (prob.notes["n"] * gas.m)
    y = (np.arange(M) + 0.5) * g.dy
    (curv, slip), sd = bulk_fit(y, U, L, 50e-6)
    g_x = prob.bc.g[0]
    # 4500 steps of 6000 particles: the fit's own noise is ~5% (sd)
    assert abs(curv / (g_x / (2 * nu)) - 1.0) < 0.08, curv / (g_x / (2 * nu))
    # mean free path c_bar tau_c = 50 um at this density (Kn = 0.05)
    u_slip1 = 50e-6 * g_x * L / (2 * nu)
    assert 0.5 * u_slip1 < slip < 2.5 * u_slip1, (slip, u_slip1)
    # symmetric about the centre line
    assert np.abs(U - U[::-1]).mean() < 0.08 * U.max()


@pytest.mark.parametrize("kn,golden,mfp", [(0.05, "poiseuille_kn005_200x1000.txt", 50e-6),
                                           (0.01, "poiseuille_kn001_200x1000.txt", 10e-6)])
def test_stored_full_size_profile(kn, golden, mfp):
    """The stored oracle profiles of the full-size channel (200 cells x 1000
    particles, tests/golden/) meet the same continuum pins: NS curvature
    over the bulk within 5% (measured 1.042 +- 0.005 at Kn = 0.05, where
    the O(Kn^2) departures from Navier-Stokes are largest, and 0.974 +-
    0.004 at Kn = 0.01, whose step is 1.9 tau_c), a positive slip of the
    first-order size lambda du/dy (mean free path c_bar tau_c = Kn x gap),
    symmetric, T near the wall temperature."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", golden)
    T, U = None, []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        if k == "T_tr":
            T = float(v)
        else:
            U.append(float(v))
    U = np.array(U)
    prob = W.poiseuille(kn=kn, cells=200, ppc=1000, f32=True)
    g, gas = prob.grid, prob.gas
    M, L = g.ny, g.ny * g.dy
    assert U.size == M and abs(T - 300.0) < 5.0
    y = (np.arange(M) + 0.5) * g.dy
    (curv, slip), sd = bulk_fit(y, U, L, mfp)
    mu = gas.mu_ref * (T / gas.T_ref) ** gas.omega
    g_x = prob.bc.g[0]
    ratio = curv / (g_x / (2 * mu / (prob.notes["n"] * gas.m)))
    assert abs(ratio - 1.0) < 0.05, ratio
    assert sd < 0.01 * curv
    nu = mu / (prob.notes["n"] * gas.m)
    u_slip1 = mfp * g_x * L / (2 * nu)
    assert 0.5 * u_slip1 < slip < 2.5 * u_slip1, (slip, u_slip1)
    assert np.abs(U - U[::-1]).mean() < 0.03 * U.max()
