"""Pins of the oracle's free flight and boundaries (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import usp_workloads as W

KB = 1.380649e-23


def _parts2d(x, y, cx, cy, cz, erot=None, vib=None, cap=None):
    n = len(x)
    cap = cap or n
    z = lambda dt=np.float64: np.zeros(cap, dt)
    out = dict(n=n, cap=cap, x=z(), y=z(), cx=z(), cy=z(), cz=z(), erot=z(),
               vib=np.zeros(cap, np.int32), cell=np.zeros(cap, np.int32),
               pid=np.arange(cap, dtype=np.uint32), next_pid=n)
    for k, v in (("x", x), ("y", y), ("cx", cx), ("cy", cy), ("cz", cz)):
        out[k][:n] = v
    if erot is not None:
        out["erot"][:n] = erot
    if vib is not None:
        out["vib"][:n] = vib
    return out


def _box(nx=10, ny=10, L=1.0, kinds=(W.BC_SPECULAR,) * 4, **bckw):
    grid = W.Grid(dim=2, nx=nx, ny=ny, x0=0.0, y0=0.0, dx=L / nx, dy=L / ny, fnum=1.0,
                  volume=np.full(nx * ny, (L / nx) * (L / ny)), flags=np.zeros(nx * ny, np.uint8))
    return grid, W.BC(kind=kinds, **bckw)


def test_free_flight_is_exact():
    grid, bc = _box()
    rng = np.random.default_rng(1)
    n = 1000
    x, y = 0.3 + 0.4 * rng.random(n), 0.3 + 0.4 * rng.random(n)
    c = rng.standard_normal((3, n))
    prob = W.Problem("t", W.Gas(), grid, bc, dt=0.1, seed=1, f32=False)
    sim = oracle.Sim(prob, _parts2d(x, y, *c))
    sim.advect(0)
    st = sim.state()
    assert np.all(st["x"] == x + c[0] * 0.1) and np.all(st["y"] == y + c[1] * 0.1)
    ix = np.floor(st["x"] / 0.1).astype(int)
    iy = np.floor(st["y"] / 0.1).astype(int)
    assert np.array_equal(st["cell"], iy * 10 + ix)


def test_specular_reflection():
    grid, bc = _box()
    prob = W.Problem("t", W.Gas(), grid, bc, dt=1.0, seed=1, f32=False)
    sim = oracle.Sim(prob, _parts2d([0.5], [0.05], [0.1], [-0.25], [0.3]))
    sim.advect(0)
    st = sim.state()
    assert st["y"][0] == pytest.approx(0.2, abs=1e-15)
    assert st["cy"][0] == 0.25 and st["x"][0] == pytest.approx(0.6)


def test_diffuse_wall_reemission_moments():
    """Full accommodation at T_w: flux-weighted half-range normal speed
    (mean sqrt(pi R T_w / 2), mean square 2 R T_w), Gaussian tangential
    components (variance R T_w), rotational energy mean R T_w, Boltzmann
    levels at T_w."""
    gas = W.Gas()
    Tw = 4000.0
    grid = W.Grid(dim=1, nx=1, ny=4, y0=0.0, dy=0.25, fnum=1.0, volume=np.ones(4),
                  flags=np.zeros(4, np.uint8))
    bc = W.BC(kind=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_DIFFUSE, W.BC_DIFFUSE), Tw=(0, 0, Tw, Tw))
    n = 200_000
    dt = 1e-9
    y = np.full(n, 1e-9)
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=3, f32=False)
    parts = dict(n=n, cap=n, x=None, y=y, cx=np.zeros(n), cy=np.full(n, -10.0), cz=np.zeros(n),
                 erot=np.zeros(n), vib=np.zeros(n, np.int32), cell=np.zeros(n, np.int32),
                 pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.advect(0)
    st = sim.state()
    assert sim.cnt()["WALL_HITS"] == n
    R = gas.R
    cn = st["cy"]
    assert np.all(cn > 0)
    se = lambda v: np.std(v) / math.sqrt(n)
    assert abs(cn.mean() - math.sqrt(math.pi * R * Tw / 2)) < 4 * se(cn)
    assert abs((cn ** 2).mean() - 2 * R * Tw) < 4 * se(cn ** 2)
    for k in ("cx", "cz"):
        assert abs(st[k].var() / (R * Tw) - 1) < 0.01
    assert abs(st["erot"].mean() / (R * Tw) - 1) < 0.01
    q = math.exp(-gas.theta_vib / Tw)
    hist = np.bincount(st["vib"], minlength=6)[:6] / n
    assert np.allclose(hist, (1 - q) * q ** np.arange(6), atol=0.004)


def _speed_cdf(s):
    f = lambda u: u * math.exp(-(u - s) ** 2)
    lo, hi = 0.0, max(s, 0.0) + 8.0
    Z = integrate.quad(f, lo, hi, limit=200)[0]
    grid = np.linspace(lo, hi, 4001)
    pdf = np.array([f(u) for u in grid]) / Z
    cdf = np.concatenate([[0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    return lambda u: np.interp(u, grid, cdf)


@pytest.mark.parametrize("s", [-2.0, -0.5, 0.0, 0.3, 2.0, 8.4])
def test_inflow_speed_distribution(s):
    """Normal speeds of injected particles follow u e^{-(u-s)^2} on u > 0
    (the flux-weighted drifting Maxwellian), checked by Kolmogorov-Smirnov."""
    n = 20000
    u = np.array([oracle.inflow_speed(17, 5, pid, s) for pid in range(n)])
    assert np.all(u > 0)
    d, p = stats.kstest(u, _speed_cdf(s))
    assert p > 1e-3, (s, d, p)


def test_injection_count_matches_integrated_flux():
    """Expected injections per step on each free-stream side equal
    n * integral_{v_n > 0} v_n f(v_n) dv_n * area * dt / F_num (quadrature
    here, independent of the closed form the oracle uses)."""
    gas = W.Gas()
    T, n_inf = 300.0, 1e20
    U = (900.0, -400.0, 0.0)
    grid, bc = _box(nx=5, ny=4, L=0.02, kinds=(W.BC_FREESTREAM,) * 4, fs_n=n_inf, fs_T=T, fs_U=U,
                    depth=1.0)
    grid.fnum = 1e12
    dt = 2e-6
    R = gas.R
    sig = math.sqrt(R * T)

    def flux(Un):
        return n_inf * integrate.quad(lambda v: v * stats.norm.pdf(v, Un, sig), 0, Un + 12 * sig)[0]

    L = 0.02
    lam = (flux(U[0]) + flux(-U[0])) * L * dt / grid.fnum + (flux(U[1]) + flux(-U[1])) * L * dt / grid.fnum
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=9, f32=False)
    steps = 200
    cap = int(lam * steps * 1.3) + 100
    sim = oracle.Sim(prob, _parts2d([], [], [], [], [], cap=cap))
    for s in range(steps):
        sim.advect(s)
    got = sim.cnt()["INJECTED"]
    # floor(lambda_f + u) per face has variance <= 1/4 per face-step
    nf = 2 * 5 + 2 * 4
    assert abs(got - lam * steps) < 5 * math.sqrt(nf * steps * 0.25) + 1, (got, lam * steps)


def test_free_stream_is_preserved():
    """A box open on all sides to a drifting Maxwellian keeps its density,
    velocity and temperature through full steps (injection, deletion,
    collision at equilibrium)."""
    gas = W.Gas()
    T, n_inf = 500.0, 1e21
    U = (1500.0, 300.0, 0.0)
    nx = ny = 6
    L = 6e-3
    grid, bc = _box(nx=nx, ny=ny, L=L, kinds=(W.BC_FREESTREAM,) * 4, fs_n=n_inf, fs_T=T, fs_U=U,
                    depth=1.0)
    ppc = 200
    grid.fnum = n_inf * (L / nx) ** 2 / ppc
    dt = 2e-7
    rng = np.random.default_rng(5)
    N = ppc * nx * ny
    x, y = rng.random(N) * L, rng.random(N) * L
    s = math.sqrt(gas.R * T)
    c = rng.standard_normal((3, N)) * s + np.array(U)[:, None]
    erot = rng.exponential(gas.R * T, N)
    vib = rng.geometric(1 - math.exp(-gas.theta_vib / T), N) - 1
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=12, f32=False)
    sim = oracle.Sim(prob, _parts2d(x, y, *c, erot=erot, vib=vib, cap=3 * N))
    for st in range(30):
        sim.step(st)
    sim.bin()
    v = sim.state()
    assert abs(v["n"] / N - 1) < 0.05
    assert abs(v["cx"].mean() - U[0]) < 0.03 * s and abs(v["cy"].mean() - U[1]) < 0.03 * s
    Tm = ((v["cx"] - v["cx"].mean()) ** 2 + (v["cy"] - v["cy"].mean()) ** 2
          + (v["cz"] - v["cz"].mean()) ** 2).mean() / (3 * gas.R)
    assert abs(Tm / T - 1) < 0.03
    assert abs(v["erot"].mean() / (gas.R * T) - 1) < 0.05


def test_cylinder_wall_reemits_outward():
    gas = W.Gas()
    grid, bc = _box(nx=20, ny=10, L=0.2, kinds=(W.BC_SPECULAR,) * 4, cyl=1, cyl_xc=0.1,
                    cyl_yc=0.0, cyl_r=0.05, cyl_Tw=500.0)
    grid.dy = 0.1 / 10
    grid.ny = 10
    rng = np.random.default_rng(8)
    n = 5000
    ang = rng.uniform(0.05, math.pi - 0.05, n)
    rr = 0.05 + 0.002 * rng.random(n)
    x, y = 0.1 + rr * np.cos(ang), rr * np.sin(ang)
    cx, cy = -400 * np.cos(ang), -400 * np.sin(ang)
    prob = W.Problem("t", gas, grid, bc, dt=2e-5, seed=4, f32=False)
    sim = oracle.Sim(prob, _parts2d(x, y, cx, cy, np.zeros(n)))
    sim.advect(0)
    st = sim.state()
    r_end = np.hypot(st["x"] - 0.1, st["y"])
    assert sim.cnt()["WALL_HITS"] >= n
    assert np.all(r_end >= 0.05 - 1e-12)
    nrm = np.stack([st["x"] - 0.1, st["y"]]) / r_end
    vn = st["cx"] * nrm[0] + st["cy"] * nrm[1]
    assert np.mean(vn > 0) > 0.99


def test_native_step_equals_phase_sequence():
    prob = W.cylinder(scale=0.05, f32=True)
    parts = W.particles_for(prob)
    a = oracle.Sim(prob, parts)
    b = oracle.Sim(prob, parts)
    a.step(0, 3)
    b.step_native(0, 3)
    sa, sb = a.state(), b.state()
    assert sa["n"] == sb["n"] and sa["next_pid"] == sb["next_pid"]
    for k in ("x", "y", "cx", "cy", "cz", "erot", "vib", "cell", "pid"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.counters, b.counters)
