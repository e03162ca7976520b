"""Host post-processing of the sampled sums (paper_2508_05642_amd.sampling):
time averages of a known gas and free-molecular wall fluxes in physical
units, on sums the oracle accumulates.  No GPU."""
import math

import numpy as np
import pytest

import oracle
import usp_workloads as W
from paper_2508_05642_amd import sampling
from test_oracle_sampling import _cyl_expect, _cyl_problem, _maxwellian

KB = 1.380649e-23


def test_field_averages_recover_the_gas():
    """Cells of drifting Maxwellians with their own T_tr, T_rot, T_vib,
    sampled over several steps of a frozen state: the averages give back n,
    U and the three temperatures; an empty cell gives zeros."""
    gas = W.Gas()
    R, th = gas.R, gas.theta_vib
    rng = np.random.default_rng(41)
    Ts = [(3000.0, 1000.0, 2000.0), (800.0, 800.0, 800.0), (0, 0, 0)]
    counts = [200_000, 150_000, 0]
    Us = [(400.0, -100.0, 0.0), (0.0, 0.0, 50.0), (0, 0, 0)]
    cs, es, vs = [], [], []
    for (T, Tr, Tv), n, U in zip(Ts, counts, Us):
        if n:
            c, e, v = _maxwellian(rng, n, R, T, Tr, Tv, th, U=U)
            cs.append(c); es.append(e); vs.append(v)
    c, e, v = np.concatenate(cs, 1), np.concatenate(es), np.concatenate(vs)
    n = c.shape[1]
    M = len(counts)
    vol = np.array([1e-6, 2e-6, 1e-6])
    fnum = 1e12
    grid = W.Grid(dim=0, nx=M, ny=1, fnum=fnum, volume=vol, flags=np.zeros(M, np.uint8))
    prob = W.Problem("t", gas, grid, W.BC(), dt=1e-9, seed=1, f32=False)
    parts = dict(n=n, cap=n, x=None, y=None, cx=c[0], cy=c[1], cz=c[2], erot=e, vib=v,
                 cell=np.repeat(np.arange(M, dtype=np.int32), counts),
                 pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.bin()
    sim.enable_sampling()
    for _ in range(3):
        sim.sample_fields()
    f = sampling.field_averages(sim.fields, vol, fnum, gas.m, th, 3)
    for k, ((T, Tr, Tv), N, U) in enumerate(zip(Ts, counts, Us)):
        if not N:
            assert f["n"][k] == 0 and f["T_tr"][k] == 0 and f["T_vib"][k] == 0
            continue
        assert f["n"][k] == pytest.approx(N * fnum / vol[k], rel=1e-12)
        assert np.allclose(f["U"][:, k], U, atol=5 * math.sqrt(R * T / N))
        assert f["T_tr"][k] == pytest.approx(T, rel=0.01)
        assert f["T_rot"][k] == pytest.approx(Tr, rel=0.01)
        assert f["T_vib"][k] == pytest.approx(Tv, rel=0.02)
        assert f["p"][k] == pytest.approx(f["n"][k] * KB * f["T_tr"][k], rel=1e-12)
        # no heat flux in an equilibrium (drifting) Maxwellian
        qs = f["n"][k] * gas.m * (R * T) ** 1.5
        assert np.abs(f["q_tr"][:, k]).max() < 0.02 * qs


def test_flat_wall_fluxes_in_physical_units():
    """Shear rho U sqrt(RT/(2 pi)) and pressure rho RT/2 + rho sqrt(RT RT_w)/2
    of a drifting Maxwellian on a diffuse wall, from the element's sums,
    the molecular mass, fnum and the sampled time."""
    gas = W.Gas()
    R = gas.R
    T, Tw, U = 900.0, 300.0, 600.0
    dt = 1e-6
    L = 40 * math.sqrt(R * T) * dt
    npart = 1_500_000
    rng = np.random.default_rng(42)
    c, erot, vib = _maxwellian(rng, npart, R, T, T, T, gas.theta_vib, U=(U, 0.0, 0.0))
    y = rng.random(npart) * L
    area = 2.0  # cross-section of the channel [m^2]
    fnum = 1e10
    grid = W.Grid(dim=1, nx=1, ny=2, y0=0.0, dy=L / 2, fnum=fnum,
                  volume=np.full(2, L / 2 * area), flags=np.zeros(2, np.uint8))
    bc = W.BC(kind=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_DIFFUSE, W.BC_SPECULAR), Tw=(0, 0, Tw, 0))
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=6, f32=False)
    parts = dict(n=npart, cap=npart, x=None, y=y, cx=c[0], cy=c[1], cz=c[2], erot=erot, vib=vib,
                 cell=np.zeros(npart, np.int32), pid=np.arange(npart, dtype=np.uint32),
                 next_pid=npart)
    sim = oracle.Sim(prob, parts)
    sim.enable_sampling()
    sim.advect(0)
    fl = sampling.surface_fluxes(sim.surf, grid, bc, 0, gas.m, fnum, gas.theta_vib, dt)
    assert fl["area"][0] == pytest.approx(area)
    rho = npart * fnum / (L * area) * gas.m
    hits = fl["hits"][0]
    s = math.sqrt(R * T)
    assert fl["sigma"][0] == pytest.approx(rho * U * s / math.sqrt(2 * math.pi),
                                           rel=5 * 1.6 / math.sqrt(hits))
    want_p = rho * R * T / 2 + rho * math.sqrt(R * T * R * Tw) / 2
    assert fl["p"][0] == pytest.approx(want_p, rel=5 * 0.8 / math.sqrt(hits))
    assert np.all(fl["hits"][1:] == 0)


def test_cylinder_drag_and_coefficients():
    """The free-molecular cylinder of the oracle pins, in physical units:
    the drag per unit span from the summed x momentum equals the integral
    of the incident and re-emitted momentum fluxes; C_f and C_h are the
    shear and heat flux over rho U^2/2 and rho U^3/2."""
    nb = 12
    sim, geo = _cyl_problem(2_000_000, s_ratio=1.5, T=600.0, Tw=300.0, nb=nb, seed=33)
    gas = W.Gas()
    grid, bc = sim.prob.grid, sim.prob.bc
    fl = sampling.surface_fluxes(sim.surf, grid, bc, nb, gas.m, grid.fnum, gas.theta_vib,
                                 geo["dt"])
    assert fl["halves"] == 2
    want = sum(_cyl_expect(k, nb, geo, "px") for k in range(nb))
    drag_sum = gas.m * grid.fnum / geo["dt"] * want
    assert fl["body_force"][0] == pytest.approx(drag_sum, rel=0.02)
    rho = geo["dens"] * grid.fnum * gas.m
    co = sampling.cylinder_coefficients(fl, rho, geo["U"])
    assert co["drag"] == fl["body_force"][0]
    body = fl["kind"] == sampling.BODY
    assert np.allclose(co["C_f"], fl["sigma"][body] / (0.5 * rho * geo["U"] ** 2))
    assert np.allclose(co["C_h"], fl["q"][body] / (0.5 * rho * geo["U"] ** 3))
    assert co["peak_heat_flux"] == fl["q"][body].max()
    assert co["theta_deg"][0] == pytest.approx(180.0 / nb / 2)
    # windward elements carry the largest pressure
    assert np.argmax(co["C_p"]) == 0


def test_surface_elements_of_the_half_body_cylinder():
    """The cylinder workload (half body on the symmetry plane y = 0): the
    element order and areas, one half in the domain, and the mirror half
    added to the force (drag doubled, lift cancelled)."""
    prob = W.cylinder(scale=0.05, f32=True)
    g, bc = prob.grid, prob.bc
    nb = 18
    el = sampling.surface_elements(g, bc, nb)
    assert el["halves"] == 1
    k = el["kind"]
    assert list(np.bincount(k, minlength=5)) == [g.nx, g.nx, g.ny, g.ny, nb]
    assert np.allclose(el["area"][:g.nx], g.dx * bc.depth)
    assert np.allclose(el["area"][2 * g.nx:2 * g.nx + g.ny], g.dy * bc.depth)
    assert np.allclose(el["area"][-nb:], bc.cyl_r * np.pi / nb * bc.depth)
    assert np.allclose(np.degrees(el["coord"][-nb:]), (np.arange(nb) + 0.5) * 10.0)
    # one hit on the first body element, 1 m/s of x momentum and 2 of y
    surf = np.zeros((k.size, sampling.SURF_NQ), np.int64)
    e = 2 * g.nx + 2 * g.ny
    surf[e, sampling.SURF_HITS] = 1
    surf[e, sampling.SURF_PX] = int(sampling.SURF_P_SCALE)
    surf[e, sampling.SURF_PY] = int(2 * sampling.SURF_P_SCALE)
    fl = sampling.surface_fluxes(surf, g, bc, nb, 1.0, 1.0, 3371.0, 1.0)
    assert fl["body_force"][0] == pytest.approx(2.0 / bc.depth)
    assert fl["body_force"][1] == 0.0
