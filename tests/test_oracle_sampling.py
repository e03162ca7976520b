"""Pins of the oracle's sampling (the N_sampling phase of Sec. V.C): the
field sums against the moments and exact integer arithmetic, and the wall
sums against free-molecular closed forms for a flat wall and for the
cylinder (drag, pressure and shear per angular element).  No GPU."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import usp_workloads as W

KB = 1.380649e-23
MN = oracle.MOM_NAMES
SN = oracle.SAMP_NAMES
Q = {k: i for i, k in enumerate(oracle.SURF_NAMES)}


def _binned_sim(counts, rng, integer=False, f32=False):
    """A 0D state (independent cells of the given counts), binned."""
    M = len(counts)
    n = int(sum(counts))
    cell = np.repeat(np.arange(M, dtype=np.int32), counts)
    if integer:
        c = rng.integers(-40, 41, size=(3, n)).astype(np.float64)
        erot = rng.integers(0, 30, size=n).astype(np.float64)
    else:
        c = 300.0 * rng.standard_normal((3, n)) + rng.normal(0, 500, (3, 1))
        erot = rng.exponential(2e5, n)
    vib = rng.integers(0, 6, size=n).astype(np.int32)
    grid = W.Grid(dim=0, nx=M, ny=1, fnum=1.0, volume=np.ones(M), flags=np.zeros(M, np.uint8))
    prob = W.Problem("t", W.Gas(), grid, W.BC(), dt=1e-9, seed=1, f32=f32)
    parts = dict(n=n, cap=n, x=None, y=None, cx=c[0], cy=c[1], cz=c[2], erot=erot, vib=vib,
                 cell=cell, pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.bin()
    return sim, parts


def test_field_sums_exact_on_integers():
    """Integer-valued velocities, energies and levels: every sum is an exact
    integer, equal to exact Python integer arithmetic over each cell."""
    rng = np.random.default_rng(11)
    counts = [0, 1, 2, 7, 5, 0, 3]
    sim, parts = _binned_sim(counts, rng, integer=True)
    sim.enable_sampling()
    sim.sample_fields()
    sim.sample_fields()
    got = sim.fields
    st = sim.state()
    off = np.concatenate([[0], np.cumsum(counts)])
    for c in range(len(counts)):
        cx = [int(v) for v in st["cx"][off[c]:off[c + 1]]]
        cy = [int(v) for v in st["cy"][off[c]:off[c + 1]]]
        cz = [int(v) for v in st["cz"][off[c]:off[c + 1]]]
        er = [int(v) for v in st["erot"][off[c]:off[c + 1]]]
        lv = [int(v) for v in st["vib"][off[c]:off[c + 1]]]
        vs = list(zip(cx, cy, cz))
        want = [len(vs), sum(cx), sum(cy), sum(cz),
                sum(a * a for a in cx), sum(b * b for b in cy), sum(d * d for d in cz),
                sum(a * b for a, b, _ in vs), sum(a * d for a, _, d in vs),
                sum(b * d for _, b, d in vs), sum(er), sum(lv)]
        # (1/2)|c|^2 c is a half-integer multiple: compare twice the sum
        h2 = [sum((a * a + b * b + d * d) * v[k] for (a, b, d), v in zip(vs, vs)) for k in range(3)]
        want += [x / 2 for x in h2]
        want += [sum(v[k] * e for v, e in zip(vs, er)) for k in range(3)]
        want += [sum(v[k] * i for v, i in zip(vs, lv)) for k in range(3)]
        for k, w in enumerate(want):
            assert got[k, c] == 2 * w, (SN[k], c, got[k, c], 2 * w)


def test_field_sums_agree_with_central_moments():
    """The raw sums and the (separately pinned) central moments describe the
    same cell: U = S_c/N, Pi = S_cc/N - U U, <e_rot>, <I>, and the third
    moments q_tr = (1/2)<C^2 C>, <C e_rot>, <C I> from the raw ones."""
    rng = np.random.default_rng(12)
    counts = list(rng.integers(0, 400, 40))
    sim, _ = _binned_sim(counts, rng)
    sim.do_moments()
    mom = sim.moments()
    sim.enable_sampling()
    sim.sample_fields()
    S = sim.fields
    N = S[0]
    assert np.array_equal(N, mom[0])
    ok = N > 0
    U = S[1:4, ok] / N[ok]
    scale_u = np.abs(U).max() + 300.0
    assert np.abs(U - mom[1:4, ok]).max() < 1e-12 * scale_u
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (i, j) in enumerate(pairs):
        P = S[4 + k, ok] / N[ok] - U[i] * U[j]
        assert np.abs(P - mom[MN.index("PXX") + k, ok]).max() < 1e-9 * scale_u ** 2
    er, Ib = S[10, ok] / N[ok], S[11, ok] / N[ok]
    assert np.allclose(er, mom[MN.index("EROT"), ok], rtol=1e-13)
    assert np.allclose(Ib, mom[MN.index("IBAR"), ok], rtol=1e-13, atol=1e-15)
    Pm = np.zeros((3, 3, ok.sum()))
    for k, (i, j) in enumerate(pairs):
        Pm[i, j] = Pm[j, i] = mom[MN.index("PXX") + k, ok]
    hU2 = 0.5 * (U ** 2).sum(0)
    htr = 0.5 * np.trace(Pm)
    for i in range(3):
        raw = S[12 + i, ok] / N[ok]
        central = raw - (hU2 + htr) * U[i] - (Pm[i] * U).sum(0)
        assert np.abs(central - mom[MN.index("QTRX") + i, ok]).max() < 1e-8 * scale_u ** 3
        qr = S[15 + i, ok] / N[ok] - U[i] * er
        assert np.abs(qr - mom[MN.index("QROTX") + i, ok]).max() < 1e-9 * scale_u * er.max()
        qi = S[18 + i, ok] / N[ok] - U[i] * Ib
        assert np.abs(qi - mom[MN.index("QIX") + i, ok]).max() < 1e-9 * scale_u * 6


# --------------------------------------------------------------------------
# wall sums: free-molecular closed forms
# --------------------------------------------------------------------------
def _trunc(a, s):
    """Moments of the incident part of w ~ N(a, s^2), w < 0: E[(-w)+],
    E[w^2; w<0], E[-w^3; w<0] (truncated-normal integrals)."""
    z = a / s
    phi, Phi = stats.norm.pdf(z), stats.norm.cdf(-z)
    m1 = s * phi - a * Phi
    m2 = (a * a + s * s) * Phi - a * s * phi
    m3 = s * (a * a + 2 * s * s) * phi - (a ** 3 + 3 * a * s * s) * Phi
    return m1, m2, m3


def test_truncated_moments_by_quadrature():
    for a, s in ((0.0, 1.0), (-1.7, 0.8), (2.3, 1.5)):
        f = lambda w, k: (-w) ** k * stats.norm.pdf(w, a, s)
        ref = [integrate.quad(f, -np.inf, 0, args=(k,))[0] for k in (1, 2, 3)]
        ref[1] = integrate.quad(lambda w: w * w * stats.norm.pdf(w, a, s), -np.inf, 0)[0]
        assert np.allclose(_trunc(a, s), ref, rtol=1e-9, atol=1e-12)


def _maxwellian(rng, n, R, T, Trot, Tvib, theta, U=(0.0, 0.0, 0.0)):
    s = math.sqrt(R * T)
    c = s * rng.standard_normal((3, n)) + np.asarray(U)[:, None]
    erot = rng.exponential(R * Trot, n)
    q = math.exp(-theta / Tvib)
    vib = rng.geometric(1 - q, n) - 1
    return c, erot, vib.astype(np.int32)


def test_flat_wall_free_molecular_fluxes():
    """A drifting Maxwellian (T, T_rot, T_vib, drift U along x) over a
    diffuse wall at T_w, one flight: per hit, the shear part is U, the
    pressure part sqrt(pi R T/2) + sqrt(pi R T_w/2), the translational
    energy 2R(T - T_w) + U^2/2, the rotational R(T_rot - T_w), the quanta
    <I>(T_vib) - <I>(T_w); the hit count is n dt sqrt(R T/(2 pi))."""
    gas = W.Gas()
    R, th = gas.R, gas.theta_vib
    T, Trot, Tvib, Tw, U = 1000.0, 800.0, 2500.0, 300.0, 500.0
    dt = 1e-6
    L = 40 * math.sqrt(R * T) * dt
    n = 2_000_000
    rng = np.random.default_rng(21)
    c, erot, vib = _maxwellian(rng, n, R, T, Trot, Tvib, th, U=(U, 0.0, 0.0))
    y = rng.random(n) * L
    ny = 4
    grid = W.Grid(dim=1, nx=1, ny=ny, y0=0.0, dy=L / ny, fnum=1.0, volume=np.ones(ny),
                  flags=np.zeros(ny, np.uint8))
    bc = W.BC(kind=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_DIFFUSE, W.BC_SPECULAR), Tw=(0, 0, Tw, 0))
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=5, f32=False)
    parts = dict(n=n, cap=n, x=None, y=y, cx=c[0], cy=c[1], cz=c[2], erot=erot, vib=vib,
                 cell=np.zeros(n, np.int32), pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.enable_sampling()
    sim.advect(0)
    S = sim.surf[0].astype(np.float64)   # the ylo element
    assert np.all(sim.surf[1:] == 0)     # the specular wall is not a surface
    hits = S[Q["HITS"]]
    want_hits = n / L * dt * math.sqrt(R * T / (2 * math.pi))
    assert abs(hits - want_hits) < 5 * math.sqrt(want_hits)
    P, E = oracle.SURF_P_SCALE, oracle.SURF_E_SCALE
    pt = S[Q["PT"]] / P / hits
    pn = S[Q["PN"]] / P / hits
    assert abs(pt - U) < 5 * math.sqrt(R * (T + Tw) / hits)
    want_pn = math.sqrt(math.pi * R * T / 2) + math.sqrt(math.pi * R * Tw / 2)
    assert abs(pn - want_pn) < 5 * math.sqrt(R * (T + Tw) * (2 - math.pi / 2) / hits)
    # y wall: t = +x, n = +y
    assert S[Q["PX"]] == S[Q["PT"]] and S[Q["PY"]] == -S[Q["PN"]]
    assert abs(S[Q["PZ"]] / P / hits) < 5 * math.sqrt(R * (T + Tw) / hits)
    etr = S[Q["ETR"]] / E / hits
    want_etr = 2 * R * (T - Tw) + U * U / 2
    assert etr == pytest.approx(want_etr, rel=0.02)
    erot_w = S[Q["EROT"]] / E / hits
    assert erot_w == pytest.approx(R * (Trot - Tw), rel=0.02)
    mI = lambda Tx: 1.0 / math.expm1(th / Tx)
    assert S[Q["QVIB"]] / hits == pytest.approx(mI(Tvib) - mI(Tw), rel=0.03)


def _cyl_problem(n, s_ratio, T, Tw, nb, seed):
    gas = W.Gas()
    R = gas.R
    sig = math.sqrt(R * T)
    U = s_ratio * math.sqrt(2 * R * T)
    r, L = 0.05, 0.4
    dt = 0.05 / (U + 7 * sig)
    rng = np.random.default_rng(seed)
    # uniform outside the cylinder (rejection), drifting Maxwellian
    m = int(n / (1 - math.pi * r * r / (L * L))) + 1000
    x, y = rng.random(m) * L, rng.random(m) * L
    keep = np.hypot(x - L / 2, y - L / 2) >= r
    x, y = x[keep][:n], y[keep][:n]
    c, erot, vib = _maxwellian(rng, n, R, T, T, T, gas.theta_vib, U=(U, 0.0, 0.0))
    nx = 8
    grid = W.Grid(dim=2, nx=nx, ny=nx, x0=0.0, y0=0.0, dx=L / nx, dy=L / nx, fnum=1.0,
                  volume=np.full(nx * nx, (L / nx) ** 2), flags=np.zeros(nx * nx, np.uint8))
    bc = W.BC(kind=(W.BC_PERIODIC,) * 4, cyl=1, cyl_xc=L / 2, cyl_yc=L / 2, cyl_r=r, cyl_Tw=Tw)
    prob = W.Problem("t", gas, grid, bc, dt=dt, seed=seed, f32=False)
    parts = dict(n=n, cap=n, x=x, y=y, cx=c[0], cy=c[1], cz=c[2], erot=erot, vib=vib,
                 cell=np.zeros(n, np.int32), pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.enable_sampling(nb)
    sim.advect(0)
    dens = n / (L * L - math.pi * r * r)   # particles per unit area (unit depth)
    return sim, dict(R=R, sig=sig, U=U, r=r, dt=dt, dens=dens, Tw=Tw, nx=nx)


def _cyl_expect(k, nb, geo, what):
    """Expected sum over the hits of angular element k (both halves):
    dt * dens * r * integral over the element of the per-area flux, where a
    surface point with outward normal (cos phi, sin phi) sees the normal
    drift a = U cos phi."""
    R, sig, U, r, Tw = geo["R"], geo["sig"], geo["U"], geo["r"], geo["Tw"]
    vr = math.sqrt(math.pi * R * Tw / 2)

    def flux(phi):
        a = U * math.cos(phi)
        m1, m2, _ = _trunc(a, sig)
        if what == "hits":
            return m1
        if what == "pn":
            return m2 + m1 * vr
        if what == "pt":
            return m1 * U * abs(math.sin(phi))
        if what == "px":
            # -n_x (pressure part) + tangential drift U sin^2 phi (shear part)
            return -math.cos(phi) * (m2 + m1 * vr) + m1 * U * math.sin(phi) ** 2
        raise ValueError(what)

    lo, hi = k * math.pi / nb, (k + 1) * math.pi / nb
    # Theta = pi - phi on the upper half, phi - pi on the lower half
    up = integrate.quad(lambda t: flux(math.pi - t), lo, hi)[0]
    dn = integrate.quad(lambda t: flux(math.pi + t), lo, hi)[0]
    return geo["dt"] * geo["dens"] * r * (up + dn)


def test_cylinder_free_molecular_pressure_shear_and_drag():
    """Free-molecular drifting Maxwellian around a diffuse cylinder (one
    flight, convex body: every element sees the undisturbed gas): per angular
    element the hit count, the pressure and shear sums, and the total x
    momentum (the drag) follow from the truncated-normal integrals of the
    incident flux and the diffuse re-emission."""
    nb = 12
    sim, geo = _cyl_problem(3_000_000, s_ratio=1.5, T=600.0, Tw=300.0, nb=nb, seed=31)
    base = 4 * geo["nx"]
    S = sim.surf[base:base + nb].astype(np.float64)
    assert np.all(sim.surf[:base] == 0)
    P = oracle.SURF_P_SCALE
    hits = S[:, Q["HITS"]]
    for k in range(nb):
        h = _cyl_expect(k, nb, geo, "hits")
        assert abs(hits[k] - h) < 5 * math.sqrt(h) + 1, (k, hits[k], h)
        pn = _cyl_expect(k, nb, geo, "pn")
        assert S[k, Q["PN"]] / P == pytest.approx(pn, rel=5 * 1.2 / math.sqrt(h) + 0.005), k
        pt = _cyl_expect(k, nb, geo, "pt")
        tol = 5 * math.sqrt(2 * geo["R"] * 600.0 * h)
        assert abs(S[k, Q["PT"]] / P - pt) < tol + 0.005 * abs(pt), k
    drag = S[:, Q["PX"]].sum() / P
    want = sum(_cyl_expect(k, nb, geo, "px") for k in range(nb))
    assert drag == pytest.approx(want, rel=0.02)
    # nothing drives a net lift across the two halves
    assert abs(S[:, Q["PY"]].sum() / P) < 0.03 * abs(want)


def test_cylinder_equilibrium_is_uniform_and_adiabatic():
    """Gas at rest at the wall temperature: every angular element receives
    the same number of hits (equal areas), the pressure sum per hit is
    sqrt(2 pi R T), shear and net translational energy vanish."""
    nb = 9
    sim, geo = _cyl_problem(2_000_000, s_ratio=0.0, T=500.0, Tw=500.0, nb=nb, seed=32)
    base = 4 * geo["nx"]
    S = sim.surf[base:base + nb].astype(np.float64)
    hits = S[:, Q["HITS"]]
    chi2 = ((hits - hits.mean()) ** 2 / hits.mean()).sum()
    assert chi2 < stats.chi2.ppf(0.9999, nb - 1)
    P, E = oracle.SURF_P_SCALE, oracle.SURF_E_SCALE
    R, T = geo["R"], 500.0
    pn = S[:, Q["PN"]].sum() / P / hits.sum()
    assert pn == pytest.approx(math.sqrt(2 * math.pi * R * T), rel=5 * 0.3 / math.sqrt(hits.sum()) + 1e-3)
    assert abs(S[:, Q["PT"]].sum() / P / hits.sum()) < 5 * math.sqrt(2 * R * T / hits.sum())
    assert abs(S[:, Q["ETR"]].sum() / E / hits.sum()) < 5 * 2.5 * R * T / math.sqrt(hits.sum())
