"""Brute-force pins of the oracle's binning, moments and reconstruction."""
import numpy as np
import pytest

import oracle
import usp_workloads as W


def _grid2d(nx=7, ny=5, dx=0.3, dy=0.2, x0=-0.4, y0=0.1):
    M = nx * ny
    return W.Grid(dim=2, nx=nx, ny=ny, x0=x0, y0=y0, dx=dx, dy=dy, fnum=1.0,
                  volume=np.full(M, dx * dy), flags=np.zeros(M, np.uint8))


def _prob(grid, f32):
    return W.Problem("t", W.Gas(), grid, W.BC(), dt=1e-9, seed=5, f32=f32)


@pytest.mark.parametrize("f32", [False, True])
def test_bin_is_stable_counting_sort(f32):
    """Cell index = number of interior edges at or below the position; the
    order inside a cell is the input order (np.argsort, kind='stable')."""
    grid = _grid2d()
    prob = _prob(grid, f32)
    rng = np.random.default_rng(1)
    n = 3000
    ft = np.float32 if f32 else np.float64
    x = (grid.x0 + rng.random(n) * grid.nx * grid.dx).astype(ft)
    y = (grid.y0 + rng.random(n) * grid.ny * grid.dy).astype(ft)
    # put a few particles exactly on interior edges (stored precision)
    ex = (grid.x0 + np.arange(grid.nx + 1) * grid.dx).astype(ft)
    ey = (grid.y0 + np.arange(grid.ny + 1) * grid.dy).astype(ft)
    x[:50] = ex[rng.integers(0, grid.nx, 50)]
    y[50:100] = ey[rng.integers(0, grid.ny, 50)]
    cell = np.zeros(n, np.int32)
    cell[100:130] = -1   # already removed
    parts = dict(n=n, cap=n, x=x, y=y, cx=rng.standard_normal(n), cy=rng.standard_normal(n),
                 cz=rng.standard_normal(n), erot=rng.random(n), vib=rng.integers(0, 4, n).astype(np.int32),
                 cell=cell, pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.bin()
    st = sim.state()
    # brute force: count edges
    ix = np.array([np.sum(ex[1:grid.nx] <= v) for v in x.astype(np.float64)])
    iy = np.array([np.sum(ey[1:grid.ny] <= v) for v in y.astype(np.float64)])
    key = (iy * grid.nx + ix).astype(np.int64)
    key[cell < 0] = -1
    keep = np.nonzero(key >= 0)[0]
    order = keep[np.argsort(key[keep], kind="stable")]
    assert st["n"] == len(order)
    assert np.array_equal(st["pid"], order.astype(np.uint32))
    assert np.array_equal(st["cell"], key[order])
    counts = np.bincount(key[keep], minlength=grid.ncells)
    assert np.array_equal(sim.offsets, np.concatenate([[0], np.cumsum(counts)]))


def test_moments_exact_on_integer_velocities():
    """With small integer velocities every moment is an exact rational; the
    oracle's FP64 two-pass sums reproduce the brute-force values."""
    grid = W.Grid(dim=0, nx=4, ny=1, fnum=1.0, volume=np.ones(4), flags=np.zeros(4, np.uint8))
    prob = _prob(grid, False)
    rng = np.random.default_rng(2)
    counts = [1, 8, 64, 0]
    cell = np.repeat(np.arange(4), counts).astype(np.int32)
    n = len(cell)
    v = rng.integers(-4, 5, (3, n)).astype(np.float64)
    er = rng.integers(0, 9, n).astype(np.float64)
    vib = rng.integers(0, 5, n).astype(np.int32)
    parts = dict(n=n, cap=n, x=None, y=None, cx=v[0], cy=v[1], cz=v[2], erot=er, vib=vib,
                 cell=cell, pid=np.arange(n, dtype=np.uint32), next_pid=n)
    sim = oracle.Sim(prob, parts)
    sim.bin()
    sim.do_moments()
    mom = sim.moments()
    o = 0
    for c, N in enumerate(counts):
        sl = slice(o, o + N)
        o += N
        if N == 0:
            assert np.all(mom[:, c] == 0)
            continue
        U = v[:, sl].mean(axis=1)
        C = v[:, sl] - U[:, None]
        want = dict(N=N, UX=U[0], UY=U[1], UZ=U[2],
                    PXX=(C[0] * C[0]).mean(), PYY=(C[1] * C[1]).mean(), PZZ=(C[2] * C[2]).mean(),
                    PXY=(C[0] * C[1]).mean(), PXZ=(C[0] * C[2]).mean(), PYZ=(C[1] * C[2]).mean(),
                    EROT=er[sl].mean(), IBAR=vib[sl].mean(),
                    QTRX=0.5 * ((C * C).sum(0) * C[0]).mean(), QROTX=(C[0] * er[sl]).mean(),
                    QIZ=(C[2] * vib[sl]).mean())
        for k, w in want.items():
            got = mom[oracle.MOM_NAMES.index(k), c]
            assert abs(got - w) <= 1e-13 * max(1.0, abs(w)), (c, k, got, w)


def _cs_fields(sim):
    return sim.cs.reshape(oracle.NCS, sim.M)


def test_reconstruction_exact_on_bilinear_fields():
    """Interior particles see exactly phi = a + b x + c y + d x y when the
    cell values are that field at the cell centres (Sec. III.B); linear
    fields are reproduced exactly everywhere, boundary cells included."""
    grid = _grid2d(nx=6, ny=5)
    prob = _prob(grid, False)
    sim = oracle.Sim(prob, dict(n=0, cap=1, x=np.zeros(1), y=np.zeros(1), cx=np.zeros(1),
                                cy=np.zeros(1), cz=np.zeros(1), erot=np.zeros(1),
                                vib=np.zeros(1, np.int32), cell=np.zeros(1, np.int32),
                                pid=np.zeros(1, np.uint32), next_pid=0))
    cs = _cs_fields(sim)
    i, j = np.meshgrid(np.arange(grid.nx), np.arange(grid.ny))
    xc = (grid.x0 + (i + 0.5) * grid.dx).ravel()
    yc = (grid.y0 + (j + 0.5) * grid.dy).ravel()
    bil = lambda x, y: 1.5 - 2.0 * x + 3.0 * y + 4.0 * x * y
    lin = lambda x, y: -0.7 + 0.25 * x - 1.5 * y
    cs[oracle.CS_NAMES.index("NBR_OK")] = 1.0
    cs[oracle.CS_NAMES.index("TTR")] = bil(xc, yc)
    cs[oracle.CS_NAMES.index("TROT")] = lin(xc, yc)
    rng = np.random.default_rng(4)
    for c in range(grid.ncells):
        ci, cj = c % grid.nx, c // grid.nx
        for _ in range(10):
            x = grid.x0 + (ci + rng.random()) * grid.dx
            y = grid.y0 + (cj + rng.random()) * grid.dy
            got_l = sim.interp("TROT", c, x, y)
            assert abs(got_l - lin(x, y)) < 1e-12
            # bilinear is exact where the whole quadrant stencil exists
            sx = 1 if x >= xc[c] else -1
            sy = 1 if y >= yc[c] else -1
            if 0 <= ci + sx < grid.nx and 0 <= cj + sy < grid.ny:
                assert abs(sim.interp("TTR", c, x, y) - bil(x, y)) < 1e-12
    # mark one cell unusable: linear fields are still exact around it
    cs[oracle.CS_NAMES.index("NBR_OK"), 2 * grid.nx + 3] = 0.0
    for c in (2 * grid.nx + 2, 2 * grid.nx + 4, 1 * grid.nx + 3, 3 * grid.nx + 3):
        ci, cj = c % grid.nx, c // grid.nx
        for _ in range(10):
            x = grid.x0 + (ci + rng.random()) * grid.dx
            y = grid.y0 + (cj + rng.random()) * grid.dy
            assert abs(sim.interp("TROT", c, x, y) - lin(x, y)) < 1e-12


def test_reconstruction_1d_and_isolated():
    grid = W.Grid(dim=1, nx=1, ny=4, y0=0.0, dy=1.0, fnum=1.0, volume=np.ones(4),
                  flags=np.zeros(4, np.uint8))
    prob = _prob(grid, False)
    sim = oracle.Sim(prob, dict(n=0, cap=1, x=None, y=np.zeros(1), cx=np.zeros(1),
                                cy=np.zeros(1), cz=np.zeros(1), erot=np.zeros(1),
                                vib=np.zeros(1, np.int32), cell=np.zeros(1, np.int32),
                                pid=np.zeros(1, np.uint32), next_pid=0))
    cs = _cs_fields(sim)
    k = oracle.CS_NAMES.index("TTR")
    cs[k] = [1.0, 3.0, 4.0, 10.0]
    cs[oracle.CS_NAMES.index("NBR_OK")] = 1.0
    assert sim.interp("TTR", 1, 0, 1.75) == pytest.approx(3.0 + 0.25 * 1.0)
    assert sim.interp("TTR", 1, 0, 1.25) == pytest.approx(3.0 - 0.25 * 2.0)
    # wall side: the quadrant toward y=0 has no neighbour beyond cell 0 -> opposite
    assert sim.interp("TTR", 0, 0, 0.25) == pytest.approx(1.0 - 0.25 * 2.0)
    cs[oracle.CS_NAMES.index("NBR_OK")] = [1, 0, 1, 0]
    # cell 2 upper quadrant: neighbour 3 unusable -> use 1 (unusable too) -> no slope
    assert sim.interp("TTR", 2, 0, 2.75) == pytest.approx(4.0)
