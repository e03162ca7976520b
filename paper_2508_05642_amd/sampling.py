"""Time averages and surface coefficients from the sampled sums.

The device side accumulates two kinds of sums during the sampling phase of
a run (the N_sampling steps of Sec. V.C):

- field sums (usp_sample_fields): per cell, over the sampled steps, the
  raw particle sums N, sum c, sum c_i c_j, sum eps_rot, sum I,
  sum |c|^2 c / 2, sum c eps_rot, sum c I;
- surface sums (usp_bc.surf): per surface element, over every diffuse
  re-emission, the momentum and energy per unit mass the particles gave
  the wall, in fixed point.

This module turns them into the quantities the paper reports: number
density, velocity, the three temperatures, pressure and heat fluxes per
cell, and pressure, shear and heat flux per surface element with the
coefficients C_f = sigma / (rho U^2 / 2) and C_h = q / (rho U^3 / 2), the
total drag and the peak heat flux of the cylinder (Sec. V.C).  Host-side
numpy post-processing only; no part of the step runs here.
"""
from __future__ import annotations

import math

import numpy as np

KB = 1.380649e-23
NSAMP, SURF_NQ = 21, 9
SURF_HITS, SURF_PX, SURF_PY, SURF_PZ, SURF_PN, SURF_PT, SURF_ETR, SURF_EROT, SURF_QVIB = range(9)
SURF_P_SCALE, SURF_E_SCALE = 65536.0, 16.0

# surface element kinds
YLO, YHI, XLO, XHI, BODY = range(5)


def field_averages(sums, volume, fnum, m, theta_vib, nsamples):
    """Time-averaged cell fields from the field sums (shape [21, M]).

    Returns a dict of arrays over cells: n [1/m^3], U [3, M] m/s, T_tr,
    T_rot, T_vib [K], p [Pa], q_tr, q_rot, q_vib [3, M] W/m^2, and Np (mean
    simulated particles per cell).  Averages are ratios of the summed
    particle sums (the usual particle-method time average), so a cell's
    temperature is that of all the particles it held over the sampled steps.
    Empty cells get zeros."""
    S = np.asarray(sums, np.float64).reshape(NSAMP, -1)
    M = S.shape[1]
    R = KB / m
    N = S[0]
    ok = N > 0
    inv = np.where(ok, 1.0 / np.where(ok, N, 1.0), 0.0)
    U = S[1:4] * inv
    raw = S[4:10] * inv
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    P = np.zeros((3, 3, M))
    for k, (i, j) in enumerate(pairs):
        P[i, j] = P[j, i] = raw[k] - U[i] * U[j]
    trP = P[0, 0] + P[1, 1] + P[2, 2]
    erot = S[10] * inv
    Ibar = S[11] * inv
    Np = N / max(nsamples, 1)
    n = Np * fnum / np.asarray(volume, np.float64)
    rho = n * m
    T_tr = trP / (3.0 * R)
    T_rot = erot / R
    T_vib = np.zeros(M)
    pos = Ibar > 0
    T_vib[pos] = theta_vib / np.log1p(1.0 / Ibar[pos])
    hU2 = 0.5 * (U * U).sum(0)
    PU = np.einsum("ijc,jc->ic", P, U)
    q_tr = rho * (S[12:15] * inv - (hU2 + 0.5 * trP) * U - PU)
    q_rot = rho * (S[15:18] * inv - U * erot)
    q_vib = rho * R * theta_vib * (S[18:21] * inv - U * Ibar)
    return dict(n=n, U=U, T_tr=T_tr, T_rot=T_rot, T_vib=T_vib, p=n * KB * T_tr, q_tr=q_tr,
                q_rot=q_rot, q_vib=q_vib, Np=Np)


def surface_elements(grid, bc, nbody):
    """Kind, area [m^2] and a coordinate of every surface element in the
    order of the device sums: ylo and yhi walls by x cell, xlo and xhi walls
    by y cell, then the cylinder by angle Theta from the upstream stagnation
    point (both halves share an element; `halves` of them lie in the
    domain).  The coordinate is the cell centre along the wall, or the
    element's mid angle in radians on the cylinder."""
    nx, ny = grid.nx, grid.ny
    depth = getattr(bc, "depth", 1.0)
    if grid.dim == 1:
        across = float(np.asarray(grid.volume, np.float64)[0]) / grid.dy
        ywall = np.full(nx, across)
    else:
        ywall = np.full(nx, grid.dx * depth)
    xwall = np.full(ny, grid.dy * depth)
    kinds = [np.full(nx, YLO), np.full(nx, YHI), np.full(ny, XLO), np.full(ny, XHI)]
    areas = [ywall, ywall, xwall, xwall]
    xc = grid.x0 + (np.arange(nx) + 0.5) * (grid.dx if grid.dim == 2 else 0.0)
    yc = grid.y0 + (np.arange(ny) + 0.5) * grid.dy
    coord = [xc, xc, yc, yc]
    halves = 0
    if nbody:
        # a half body when the domain ends on the centre line
        lo, hi = grid.y0, grid.y0 + grid.ny * grid.dy
        halves = (1 if hi > bc.cyl_yc else 0) + (1 if lo < bc.cyl_yc else 0)
        dth = math.pi / nbody
        kinds.append(np.full(nbody, BODY))
        areas.append(np.full(nbody, bc.cyl_r * dth * depth * max(halves, 1)))
        coord.append((np.arange(nbody) + 0.5) * dth)
    return dict(kind=np.concatenate(kinds), area=np.concatenate(areas),
                coord=np.concatenate(coord), halves=halves, depth=depth)


def surface_fluxes(surf, grid, bc, nbody, m, fnum, theta_vib, time):
    """Per surface element: number flux [1/(m^2 s)], pressure p [Pa],
    shear sigma [Pa] (along the element's tangent), heat flux q [W/m^2]
    (translational, rotational and vibrational energy given to the wall),
    over the sampled `time` [s] (steps x dt); plus the force on the
    cylinder per unit span [N/m], both halves counted, with the half-body
    mirror image added when only one half is in the domain."""
    S = np.asarray(surf, np.int64).reshape(-1, SURF_NQ).astype(np.float64)
    el = surface_elements(grid, bc, nbody)
    A = el["area"]
    if S.shape[0] != A.size:
        raise ValueError(f"{S.shape[0]} surface elements in the sums, {A.size} expected")
    R = KB / m
    w = m * fnum / (A * time)
    out = dict(el)
    out["hits"] = S[:, SURF_HITS]
    out["number_flux"] = fnum * S[:, SURF_HITS] / (A * time)
    out["p"] = w * S[:, SURF_PN] / SURF_P_SCALE
    out["sigma"] = w * S[:, SURF_PT] / SURF_P_SCALE
    out["q"] = (w * (S[:, SURF_ETR] + S[:, SURF_EROT]) / SURF_E_SCALE
                + w * R * theta_vib * S[:, SURF_QVIB])
    body = el["kind"] == BODY
    F = m * fnum / time * S[body][:, SURF_PX:SURF_PZ + 1].sum(0) / SURF_P_SCALE / el["depth"]
    if el["halves"] == 1:
        # the mirror half: same drag, opposite lift
        F = np.array([2.0 * F[0], 0.0, 2.0 * F[2]])
    out["body_force"] = F
    return out


def cylinder_coefficients(flux, rho_inf, U_inf):
    """C_f, C_h (and C_p = (p - 0)/(rho U^2/2), the wall pressure
    coefficient) along the cylinder against Theta [deg], the total drag per
    unit span [N/m] and the peak heat flux [W/m^2] (Sec. V.C)."""
    body = flux["kind"] == BODY
    qinf = 0.5 * rho_inf * U_inf * U_inf
    return dict(theta_deg=np.degrees(flux["coord"][body]),
                C_f=flux["sigma"][body] / qinf,
                C_h=flux["q"][body] / (qinf * U_inf),
                C_p=flux["p"][body] / qinf,
                drag=float(flux["body_force"][0]),
                peak_heat_flux=float(flux["q"][body].max()) if body.any() else 0.0)
