"""Checkpointed pathwise adjoint of a 1D run (FP64 state, USP-FPM scheme).

Outputs of a run of K steps, for theta = (Z_rot, omega, mu_ref):
  mdot  = m fnum / (area K) * sum over steps of sum_i c_x,i at the start of
          the step (mass flow per unit depth, area = cell volume / dy);
  tau_w = m fnum / (2 area K dt) * sum over the steps of the x momentum the
          particles give the boundaries (the mean shear of the two walls).
The gradient is taken along the path of the run with every discrete
outcome held fixed (see usp_adjoint_step in include/usp.h); horizons
beyond VALID_HORIZON steps are refused by default (see below).

The forward pass runs the K steps with usp_step, sampling the two outputs
on the device, and keeps the particle state every `segment` steps.  The
reverse pass walks the segments backwards: it restores a segment's
checkpoint, re-runs its steps with usp_step_taped (same bits, tape kept per
step) and then reverses them with usp_adjoint_step.  Memory: one
checkpoint per segment plus `segment` tapes.

`PathwiseOutputs` wraps both passes as a torch.autograd.Function of theta.
"""
from __future__ import annotations

import dataclasses

import torch

from . import usp

KB = 1.380649e-23
NOBJ, NPAR = 2, 3
FIELDS = ("y", "cx", "cy", "cz", "erot", "vib", "cell", "pid", "count")


def weights(prob, K):
    g = prob.grid
    area = float(g.volume[0]) / g.dy
    w_m = prob.gas.m * g.fnum / (area * K)
    return w_m, w_m / (2.0 * prob.dt)


# The longest horizon over which the pathwise gradient has been shown to be
# the derivative of the run: on the differentiable channel (Kn 0.05, 100
# cells x 500 particles, FP64) central differences of complete runs at
# theta +- h, with h small enough that no discrete outcome of the run
# changes (1e-8 relative at 32 and 64 steps), agree with it within ~1e-3.
# Beyond that the particle dynamics is chaotic: through the position
# dependence of the reconstruction weights the path derivative grows about
# 30x per 100 steps, while any finite perturbation flips cell switches and
# wall hits, so the gradient says nothing about the run's statistics.
VALID_HORIZON = 64


class PathwiseAdjoint:
    """Forward and reverse passes of K steps of `prob` from `parts`.
    K above VALID_HORIZON is refused unless allow_long is set (e.g. to time
    the passes)."""

    def __init__(self, prob, parts, K, segment=32, device="cuda", allow_long=False):
        if prob.grid.dim != 1 or prob.f32:
            raise ValueError("the pathwise adjoint runs 1D FP64 states")
        if int(K) > VALID_HORIZON and not allow_long:
            raise ValueError(
                f"K = {K} steps is beyond the horizon ({VALID_HORIZON} steps) over which the "
                "pathwise gradient has been checked against central differences of complete "
                "runs: past it the particle dynamics is chaotic (the path derivative grows ~30x "
                "per 100 steps through the position dependence of the reconstruction weights) "
                "and the gradient no longer describes the run's statistics; pass "
                "allow_long=True to run it anyway")
        self.prob, self.K, self.seg = prob, int(K), int(segment)
        self.st = usp.DeviceState(prob, parts, device=device)
        self.rs = usp.DeviceState(prob, parts, device=device)   # re-run state
        dev, cap = self.st.dev, self.st.cap
        L = usp.lib()
        tb = L.usp_tape_bytes(usp.C.byref(self.st.grid), cap)
        ab = L.usp_adjoint_ws_bytes(usp.C.byref(self.st.grid), cap)
        if tb == 0 or ab == 0:
            raise usp.UspError("usp_tape_bytes / usp_adjoint_ws_bytes rejected the grid")
        self.tapes = [torch.zeros(tb, dtype=torch.uint8, device=dev)
                      for _ in range(min(self.seg, self.K))]
        self.aws = torch.zeros(ab, dtype=torch.uint8, device=dev)
        self.lam = [torch.zeros(NOBJ * 5 * cap, dtype=torch.float64, device=dev) for _ in range(2)]
        self.grad = torch.zeros(NOBJ * NPAR, dtype=torch.float64, device=dev)
        self.ckpt = []
        self.w_m, self.w_t = weights(prob, self.K)
        self.step0 = None

    # -- state copies ------------------------------------------------------
    @staticmethod
    def _save(st):
        B = st.bufs[st.cur]
        snap = {k: B[k].clone() for k in FIELDS}
        snap["offsets"] = st.offsets.clone()
        snap["binned"] = st.binned
        return snap

    @staticmethod
    def _restore(st, snap):
        B = st.bufs[st.cur]
        for k in FIELDS:
            B[k].copy_(snap[k])
        st.offsets.copy_(snap["offsets"])
        st.binned = snap["binned"]

    # -- passes ------------------------------------------------------------
    def forward(self, step0=0, stream=None):
        """Run the K steps; returns (mdot, tau_w) as a device tensor."""
        st = self.st
        self.step0 = int(step0)
        st.enable_sampling(0)
        self.ckpt = []
        for k in range(self.K):
            if k % self.seg == 0:
                self.ckpt.append(self._save(st))
            st.step(self.step0 + k, 1, stream)
            st.sample_fields(stream)
        fields = st.fields.view(usp.NSAMP, st.M)
        surf = st.surf.view(-1, usp.SURF_NQ)
        g = self.prob.grid
        walls = surf[: 2 * g.nx, usp.SURF_PX].sum().to(torch.float64) / usp.SURF_P_SCALE
        return torch.stack([self.w_m * fields[1].sum(), self.w_t * walls])

    def backward(self, stream=None):
        """dJ/dtheta (2 x 3, objective-major) along the forward's path."""
        rs = self.rs
        lam_in, lam_out = self.lam
        lam_in.zero_()
        self.grad.zero_()
        cap = rs.cap
        nseg = len(self.ckpt)
        for s in reversed(range(nseg)):
            k0, k1 = s * self.seg, min((s + 1) * self.seg, self.K)
            self._restore(rs, self.ckpt[s])
            for k in range(k0, k1):
                rs.step_taped(self.step0 + k, self.tapes[k - k0], self.aws, stream)
            for k in reversed(range(k0, k1)):
                usp.usp_adjoint_step(rs.grid, rs.gas, rs.bc, self.prob.dt, self.tapes[k - k0], cap,
                                     self.prob.seed, self.step0 + k, lam_in, lam_out, self.w_m,
                                     self.w_t, self.grad, self.aws, stream)
                lam_in, lam_out = lam_out, lam_in
        self.lam_initial = lam_in
        return self.grad.view(NOBJ, NPAR)


def with_theta(prob, theta):
    """The problem with (Z_rot, omega, mu_ref) replaced."""
    z, w, m = (float(v) for v in theta)
    return dataclasses.replace(prob, gas=dataclasses.replace(prob.gas, Z_rot=z, omega=w, mu_ref=m))


class PathwiseOutputs(torch.autograd.Function):
    """(mdot, tau_w) of K steps as a differentiable function of theta =
    (Z_rot, omega, mu_ref) (a CPU or device tensor of 3 doubles)."""

    @staticmethod
    def forward(ctx, theta, prob, parts, step0, K, segment, allow_long=False):
        adj = PathwiseAdjoint(with_theta(prob, theta.detach().cpu().tolist()), parts, K, segment,
                              allow_long=allow_long)
        J = adj.forward(step0)
        ctx.adj = adj
        return J.to(theta.device)

    @staticmethod
    def backward(ctx, gJ):
        G = ctx.adj.backward().to(gJ.device)
        return gJ.to(torch.float64) @ G, None, None, None, None, None, None
