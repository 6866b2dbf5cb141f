"""FP64 discrete adjoint of a PD trajectory with respect to the per-element
stiffness gamma_s.  Test infrastructure only: the product never imports it.

The forward map is the PD iteration of Sec. 7.1 exactly as `oracle.pd`
runs it, per frame n:

    y = x_n + dt v_n + dt^2 g,   x^(0) = y,
    x^(k+1) = L^{-1} b(x^(k)),   b(x) = M y / dt^2 + sum_e G_e^T P_e(F_e(x)) - L_fp x_p,
    x_{n+1} = x^(K),             v_{n+1} = (x_{n+1} - x_n) / dt,

with P_e(F) = V_e (gs_e R(F) + gv_e V(F)) and L = M/dt^2 + sum_e V_e (gs_e + gv_e)
G_e^T G_e (both depend on gs).  Reversing one iteration with lambda =
L^{-1} xbar^(k+1) (L is symmetric):

    gsbar_e += V_e <G_e lambda, R_e(x^(k)) - F_e(x^(k+1))>   (b and L both move)
    xbar^(k) = sum_e G_e^T J_P(F_e(x^(k))) [G_e lambda]     (J_P is symmetric)
    ybar    += M lambda / dt^2

then x^(0) = y, the predictor and the BDF1 velocity are reversed.  The
Jacobian-vector product of P is a central finite difference of P itself
(per element, step 1e-6 in the direction's norm), not an analytic formula.
"""

from __future__ import annotations

import numpy as np

from .pd import OracleSim, deformation_gradient, proj_sl3, scatter_corners, signed_svd


def projections(F, w_s, w_v):
    """(P, R) for deformation gradients F (nt, 3, 3): P = w_s R + w_v V."""
    U, S, W = signed_svd(F)
    s, _ = proj_sl3(S)
    Wt = np.swapaxes(W, 1, 2)
    R = U @ Wt
    Vp = (U * s[:, None, :]) @ Wt
    return w_s[:, None, None] * R + w_v[:, None, None] * Vp, R


def jvp_P(F, D, w_s, w_v, h=1e-6):
    """d/dt P(F + t D) at t = 0 by a central difference with |t D| = h per element."""
    nD = np.sqrt((D * D).sum(axis=(1, 2)))
    t = np.where(nD > 0, h / np.maximum(nD, 1e-300), 0.0)[:, None, None]
    Pp, _ = projections(F + t * D, w_s, w_v)
    Pm, _ = projections(F - t * D, w_s, w_v)
    out = (Pp - Pm) / np.where(t > 0, 2.0 * t, 1.0)
    out[nD == 0] = 0.0
    return out


class OracleTrajectory:
    """A trajectory of `frames` PD steps from (x0, v0) and its adjoint."""

    def __init__(self, sim: OracleSim):
        self.sim = sim

    def forward(self, x0, v0, frames):
        """Runs the frames, keeping every iterate; returns x_N."""
        s = self.sim
        x, v = np.array(x0, dtype=np.float64), np.array(v0, dtype=np.float64)
        self.records = []
        for _ in range(frames):
            y = s.predictor(x, v)
            its = [y.copy()]
            xk = y.copy()
            for _ in range(s.pd_iters):
                F = deformation_gradient(xk, s.tets, s.grads)
                P, _ = projections(F, s.w_s, s.w_v)
                b = s.rhs(y, P)
                xk = xk.copy()
                xk[s.free] = s._solve(b)
                its.append(xk)
            self.records.append((x, its))
            v = (xk - x) / s.dt
            v[s.fixed] = 0.0
            x = xk
        return x

    def backward(self, xbar_N, vbar_N=None):
        """Gradient of a loss with dL/dx_N = xbar_N (and dL/dv_N = vbar_N) with
        respect to gamma_s, through every recorded frame."""
        s = self.sim
        dt = s.dt
        xbar = np.array(xbar_N, dtype=np.float64)
        vbar = np.zeros_like(xbar) if vbar_N is None else np.array(vbar_N, dtype=np.float64)
        xbar[s.fixed] = 0.0
        vbar[s.fixed] = 0.0
        gbar = np.zeros(s.tets.shape[0])
        for x_n, its in reversed(self.records):
            xk_bar = xbar + vbar / dt                      # x_{n+1} = x^(K) feeds x and v
            xn_bar = -vbar / dt
            ybar = np.zeros_like(xbar)
            for k in range(s.pd_iters - 1, -1, -1):
                lam = np.zeros_like(xbar)
                lam[s.free] = s._solve(xk_bar[s.free])
                Gl = deformation_gradient(lam, s.tets, s.grads)
                Fk = deformation_gradient(its[k], s.tets, s.grads)
                Fk1 = deformation_gradient(its[k + 1], s.tets, s.grads)
                _, Rk = projections(Fk, s.w_s, s.w_v)
                gbar += s.V * (Gl * (Rk - Fk1)).sum(axis=(1, 2))
                dP = jvp_P(Fk, Gl, s.w_s, s.w_v)
                xk_bar = scatter_corners(s.nv, s.tets, np.einsum("eij,eaj->eai", dP, s.grads))
                xk_bar[s.fixed] = 0.0
                ybar += s.mass[:, None] * lam / (dt * dt)
            ybar += xk_bar                                  # x^(0) = y
            ybar[s.fixed] = 0.0
            xbar = xn_bar + ybar
            vbar = dt * ybar
            xbar[s.fixed] = 0.0
            vbar[s.fixed] = 0.0
        return gbar


def loss_and_grad(p, gamma_s, x_target, frames):
    """Loss 1/2 ||x_N - x_target||^2 over the free vertices of problem p run
    with stiffness gamma_s from rest, and its gradient with respect to gamma_s."""
    sim = OracleSim(p.X, p.tets, gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    tr = OracleTrajectory(sim)
    x0, v0 = p.initial_state()
    xN = tr.forward(x0, v0, frames)
    d = xN - x_target
    d[sim.fixed] = 0.0
    return 0.5 * float((d * d).sum()), tr.backward(d)


def loss_only(p, gamma_s, x_target, frames):
    sim = OracleSim(p.X, p.tets, gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    x, v = p.initial_state()
    x, v = sim.run(x, v, frames)
    d = x - x_target
    d[sim.fixed] = 0.0
    return 0.5 * float((d * d).sum())
