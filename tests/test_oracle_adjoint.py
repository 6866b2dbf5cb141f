"""Pins of the FP64 oracle adjoint (oracle/adjoint.py): its gradient against
central finite differences of the trajectory loss, the symmetry of the
projection Jacobian it reverses through, and the closed-form derivative of the
polar rotation at a diagonal deformation gradient."""

import numpy as np
import pytest

import oracle
import synth
from oracle.adjoint import jvp_P, loss_and_grad, loss_only, projections


def _target(p, frames, seed=0):
    rng = np.random.default_rng(seed)
    gs_hidden = p.gamma_s * np.exp(0.3 * rng.standard_normal(p.nt))
    sim = oracle.OracleSim(p.X, p.tets, gs_hidden, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    x0, v0 = p.initial_state()
    xt, _ = sim.run(x0, v0, frames)
    return xt


def test_adjoint_matches_central_differences():
    p = synth.problem_by_name("box")
    frames = 3
    xt = _target(p, frames)
    _, g = loss_and_grad(p, p.gamma_s, xt, frames)
    rng = np.random.default_rng(1)
    els = rng.choice(p.nt, 6, replace=False)
    fd = []
    for e in els:
        h = 1e-4 * p.gamma_s[e]        # relative step: the loss is smooth in log gamma
        gp = p.gamma_s.copy()
        gp[e] += h
        gm = p.gamma_s.copy()
        gm[e] -= h
        fd.append((loss_only(p, gp, xt, frames) - loss_only(p, gm, xt, frames)) / (2 * h))
    fd = np.array(fd)
    err = np.abs(g[els] - fd).max() / np.abs(fd).max()
    assert err < 1e-4, (g[els], fd)


def test_projection_jacobian_is_symmetric():
    rng = np.random.default_rng(2)
    n = 64
    Q, _ = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    Q *= np.sign(np.linalg.det(Q))[:, None, None]
    S = np.eye(3) + 0.05 * rng.standard_normal((n, 3, 3))
    F = Q @ (0.5 * (S + np.swapaxes(S, 1, 2)))
    ws = rng.uniform(1.0, 2.0, n)
    wv = rng.uniform(0.1, 1.0, n)
    A = rng.standard_normal((n, 3, 3))
    B = rng.standard_normal((n, 3, 3))
    lhs = (A * jvp_P(F, B, ws, wv)).sum(axis=(1, 2))
    rhs = (B * jvp_P(F, A, ws, wv)).sum(axis=(1, 2))
    assert np.abs(lhs - rhs).max() < 1e-7 * np.abs(lhs).max()


def test_rotation_derivative_closed_form():
    # F = diag(sigma): R = I, and dR = Omega with Omega_ij = (D_ij - D_ji) / (sigma_i + sigma_j)
    rng = np.random.default_rng(3)
    n = 16
    sig = np.sort(rng.uniform(0.7, 1.3, (n, 3)), axis=1)[:, ::-1]
    F = np.zeros((n, 3, 3))
    F[:, [0, 1, 2], [0, 1, 2]] = sig
    D = rng.standard_normal((n, 3, 3))
    dR = jvp_P(F, D, np.ones(n), np.zeros(n))
    ref = (D - np.swapaxes(D, 1, 2)) / (sig[:, :, None] + sig[:, None, :])
    assert np.abs(dR - ref).max() < 1e-8
    _, R = projections(F, np.ones(n), np.zeros(n))
    assert np.abs(R - np.eye(3)).max() < 1e-14
