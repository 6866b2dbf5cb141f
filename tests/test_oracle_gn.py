"""Pins of the FP64 adjoint Gauss-Newton oracle (oracle/gn.py, Sec. 6.1-6.2)
on a 90-tet box, against what does not use the oracle's own derivative code:
the equilibrium condition of Eq. g, central differences of g and of the
equilibrium itself (each re-solved from scratch), the dense Gauss-Newton
matrix of Eq. gn built from those sensitivities, and the large-damping limit
of the Levenberg-Marquardt step."""

import numpy as np
import pytest

import oracle
import synth
from oracle import gn


@pytest.fixture(scope="module")
def case():
    p = synth.make_box_problem(seed=12, nx=3, ny=3, nz=2, n_subdomains=2, name="box_tiny")
    sim = oracle.OracleSim.from_problem(p)
    x0, v0 = p.initial_state()
    xs, y, _ = gn.equilibrium(sim, x0, v0)
    rng = np.random.default_rng(4)
    xt = xs + 2e-4 * rng.standard_normal(xs.shape)
    xt[sim.fixed] = p.X[sim.fixed]
    return p, sim, xs, y, xt


def _sim_with(p, gs):
    return oracle.OracleSim(p.X, p.tets, gs, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)


def _equilibrium_at(p, gs):
    x0, v0 = p.initial_state()
    return gn.equilibrium(_sim_with(p, gs), x0, v0)[0]


def test_equilibrium_is_stationary(case):
    p, sim, xs, y, _ = case
    g = gn.residual(sim, xs, y)
    inertia = np.abs(sim.mass[:, None] * (xs - y) / sim.dt ** 2).max()
    assert np.abs(g).max() <= 1e-9 * inertia


def test_dg_dx_against_central_differences(case):
    p, sim, xs, y, _ = case
    A = gn.dg_dx(sim, xs)
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.standard_normal(xs.shape)
        v[sim.fixed] = 0.0
        h = 1e-7
        fd = (gn.residual(sim, xs + h * v, y) - gn.residual(sim, xs - h * v, y)) / (2 * h)
        av = (A @ v[sim.free].ravel()).reshape(-1, 3)
        assert np.abs(fd - av).max() <= 1e-7 * np.abs(av).max()
    # symmetric (the Hessian of the step energy) up to the differences' noise
    assert abs(A - A.T).max() <= 1e-9 * abs(A).max()


def test_dg_dgamma_against_central_differences(case):
    p, sim, xs, y, _ = case
    B = gn.dg_dgamma_s(sim, xs)
    for e in (0, 41, 89):
        h = 1e-4 * p.gamma_s[e]
        gp, gm = p.gamma_s.copy(), p.gamma_s.copy()
        gp[e] += h
        gm[e] -= h
        fd = (gn.residual(_sim_with(p, gp), xs, y) - gn.residual(_sim_with(p, gm), xs, y)) / (2 * h)
        col = B[:, e].toarray().ravel()
        assert np.abs(fd.ravel() - col).max() <= 1e-8 * np.abs(col).max(), e


def test_gradient_and_sensitivity_against_re_solved_equilibria(case):
    """d eps / d gamma_e and the column J[:, e] = d x* / d gamma_e from
    central differences of x*(gamma), each x* solved again from rest."""
    p, sim, xs, _, xt = case
    _, grad, J = gn.gn_direction_dense(sim, xs, xt, 1e-8)
    for e in (3, 50, 77):
        h = 1e-4 * p.gamma_s[e]
        gp, gm = p.gamma_s.copy(), p.gamma_s.copy()
        gp[e] += h
        gm[e] -= h
        xp, xm = _equilibrium_at(p, gp), _equilibrium_at(p, gm)
        dx = ((xp - xm) / (2 * h))[sim.free].ravel()
        assert np.abs(dx - J[:, e]).max() <= 1e-5 * np.abs(J[:, e]).max(), e
        fd = (gn.loss(sim, xp, xt) - gn.loss(sim, xm, xt)) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-5 * np.abs(grad).max(), e


def _gn_norm(sim, xs, xt):
    _, _, J = gn.gn_direction_dense(sim, xs, xt, 1.0)
    return np.linalg.norm(J.T @ J, 2)


def test_agn_saddle_system_equals_dense_gauss_newton(case):
    p, sim, xs, _, xt = case
    pn = _gn_norm(sim, xs, xt)
    for kappa in (1e-4 * pn, 1e-2 * pn, 10 * pn):
        d_dense, grad, _ = gn.gn_direction_dense(sim, xs, xt, kappa)
        d_agn, grad2 = gn.gn_direction_agn(sim, xs, xt, kappa)
        assert np.array_equal(grad, grad2)
        assert np.abs(d_agn - d_dense).max() <= 1e-8 * np.abs(d_dense).max(), kappa
        assert d_dense @ grad < 0                          # a descent direction


def test_large_damping_is_scaled_gradient_descent(case):
    """(P + kappa I) d = -grad with kappa far above |P|: d -> -grad / kappa."""
    p, sim, xs, _, xt = case
    kappa = 1e6 * _gn_norm(sim, xs, xt)
    d, grad = gn.gn_direction_agn(sim, xs, xt, kappa)
    assert np.abs(d * kappa + grad).max() <= 1e-5 * np.abs(grad).max()


def test_gauss_newton_step_reduces_the_loss(case):
    """With a target made by another stiffness field (about 5 % apart), the
    lightly damped GN step (kappa = 1e-4 |P|) is a good step: the loss at
    gamma + d is far below the loss at gamma, and far below what a gradient
    step of the same length reaches."""
    p, sim, xs, _, _ = case
    rng = np.random.default_rng(8)
    gs_true = p.gamma_s * np.exp(0.05 * rng.standard_normal(p.nt))
    xt = _equilibrium_at(p, gs_true)
    kappa = 1e-4 * _gn_norm(sim, xs, xt)
    d, grad, _ = gn.gn_direction_dense(sim, xs, xt, kappa)
    l0 = gn.loss(sim, xs, xt)
    l1 = gn.loss(sim, _equilibrium_at(p, p.gamma_s + d), xt)
    l_gd = gn.loss(sim, _equilibrium_at(p, p.gamma_s - grad * (np.linalg.norm(d) / np.linalg.norm(grad))), xt)
    assert l1 < 0.01 * l0 and l1 < 0.1 * l_gd, (l0, l1, l_gd)
