"""Pins of the inexact CMS oracle (oracle/cms.py, Sec. 7.2) on small meshes,
against facts that do not use its own solve: the reduced matrix of Eq.
global_subspace formed explicitly, the exact sparse LU solve, the energy-norm
monotonicity of mode truncation, and Jacobi's fixed point."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from oracle.cms import CMSSolver, chebyshev_weights, jacobi_spectral_radius
from oracle.dd import bisect_elements


@pytest.fixture(scope="module")
def box():
    p = synth.problem_by_name("box")
    sim = oracle.OracleSim.from_problem(p)
    part = bisect_elements(sim.tets, p.n_subdomains)
    rhs = np.random.default_rng(3).standard_normal((sim.free.size, 3))
    return p, sim, part, rhs


def test_all_modes_is_the_exact_solve(box):
    """With every interior eigenmode kept the subspace is the whole space and
    the reduced solve is the global solve (the survey's identity)."""
    p, sim, part, rhs = box
    n_max = max(I.size for I in CMSSolver(sim.L_ff, sim.free, sim.tets, part, 1).interiors)
    cms = CMSSolver(sim.L_ff, sim.free, sim.tets, part, n_modes=n_max)
    x = cms.solve(rhs)
    xe = sim._solve(rhs)
    assert np.abs(x - xe).max() <= 1e-10 * np.abs(xe).max()


def test_reduced_matrix_is_block_diagonal(box):
    """U^T K U for the basis of Eq. global_subspace (interior modes, boundary
    modes with the shared interface unknowns) is blockdiag(Lambda_d) (+) S."""
    p, sim, part, _ = box
    cms = CMSSolver(sim.L_ff, sim.free, sim.tets, part, n_modes=6)
    n = sim.free.size
    cols = []
    for dom, (lam, phi) in zip(cms.dom, cms.modes):
        I = dom[0]
        for k in range(phi.shape[1]):
            u = np.zeros(n)
            u[I] = phi[:, k]
            cols.append(u)
    nm = len(cols)
    for j, g in enumerate(cms.gamma):
        u = np.zeros(n)
        u[g] = 1.0
        for dom in cms.dom:
            I, bc, _, Psi = dom
            hit = np.nonzero(bc == j)[0]
            if hit.size:
                u[I] = Psi[:, hit[0]]
        cols.append(u)
    U = np.stack(cols, axis=1)
    R = U.T @ (cms.K @ U)
    lam_all = np.concatenate([lam for lam, _ in cms.modes])
    assert np.abs(R[:nm, :nm] - np.diag(lam_all)).max() <= 1e-9 * lam_all.max()
    assert np.abs(R[:nm, nm:]).max() <= 1e-9 * np.abs(R).max()
    assert np.abs(R[nm:, nm:] - cms.S).max() <= 1e-9 * np.abs(cms.S).max()


def test_interface_values_exact_and_truncation_monotone(box):
    """x^b of the reduced solve is exact whatever the mode count; the interior
    error in the K-norm falls as modes are added."""
    p, sim, part, rhs = box
    xe = sim._solve(rhs)
    prev = np.inf
    for r in (1, 5, 20, 40):
        cms = CMSSolver(sim.L_ff, sim.free, sim.tets, part, n_modes=r)
        x = cms.reduced(rhs)
        assert np.abs(x[cms.gamma] - xe[cms.gamma]).max() <= 1e-10 * np.abs(xe).max(), r
        e = x - xe
        en = float(np.einsum("ij,ij->", e, cms.K @ e))
        assert en < prev, r
        prev = en


def test_jacobi_fixed_point_and_chebyshev_convergence(box):
    """The exact solution is a fixed point of the weighted Jacobi sweeps, and
    from the reduced CMS solution the Chebyshev sweeps converge to it, faster
    than plain Jacobi sweeps."""
    p, sim, part, rhs = box
    xe = sim._solve(rhs)
    cms = CMSSolver(sim.L_ff, sim.free, sim.tets, part, n_modes=20, sweeps=40)
    assert np.abs(cms.polish(rhs, xe) - xe).max() <= 1e-12 * np.abs(xe).max()
    x0 = cms.reduced(rhs)
    e0 = np.abs(x0 - xe).max()
    e_cheb = np.abs(cms.polish(rhs, x0) - xe).max()
    plain = CMSSolver(sim.L_ff, sim.free, sim.tets, part, n_modes=20, sweeps=40, rho=0.0)
    e_plain = np.abs(plain.polish(rhs, x0) - xe).max()
    assert e_cheb < 0.01 * e0 and e_cheb < 0.2 * e_plain, (e0, e_cheb, e_plain)


def test_spectral_radius_and_weights():
    """rho of a 1-D Laplacian's Jacobi iteration is cos(pi / (n + 1)) (closed
    form); after omega_1 = 1 the weights jump to 2 / (2 - rho^2) and fall
    monotonically to the optimal SOR-like limit 2 / (1 + sqrt(1 - rho^2))."""
    n = 50
    K = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    rho = jacobi_spectral_radius(K)
    assert abs(rho - np.cos(np.pi / (n + 1))) < 1e-12
    w = chebyshev_weights(rho, 200)
    assert w[0] == 1.0 and abs(w[1] - 2.0 / (2.0 - rho * rho)) < 1e-15
    assert all(b < a for a, b in zip(w[1:], w[2:]))
    assert abs(w[-1] - 2.0 / (1.0 + np.sqrt(1.0 - rho * rho))) < 1e-9


def test_cms_step_error_is_reported_against_exact():
    """A whole PD step with the CMS solve correcting each iterate (20 modes)
    stays near the exact step, and the 10 Chebyshev-weighted Jacobi sweeps
    bring it more than 20 times closer (displacement-relative error)."""
    p = synth.problem_by_name("box")
    x0, v0 = p.initial_state()
    xe, _ = oracle.OracleSim.from_problem(p).step(x0, v0)
    errs = []
    for sw in (0, 10):
        sim = oracle.OracleSim(p.X, p.tets, p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt,
                               p.pd_iters, solver="cms", n_subdomains=p.n_subdomains, cms_sweeps=sw)
        x, _ = sim.step(x0, v0)
        errs.append(np.linalg.norm(x - xe) / np.linalg.norm(xe - p.X))
    assert errs[0] < 0.2 and errs[1] < 0.05 * errs[0], errs
