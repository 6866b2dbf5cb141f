"""FP64 adjoint Gauss-Newton direction for the per-element stiffness gamma_s
(paper Sec. 6.1-6.2: Eq. var, Eq. g, Eq. pxpgamma, Eq. adjoint_state,
Eq. adjoint_state_solve, Eq. gn, Eq. agn).  TEST INFRASTRUCTURE ONLY: the
product never imports it.

The forward map is one implicit Euler step solved to equilibrium: x*(gamma)
minimises the step energy of Eq. var with the elastic energy of Eq. energy
(with the 1/2 that K and b as printed imply),

    W(x) = 1/(2 dt^2) ||x - y||_M^2 + sum_e 1/2 V_e (gs_e ||F_e - R_e||^2 + gv_e ||F_e - V_e||^2),

so the equilibrium condition g(x, gamma) = 0 of Eq. g reads, on the free rows,

    g = M (x - y) / dt^2 + sum_e G_e^T P~_e,   P~_e = V_e (gs_e (F_e - R_e) + gv_e (F_e - V_e)),

where G_e maps x to F_e (F_e = sum_a x_a (outer) gradN_a) and R_e, V_e are the
projections of Eq. pd_local / Eq. vol_pre.  The projected PD iteration of
Sec. 7.1 converges to this point.  Its derivatives:

    dg/dx      = M / dt^2 + sum_e G_e^T ((w_s + w_v) I - J_P,e) G_e    (A, symmetric)
    dg/dgs_e   = V_e G_e^T (F_e - R_e)                                   (column e of B)

with J_P the derivative of P = w_s R + w_v V with respect to F, taken here by
central differences of P itself (per element, 9 directions).  For the loss
eps = 1/2 ||x* - x_target||^2 over the free vertices (so G = d2 eps / dx2 = I):

    gradient   d eps / d gamma = -lambda^T B,  A lambda = x* - x_target      (Eq. adjoint_state*)
    GN matrix  P = J^T G J,  J = dx*/dgamma = -A^{-1} B                        (Eq. pxpgamma, Eq. gn)
    direction  (P + kappa I) d = -(d eps / d gamma)^T                          (Eq. gn, Levenberg-Marquardt)

and the same direction from the sparse saddle system of Eq. agn,

    [ G    -A^T   0     ] [mu]   [ 0          ]
    [ -A    0     B     ] [nu] = [ 0          ]
    [ 0     B^T   kappa ] [ d]   [ -grad^T    ]

(the kappa I of the Levenberg-Marquardt step in the gamma block; the right-hand
side carries the minus sign of Eq. gn, so that d is a descent direction).
Vectors over vertices are flattened vertex-major over the free vertices.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .pd import OracleSim, deformation_gradient, local_step, scatter_corners


def equilibrium(sim: OracleSim, x, v, tol=1e-14, max_iters=20000):
    """x* of the step from (x, v): PD local/global iterations from x^(0) = y
    until the largest update is below tol times the mesh size."""
    y = sim.predictor(np.asarray(x, dtype=np.float64), np.asarray(v, dtype=np.float64))
    xk = y.copy()
    scale = np.abs(sim.X).max()
    for it in range(max_iters):
        loc = local_step(xk, sim.tets, sim.grads, sim.w_s, sim.w_v)
        xn = xk.copy()
        xn[sim.free] = sim._solve(sim.rhs(y, loc["P"]))
        step = np.abs(xn - xk).max()
        xk = xn
        if step <= tol * scale:
            return xk, y, it + 1
    raise RuntimeError("PD iteration did not reach the tolerance")


def residual(sim: OracleSim, x, y):
    """g of Eq. g on the free rows, [n_free, 3]."""
    loc = local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    Pt = (sim.w_s + sim.w_v)[:, None, None] * loc["F"] - loc["P"]
    f = scatter_corners(sim.nv, sim.tets, np.einsum("eij,eaj->eai", Pt, sim.grads))
    g = sim.mass[:, None] * (x - y) / (sim.dt * sim.dt) + f
    return g[sim.free]


def _projection(F, w_s, w_v):
    """P = w_s R + w_v V for deformation gradients F (n, 3, 3)."""
    from .pd import proj_sl3, signed_svd
    U, S, W = signed_svd(F)
    s, _ = proj_sl3(S)
    Wt = np.swapaxes(W, 1, 2)
    return w_s[:, None, None] * (U @ Wt) + w_v[:, None, None] * ((U * s[:, None, :]) @ Wt)


def projection_jacobian(F, w_s, w_v, h=1e-6):
    """dP/dF per element, (n, 9, 9) with rows the entries of dP and columns the
    entries of dF (row-major), by central differences with step h."""
    n = F.shape[0]
    J = np.zeros((n, 9, 9))
    for k in range(9):
        E = np.zeros(9)
        E[k] = h
        E = E.reshape(3, 3)
        Pp = _projection(F + E, w_s, w_v)
        Pm = _projection(F - E, w_s, w_v)
        J[:, :, k] = ((Pp - Pm) / (2 * h)).reshape(n, 9)
    return J


def _element_map(sim: OracleSim):
    """Per element the 9 x 12 matrix D_e with vec(F_e) = D_e [x_a0; x_a1; x_a2; x_a3]
    (F row-major, corners' coordinates in order)."""
    nt = sim.tets.shape[0]
    D = np.zeros((nt, 9, 12))
    for a in range(4):
        for c in range(3):
            for j in range(3):
                D[:, 3 * c + j, 3 * a + c] = sim.grads[:, a, j]
    return D


def _free_index(sim: OracleSim):
    idx = -np.ones(sim.nv, dtype=np.int64)
    idx[sim.free] = np.arange(sim.free.size)
    return idx


def dg_dx(sim: OracleSim, x):
    """A = dg/dx on the free rows and columns, sparse (3 n_free)^2."""
    loc = local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    JP = projection_jacobian(loc["F"], sim.w_s, sim.w_v)
    D = _element_map(sim)
    w = (sim.w_s + sim.w_v)[:, None, None]
    Ke = np.einsum("eki,ekl,elj->eij", D, w * np.eye(9)[None] - JP, D)      # 12 x 12 per element
    fi = _free_index(sim)
    dof = (3 * fi[sim.tets][:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    ok = (fi[sim.tets] >= 0).repeat(3, axis=1)
    rows, cols, vals = [], [], []
    for a in range(12):
        for b in range(12):
            m = ok[:, a] & ok[:, b]
            rows.append(dof[m, a])
            cols.append(dof[m, b])
            vals.append(Ke[m, a, b])
    nf3 = 3 * sim.free.size
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf3, nf3))
    md = np.repeat(sim.mass[sim.free] / (sim.dt * sim.dt), 3)
    return (A + sp.diags(md)).tocsc()


def dg_dgamma_s(sim: OracleSim, x):
    """B = dg/dgamma_s, sparse (3 n_free) x n_t: column e is V_e G_e^T (F_e - R_e)."""
    loc = local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    M = sim.V[:, None, None] * (loc["F"] - loc["R"])
    f = np.einsum("eij,eaj->eai", M, sim.grads)                  # (nt, 4, 3) corner forces
    fi = _free_index(sim)
    rows, cols, vals = [], [], []
    for a in range(4):
        m = fi[sim.tets[:, a]] >= 0
        for c in range(3):
            rows.append(3 * fi[sim.tets[m, a]] + c)
            cols.append(np.nonzero(m)[0])
            vals.append(f[m, a, c])
    nt = sim.tets.shape[0]
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * sim.free.size, nt)).tocsc()


def loss(sim: OracleSim, xstar, x_target):
    d = (xstar - x_target)[sim.free]
    return 0.5 * float((d * d).sum())


def gradient(sim: OracleSim, xstar, x_target, A=None, B=None):
    """d eps / d gamma_s by the adjoint state (Eq. adjoint_state, Eq. adjoint_state_solve)."""
    A = dg_dx(sim, xstar) if A is None else A
    B = dg_dgamma_s(sim, xstar) if B is None else B
    lam = spla.spsolve(A, (xstar - x_target)[sim.free].ravel())
    return -(B.T @ lam)


def gn_direction_dense(sim: OracleSim, xstar, x_target, kappa):
    """(P + kappa I) d = -grad with the dense P = J^T J, J = -A^{-1} B (Eq. gn)."""
    A = dg_dx(sim, xstar)
    B = dg_dgamma_s(sim, xstar)
    J = -spla.spsolve(A, B.toarray())
    grad = gradient(sim, xstar, x_target, A, B)
    P = J.T @ J
    d = np.linalg.solve(P + kappa * np.eye(P.shape[0]), -grad)
    return d, grad, J


def gn_direction_agn(sim: OracleSim, xstar, x_target, kappa):
    """The same direction from the sparse saddle system of Eq. agn."""
    A = dg_dx(sim, xstar)
    B = dg_dgamma_s(sim, xstar)
    grad = gradient(sim, xstar, x_target, A, B)
    n, m = A.shape[0], B.shape[1]
    I = sp.identity(n, format="csc")
    K = sp.bmat([[I, -A.T, None], [-A, None, B], [None, B.T, kappa * sp.identity(m)]], format="csc")
    rhs = np.concatenate([np.zeros(2 * n), -grad])
    sol = spla.splu(K).solve(rhs)
    return sol[2 * n:], grad
