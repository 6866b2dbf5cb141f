"""FP64 inexact component-mode-synthesis (CMS) solve of the PD global step
(paper Sec. 7.2: Eq. cms_boundary, the interior eigenmodes, Eq. global_subspace;
its closing paragraph and Sec. 8's implementation paragraph: Jacobi polishing
with Chebyshev weights).  TEST INFRASTRUCTURE ONLY: the product never imports it.

Per domain d (interior unknowns I_d, boundary unknowns touching it B_d):
  boundary modes   Psi_d = -(K_d^ii)^{-1} K_d^ib                 (Eq. cms_boundary)
  interior modes   Phi_d = the r eigenvectors of K_d^ii with the smallest
                   eigenvalues, K_d^ii Phi_d = Phi_d Lambda_d
and the subspace of Eq. global_subspace: x_d^i = Phi_d q_d + Psi_d x^b with one
shared x^b.  Because Phi_d^T (K_d^ii Psi_d + K_d^ib) = 0, the reduced matrix is
block diagonal, blockdiag(Lambda_d) and the interface Schur complement
S = K^bb + sum_d K_d^bi Psi_d, so the reduced solve is

    x^b   = S^{-1} (b^b + sum_d Psi_d^T b_d^i)
    q_d   = Lambda_d^{-1} Phi_d^T b_d^i
    x_d^i = Phi_d q_d + Psi_d x^b

(x^b is exact; x_d^i misses the response of the interior modes beyond r).
Then `sweeps` Jacobi iterations on K x = b polish the whole vector, with the
Chebyshev weights of the semi-iterative method (omega_1 = 1,
omega_2 = 2 / (2 - rho^2), omega_{k+1} = 4 / (4 - rho^2 omega_k), x_{k+1} =
omega_{k+1} (xhat_{k+1} - x_{k-1}) + x_{k-1}, xhat the plain Jacobi update of
x_k), rho the spectral radius of the Jacobi iteration matrix I - D^{-1} K.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dd import DDSolver


def jacobi_spectral_radius(K):
    """rho(I - D^{-1} K) from the extreme eigenvalues of D^{-1/2} K D^{-1/2}."""
    K = sp.csr_matrix(K)
    d = K.diagonal()
    Ds = sp.diags(1.0 / np.sqrt(d))
    A = (Ds @ K @ Ds).toarray() if K.shape[0] <= 4000 else None
    if A is not None:
        ev = np.linalg.eigvalsh(A)
    else:
        lo = spla.eigsh(Ds @ K @ Ds, k=1, which="SA", return_eigenvectors=False)
        hi = spla.eigsh(Ds @ K @ Ds, k=1, which="LA", return_eigenvectors=False)
        ev = np.array([lo[0], hi[0]])
    return float(max(abs(1.0 - ev.min()), abs(1.0 - ev.max())))


def chebyshev_weights(rho, n):
    """omega_1 .. omega_n of the Chebyshev semi-iteration."""
    w = []
    for k in range(n):
        if k == 0:
            w.append(1.0)
        elif k == 1:
            w.append(2.0 / (2.0 - rho * rho))
        else:
            w.append(4.0 / (4.0 - rho * rho * w[-1]))
    return w


class CMSSolver(DDSolver):
    """Reduced CMS solve plus Chebyshev-weighted Jacobi sweeps of L_ff x = b."""

    def __init__(self, L_ff, free, tets, elem_part, n_modes=20, sweeps=0, rho=None):
        super().__init__(L_ff, free, tets, elem_part)
        self.K = sp.csr_matrix(L_ff)
        self.n_modes = int(n_modes)
        self.modes = []
        for dom in self.dom:
            if dom is None:
                self.modes.append(None)
                continue
            I = dom[0]
            Kii = self.K[I][:, I].toarray()
            r = min(self.n_modes, I.size)
            lam, phi = sla.eigh(Kii, subset_by_index=[0, r - 1])
            self.modes.append((lam, phi))
        self.sweeps = int(sweeps)
        self.rho = jacobi_spectral_radius(self.K) if (rho is None and sweeps > 0) else rho
        self.inv_diag = 1.0 / self.K.diagonal()

    def reduced(self, b):
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = b[:, None] if vec else b
        x = np.zeros_like(B)
        rb = B[self.gamma].copy()
        for dom in self.dom:
            if dom is None:
                continue
            I, cols, _, Psi = dom
            rb[cols] += Psi.T @ B[I]                                    # b^b + Psi^T b^i
        xb = sla.cho_solve(self._S_chol, rb) if self.gamma.size else rb
        x[self.gamma] = xb
        for dom, md in zip(self.dom, self.modes):
            if dom is None:
                continue
            I, cols, _, Psi = dom
            lam, phi = md
            q = (phi.T @ B[I]) / lam[:, None]                            # Lambda^{-1} Phi^T b^i
            x[I] = phi @ q + Psi @ xb[cols]
        return x[:, 0] if vec else x

    def polish(self, b, x0):
        """`sweeps` Chebyshev-weighted Jacobi iterations from x0."""
        b = np.asarray(b, dtype=np.float64)
        D = self.inv_diag[:, None] if b.ndim == 2 else self.inv_diag
        w = chebyshev_weights(self.rho, self.sweeps)
        x_prev = x0.copy()
        x = x0.copy()
        for k in range(self.sweeps):
            xhat = x + D * (b - self.K @ x)
            x_new = w[k] * (xhat - x_prev) + x_prev
            x_prev, x = x, x_new
        return x

    def solve(self, b):
        x = self.reduced(b)
        return self.polish(b, x) if self.sweeps > 0 else x
