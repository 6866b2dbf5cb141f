"""FP64 embedding of points in the tet mesh (Eq. m2y).  Test infrastructure
only: the product never imports it.

The mesh-to-yarn map is phi(x) = N x: each embedded point moves with the
linear shape functions of its tet.  N is evaluated at the point's rest
position through the element Jacobian J = [X_1 - X_0, X_2 - X_0, X_3 - X_0]
that maps natural to material coordinates (the same J^{-1} Delta x as in the
mass lumping of Sec. 4): the natural coordinates are xi = J^{-1} (X^Y - X_0),
and N = (1 - xi_1 - xi_2 - xi_3, xi_1, xi_2, xi_3).
"""

from __future__ import annotations

import numpy as np


def shape_values(X, tets, tet, rest_xyz):
    """N [n, 4] of each point in its tet, from the rest positions."""
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)[np.asarray(tet, dtype=np.int64)]
    X0 = X[t[:, 0]]
    J = np.stack([X[t[:, 1]] - X0, X[t[:, 2]] - X0, X[t[:, 3]] - X0], axis=2)   # columns: edges
    xi = np.linalg.solve(J, (np.asarray(rest_xyz, dtype=np.float64) - X0)[:, :, None])[:, :, 0]
    return np.concatenate([1.0 - xi.sum(axis=1, keepdims=True), xi], axis=1)


def embed(x, tets, tet, N):
    """phi(x) = N x: positions [n, 3] of the points for vertex positions x."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)[np.asarray(tet, dtype=np.int64)]
    return np.einsum("na,nac->nc", N, x[t])
