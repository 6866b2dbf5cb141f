"""Seeded stand-ins for yarn points embedded in a tet mesh.

The paper embeds the yarn curves of a knit in its volume mesh; no yarn models
are available here, so each tet receives `per_tet` points at uniformly random
positions inside it (Dirichlet(1, 1, 1, 1) weights of its corners), listed tet
by tet.  Only the tet index and the rest position of each point leave this
module.
"""

from __future__ import annotations

import numpy as np


def yarn_points(X, tets, per_tet=4, seed=9):
    """(tet[n], rest_xyz[n, 3]) with n = per_tet * number of tets."""
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.dirichlet(np.ones(4), size=(t.shape[0], per_tet))        # [nt, k, 4]
    P = np.einsum("tka,tac->tkc", w, X[t])                           # [nt, k, 3]
    tet = np.repeat(np.arange(t.shape[0], dtype=np.int32), per_tet)
    return tet, P.reshape(-1, 3)
