"""FP64 domain-decomposed global solve (paper Sec. 7.2), for the oracle.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper partitions the mesh into domains, splits each domain's unknowns into
internal (i) and boundary (b) DOFs, builds the boundary modes of
Eq. (cms_boundary), Psi_d = -(K_d^ii)^{-1} K_d^ib, and solves the global system
in the subspace of Eq. (global_subspace), where the duplicated boundary DOFs of
neighbouring domains become one shared x^b (Eq. dd and the text after it).

Reading used here: the interior eigenmodes Phi_d of the paper are replaced by
the exact interior solve (K_d^ii)^{-1}.  With that, the subspace of
Eq. (global_subspace) spans the whole space and the reduced matrix splits into
the interior blocks and the interface Schur complement
S = K^bb - sum_d K_d^bi (K_d^ii)^{-1} K_d^ib = K^bb + sum_d K_d^bi Psi_d,
so the decomposed solve equals the global solve up to rounding:
  x^b    = S^{-1} (b^b + sum_d Psi_d^T b_d^i)
  x_d^i  = (K_d^ii)^{-1} b_d^i + Psi_d x^b.

Partition: recursive bisection of the element face-adjacency graph; each cut
runs a breadth-first search from a pseudo-peripheral element (two sweeps,
neighbours visited in ascending index) and splits the visit order at floor(n/2);
part p splits into 2p and 2p+1.  Boundary DOFs are the free vertices touched
by elements of two or more parts.
"""

from __future__ import annotations

from collections import deque

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def face_adjacency(tets):
    """CSR (indptr, indices) of tets sharing a triangular face."""
    t = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    nt = t.shape[0]
    faces = np.concatenate([t[:, [0, 1, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 3]], t[:, [1, 2, 3]]])
    owner = np.tile(np.arange(nt), 4)
    order = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    f = faces[order]
    o = owner[order]
    same = np.all(f[1:] == f[:-1], axis=1)
    a = o[:-1][same]
    b = o[1:][same]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    A = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(nt, nt)).tocsr()
    A.sort_indices()
    return A.indptr, A.indices


def _bfs_order(start, members, indptr, indices, inset):
    """BFS over ``members`` (boolean mask inset) from ``start``; continues from the
    lowest unvisited member when a component is exhausted."""
    seen = {start}
    order = [start]
    q = deque([start])
    pending = sorted(members)
    pi = 0
    while len(order) < len(members):
        while q:
            u = q.popleft()
            for w in indices[indptr[u]:indptr[u + 1]]:
                w = int(w)
                if inset[w] and w not in seen:
                    seen.add(w)
                    order.append(w)
                    q.append(w)
        while len(order) < len(members) and pi < len(pending):
            c = pending[pi]
            pi += 1
            if c not in seen:
                seen.add(c)
                order.append(c)
                q.append(c)
                break
    return order


def bisect_elements(tets, n_parts):
    """Element -> part id, n_parts = 2^k parts by recursive BFS bisection."""
    tets = np.asarray(tets)
    nt = tets.shape[0]
    if n_parts < 1 or (n_parts & (n_parts - 1)):
        raise ValueError("n_parts must be a power of two")
    indptr, indices = face_adjacency(tets)
    parts = [list(range(nt))]
    while len(parts) < n_parts:
        nxt = []
        for members in parts:
            inset = np.zeros(nt, dtype=bool)
            inset[members] = True
            first = _bfs_order(min(members), members, indptr, indices, inset)
            second = _bfs_order(first[-1], members, indptr, indices, inset)
            h = len(second) // 2
            nxt.append(second[:h])
            nxt.append(second[h:])
        parts = nxt
    part = np.empty(nt, dtype=np.int64)
    for p, members in enumerate(parts):
        part[members] = p
    return part


class DDSolver:
    """Exact decomposed solve of L_ff x = b (several right-hand-side columns)."""

    def __init__(self, L_ff, free, tets, elem_part):
        L_ff = sp.csr_matrix(L_ff)
        n = L_ff.shape[0]
        nv = int(max(np.max(tets) + 1, np.max(free) + 1))
        g2f = -np.ones(nv, dtype=np.int64)
        g2f[np.asarray(free)] = np.arange(n)
        nparts = int(elem_part.max()) + 1
        touch = [set() for _ in range(n)]
        for e, p in enumerate(np.asarray(elem_part)):
            for a in tets[e]:
                fa = g2f[a]
                if fa >= 0:
                    touch[fa].add(int(p))
        owner = np.array([next(iter(s)) if len(s) == 1 else -1 for s in touch])
        self.gamma = np.nonzero(owner < 0)[0]
        self.interiors = [np.nonzero(owner == d)[0] for d in range(nparts)]
        self.n = n
        K_gg = L_ff[self.gamma][:, self.gamma].toarray()
        self.dom = []
        S = K_gg.copy()
        for I in self.interiors:
            if I.size == 0:
                self.dom.append(None)
                continue
            K_ii = L_ff[I][:, I].tocsc()
            K_ib = L_ff[I][:, self.gamma].tocsc()
            cols = np.unique(K_ib.nonzero()[1])            # boundary DOFs this domain touches
            lu = spla.splu(K_ii)
            # boundary modes, Eq. (cms_boundary): Psi = -(K^ii)^{-1} K^ib
            Psi = -lu.solve(K_ib[:, cols].toarray()) if cols.size else np.zeros((I.size, 0))
            # Schur contribution K^bi Psi
            S[np.ix_(cols, cols)] += K_ib[:, cols].T @ Psi
            self.dom.append((I, cols, lu, Psi))
        self.S = S
        self._S_chol = None
        if self.gamma.size:
            import scipy.linalg as sla
            self._S_chol = sla.cho_factor(S, lower=True)

    def solve(self, b):
        import scipy.linalg as sla
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = b[:, None] if vec else b
        x = np.zeros_like(B)
        rb = B[self.gamma].copy()
        ys = []
        for dom in self.dom:
            if dom is None:
                ys.append(None)
                continue
            I, cols, lu, Psi = dom
            y = lu.solve(B[I])
            ys.append(y)
            rb[cols] += Psi.T @ B[I]                       # b^b + Psi^T b^i
        xb = sla.cho_solve(self._S_chol, rb) if self.gamma.size else rb
        x[self.gamma] = xb
        for dom, y in zip(self.dom, ys):
            if dom is None:
                continue
            I, cols, lu, Psi = dom
            x[I] = y + Psi @ xb[cols]
        return x[:, 0] if vec else x
