"""FP64 reference for one projective-dynamics (PD) time step (paper Sec. 7).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Plain numpy/scipy in
float64; library primitives used as steps: batched LAPACK SVD
(``numpy.linalg.svd``), sparse LU (``scipy.sparse.linalg.splu``).

What one step computes (paper Sec. 7, Sec. 7.1):

* per element e, the energy of Eq. (energy) with projections of Eq. (pd_local):
  E_e = gs_e V_e ||F_e - R(F_e)||^2 + gv_e V_e ||F_e - V(F_e)||^2, where R is the
  nearest rotation (polar factor) and V the nearest volume-preserving matrix,
  found on the singular values by the problem of Eq. (vol_pre);
* the time discretisation of Sec. 7: a = x - x* - dt v* - dt^2 M^{-1} f, which
  makes the inertial target y = x* + dt v* + dt^2 g (gravity as f = M g);
* the PD split of Sec. 7.1: a local step (per-element projections) and a
  global step K x = b with the constant matrix and right-hand side printed
  there (the trailing "x" after K's parenthesis is read as a typo; b is taken
  with M y / dt^2 as its inertial term and with the projections of the current
  iterate, not of the previous time step -- otherwise the iteration would not
  iterate);
* ``pd_iters`` local/global iterations per step from x^(0) = y, then BDF1
  velocity v = (x_{n+1} - x_n) / dt.

The global matrix is separable: row c of F only involves coordinate c of the
four corners, so the paper's 3n x 3n K equals L (x) I_3 with the scalar
L = M / dt^2 + sum_e (gs_e + gv_e) V_e G_e, (G_e)_ab = gradN_a . gradN_b.
Pinned vertices are Dirichlet at their rest positions and eliminated.
"""

from __future__ import annotations

import math
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SL3_CLAMP = 0.01          # lower bound on a projected singular value (Sec. 7.1)


# ----------------------------------------------------------------------------
# Element geometry (Sec. 5: the operator D with F = D . (B_e x), and V_e)
# ----------------------------------------------------------------------------
def element_geometry(X, tets):
    """Rest-shape quantities per tet.

    Returns (V, grads) with V_e = det(Dm)/6, Dm = [X1-X0, X2-X0, X3-X0], and
    grads[e, a] = gradient of the linear shape function of corner a, so that
    F_e = sum_a x_a (outer) grads[e, a].  Rows 1..3 are the rows of Dm^{-1};
    row 0 is minus their sum.
    """
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)
    Dm = np.stack([X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]], X[t[:, 3]] - X[t[:, 0]]], axis=2)
    V = np.linalg.det(Dm) / 6.0
    Dinv = np.linalg.inv(Dm)
    grads = np.empty((t.shape[0], 4, 3))
    grads[:, 1:, :] = Dinv
    grads[:, 0, :] = -Dinv.sum(axis=1)
    return V, grads


def deformation_gradient(x, tets, grads):
    """F_e = sum_a x_a (outer) gradN_a  (nt, 3, 3)."""
    xe = np.asarray(x, dtype=np.float64)[np.asarray(tets, dtype=np.int64)]  # (nt, 4, 3)
    return np.einsum("eai,eaj->eij", xe, grads)


# ----------------------------------------------------------------------------
# Global matrix (Sec. 7.1, K)
# ----------------------------------------------------------------------------
def assemble_L(nv, tets, V, grads, gamma_s, gamma_v, mass, dt):
    """Scalar L = diag(m)/dt^2 + sum_e V_e (gs_e + gv_e) gradN_a . gradN_b (CSR)."""
    t = np.asarray(tets, dtype=np.int64)
    w = V * (np.asarray(gamma_s) + np.asarray(gamma_v))
    Ge = np.einsum("eai,ebi->eab", grads, grads) * w[:, None, None]
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    L = sp.coo_matrix((Ge.ravel(), (rows, cols)), shape=(nv, nv)).tocsr()
    L = L + sp.diags(np.asarray(mass, dtype=np.float64) / (dt * dt))
    L.sum_duplicates()
    return L.tocsr()


# ----------------------------------------------------------------------------
# Local step: SO(3) and SL(3) projections (Sec. 7.1, Eq. pd_local, Eq. vol_pre)
# ----------------------------------------------------------------------------
def signed_svd(F):
    """F = U diag(sigma) W^T with det U = det W = +1, sigma_1 >= sigma_2 >= |sigma_3|
    and sign(sigma_3) = sign(det F).  LAPACK SVD, then a sign fix."""
    U, S, Wt = np.linalg.svd(F)
    W = np.swapaxes(Wt, 1, 2).copy()
    U = U.copy()
    S = S.copy()
    du = np.linalg.det(U) < 0
    U[du, :, 2] *= -1.0
    S[du, 2] *= -1.0
    dw = np.linalg.det(W) < 0
    W[dw, :, 2] *= -1.0
    S[dw, 2] *= -1.0
    return U, S, W


def _plus_root(sig, mu):
    """Larger root of s^2 - sig s - mu = 0, evaluated without cancellation."""
    d = np.sqrt(np.maximum(sig * sig + 4.0 * mu, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        neg = np.where(d - sig > 0, 2.0 * mu / (d - sig), 0.0)
    return np.where(sig >= 0, 0.5 * (sig + d), neg), d


def _plus_branch(sig, logc=0.0):
    """Solve prod_i s_i(mu) = exp(logc) on the + branch s_i = (sig_i + sqrt(sig_i^2 + 4 mu))/2.

    Stationarity of the Lagrangian of Eq. (vol_pre) gives s_i (s_i - sig_i) = mu
    for every i; h(mu) = sum ln s_i(mu) - logc is increasing, so the root is
    bracketed and found by bisection, then polished by Newton.  Returns
    (s, mu, ok) where ok is False when the + branch has no root.
    """
    sig = np.atleast_2d(np.asarray(sig, dtype=np.float64))
    n = sig.shape[0]
    smin = sig.min(axis=1)
    allpos = smin > 0
    with np.errstate(divide="ignore"):
        logdet = np.where(allpos, np.log(np.abs(sig)).sum(axis=1), -np.inf)
    grow = logdet <= logc                      # root at mu >= 0
    lo = np.where(grow, 0.0, -0.25 * smin * smin)
    hi = np.where(grow, 1.0, 0.0)

    def h(mu):
        s, _ = _plus_root(sig, mu[:, None])
        with np.errstate(divide="ignore"):
            return np.log(s).sum(axis=1) - logc

    ok = np.ones(n, dtype=bool)
    # bracket: h(hi) > 0 where the root is above zero
    for _ in range(200):
        need = grow & (h(hi) <= 0)
        if not need.any():
            break
        hi = np.where(need, 2.0 * hi + 1.0, hi)
    # below zero: a root exists only if h(lo) < 0
    hlo = h(lo)
    ok &= grow | (hlo < 0)
    for _ in range(24):
        mid = 0.5 * (lo + hi)
        hm = h(mid)
        up = hm > 0
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
    mu = 0.5 * (lo + hi)
    for _ in range(6):                     # Newton polish, clipped to [lo, hi]
        s, d = _plus_root(sig, mu[:, None])
        with np.errstate(divide="ignore", invalid="ignore"):
            dh = (1.0 / (d * s)).sum(axis=1)
            f = np.log(s).sum(axis=1) - logc
            step = np.where(np.isfinite(dh) & (dh > 0), f / dh, 0.0)
        mu = np.clip(mu - step, lo, hi)
    s, _ = _plus_root(sig, mu[:, None])
    return s, mu, ok


def _squash_candidates(sig, logc=0.0):
    """Stationary points of Eq. (vol_pre) with one axis on the minus root, for
    the free axes ``sig`` (1-D) and the product target exp(logc).

    For mu < 0 the Lagrange condition s_i (s_i - sig_i) = mu also admits
    s_k = (sig_k - sqrt(sig_k^2 + 4 mu))/2 on one axis k (positive only when
    sig_k > 0).  Then s_k <= sig_k/2 and s_j <= sig_j, so such points exist
    only when every sig_i > 0 and prod sig >= 2 exp(logc).  Two axes on the
    minus root give saddle points of the Lagrangian (on the constraint's
    tangent space its Hessian weighs axis i by s_i (2 s_i - sig_i), negative
    on a minus root), so they cannot be the nearest point and are not
    searched.  Scalar search per
    axis: dense bracketing of mu in [-min sig^2/4, 0), then bisection.  Returns
    a list of candidate s vectors in axis order, roots of one axis by
    increasing |mu|.
    """
    sig = np.asarray(sig, dtype=np.float64)
    if sig.size < 2 or sig.min() <= 0 or np.log(sig).sum() < logc + math.log(2.0):
        return []
    lo = -0.25 * sig.min() ** 2
    mus = lo * np.geomspace(1e-14, 1.0, 4000)          # from just below 0 down to lo

    def branch(mu, k):
        """s on the mixed branch (axis k minus) for an array of mu."""
        mu = np.atleast_1d(mu)
        d = np.sqrt(np.maximum(sig[None, :] ** 2 + 4.0 * mu[:, None], 0.0))
        s = 0.5 * (sig[None, :] + d)
        s[:, k] = -2.0 * mu / (sig[k] + d[:, k])       # minus root without cancellation
        return s

    out = []
    for k in range(sig.size):
        with np.errstate(divide="ignore"):
            vals = np.log(branch(mus, k)).sum(axis=1) - logc
        for i in range(len(mus) - 1):
            if not (np.isfinite(vals[i]) and np.isfinite(vals[i + 1])):
                continue
            if np.sign(vals[i]) == np.sign(vals[i + 1]):
                continue
            a, b, fa = mus[i], mus[i + 1], vals[i]
            for _ in range(200):
                m = 0.5 * (a + b)
                fm = float(np.log(branch(m, k)).sum() - logc)
                if np.sign(fm) == np.sign(fa):
                    a, fa = m, fm
                else:
                    b = m
            out.append(branch(0.5 * (a + b), k)[0].copy())
    return out


def _nearest_on_product(sig, logc=0.0):
    """Nearest point to ``sig`` (the free axes, 1-D) on {prod s = exp(logc), s > 0}.

    The candidates are the + branch root (when it exists) and the mixed-branch
    roots of ``_squash_candidates``; the nearest wins, ties going to the +
    branch, then to the lower axis.  Returns (s, plus_ok, squash_won).
    """
    sig = np.asarray(sig, dtype=np.float64)
    if sig.size == 1:
        return np.array([math.exp(logc)]), True, False
    sp_, _, ok = _plus_branch(sig[None, :], logc=logc)
    cands = [sp_[0].copy()] if ok[0] else []
    cands += _squash_candidates(sig, logc)
    d = [float(((c - sig) ** 2).sum()) for c in cands]
    best = int(np.argmin(d))
    return cands[best], bool(ok[0]), (best != 0 or not ok[0])


def proj_sl3(sigma):
    """Projection of Eq. (vol_pre) with the clamp of Sec. 7.1.

    1. The nearest point on {s1 s2 s3 = 1, s_i > 0} to the signed singular
       values (the KKT problem with the equality constraint only): the + branch
       root, or, when det F >= 2, the nearest of it and the mixed-branch
       stationary points.
    2. The clamp: any component below 0.01 is set to 0.01 and frozen, and the
       remaining free components are re-solved as the nearest point with
       prod s_free = 1 / 0.01^(number frozen); repeated until no free
       component is below 0.01 (at most twice).  The result always has
       s1 s2 s3 = 1 and s_i >= 0.01.

    Returns (s, info) with info counting elements: inverted (sigma_3 <= 0),
    det_ge2 (all sigma > 0 and det F >= 2: the regime where mixed-branch
    stationary points exist), no_plus_root, squash (a mixed-branch point was
    taken, at step 1 or in a re-solve) and clamped (the clamp fired).
    """
    sigma = np.atleast_2d(np.asarray(sigma, dtype=np.float64))
    s, _, ok = _plus_branch(sigma)
    det_ge2 = (sigma.min(axis=1) > 0) & (np.prod(sigma, axis=1) >= 2.0)
    info = {"inverted": int((sigma[:, 2] <= 0).sum()), "det_ge2": int(det_ge2.sum()),
            "no_plus_root": int((~ok).sum()), "squash": 0, "clamped": 0}
    squashed = np.zeros(sigma.shape[0], dtype=bool)
    for e in np.nonzero((~ok) | det_ge2)[0]:
        s[e], _, won = _nearest_on_product(sigma[e], 0.0)
        squashed[e] = won
    for e in np.nonzero((s < SL3_CLAMP).any(axis=1))[0]:
        info["clamped"] += 1
        frozen = np.zeros(3, dtype=bool)
        se = s[e].copy()
        while True:
            newly = (~frozen) & (se < SL3_CLAMP)
            if not newly.any():
                break
            frozen |= newly
            se[frozen] = SL3_CLAMP
            free = ~frozen
            logc = -math.log(SL3_CLAMP) * int(frozen.sum())
            se[free], _, won = _nearest_on_product(sigma[e, free], logc)
            squashed[e] |= won
        s[e] = se
    info["squash"] = int(squashed.sum())
    return s, info


def local_step(x, tets, grads, w_s, w_v):
    """Per-element projections (Sec. 7.1): R = U W^T (polar rotation),
    V = U diag(Proj_SL3(sigma)) W^T, and the projection mix P = w_s R + w_v V
    with w = V_e gamma."""
    F = deformation_gradient(x, tets, grads)
    U, S, W = signed_svd(F)
    s, info = proj_sl3(S)
    Wt = np.swapaxes(W, 1, 2)
    R = U @ Wt
    Vp = (U * s[:, None, :]) @ Wt
    P = w_s[:, None, None] * R + w_v[:, None, None] * Vp
    return {"F": F, "U": U, "sigma": S, "W": W, "R": R, "s": s, "Vproj": Vp, "P": P, "info": info}


def scatter_corners(nv, tets, vec_e):
    """sum over (e, a) of vec_e[e, a, :] into vertex tets[e, a]  ->  (nv, 3)."""
    t = np.asarray(tets, dtype=np.int64).ravel()
    v = vec_e.reshape(-1, 3)
    return np.stack([np.bincount(t, weights=v[:, c], minlength=nv) for c in range(3)], axis=1)


def pd_energy(x, y, mass, dt, tets, grads, w_s, w_v):
    """Inertial plus elastic energy minimised by the PD iteration:
    (1/2dt^2) ||x - y||_M^2 + sum_e 1/2 (w_s ||F-R||^2 + w_v ||F-V||^2).

    The 1/2 on the elastic term matches K and b as printed (Sec. 7.1), which
    carry no factor 2; it is Eq. (energy) with gamma halved.
    """
    loc = local_step(x, tets, grads, w_s, w_v)
    F = loc["F"]
    el = 0.5 * (w_s * ((F - loc["R"]) ** 2).sum(axis=(1, 2)) + w_v * ((F - loc["Vproj"]) ** 2).sum(axis=(1, 2)))
    d = x - y
    return float(0.5 / (dt * dt) * (mass[:, None] * d * d).sum() + el.sum())


# ----------------------------------------------------------------------------
# The simulator
# ----------------------------------------------------------------------------
class OracleSim:
    """Plain FP64 PD simulator.  ``solver`` is 'exact' (global sparse LU of the
    free block of L), 'dd' (the exact domain-decomposed solve of oracle.dd) or
    'cms' (the inexact CMS solve of oracle.cms: cms_modes interior eigenmodes
    per domain, then cms_sweeps Chebyshev-weighted Jacobi sweeps)."""

    def __init__(self, X, tets, gamma_s, gamma_v, mass, pinned, gravity, dt, pd_iters=10,
                 solver="exact", n_subdomains=4, cms_modes=20, cms_sweeps=0):
        self.X = np.asarray(X, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.nv = self.X.shape[0]
        self.gamma_s = np.asarray(gamma_s, dtype=np.float64)
        self.gamma_v = np.asarray(gamma_v, dtype=np.float64)
        self.mass = np.asarray(mass, dtype=np.float64)
        self.pinned = np.asarray(pinned).astype(bool)
        self.g = np.asarray(gravity, dtype=np.float64)
        self.dt = float(dt)
        self.pd_iters = int(pd_iters)
        self.V, self.grads = element_geometry(self.X, self.tets)
        if (self.V <= 0).any():
            raise ValueError("non-positive rest volume")
        self.w_s = self.V * self.gamma_s
        self.w_v = self.V * self.gamma_v
        self.L = assemble_L(self.nv, self.tets, self.V, self.grads, self.gamma_s, self.gamma_v,
                            self.mass, self.dt)
        self.free = np.nonzero(~self.pinned)[0]
        self.fixed = np.nonzero(self.pinned)[0]
        self.L_ff = self.L[self.free][:, self.free].tocsc()
        self.L_fp = self.L[self.free][:, self.fixed].tocsr()
        self.solver_kind = solver
        if solver == "exact":
            self._lu = spla.splu(self.L_ff)
            self._solve = lambda b: self._lu.solve(b)
        elif solver == "dd":
            from .dd import DDSolver, bisect_elements
            part = bisect_elements(self.tets, n_subdomains)
            self._dd = DDSolver(self.L_ff, self.free, self.tets, part)
            self._solve = self._dd.solve
        elif solver == "cms":
            from .cms import CMSSolver
            from .dd import bisect_elements
            part = bisect_elements(self.tets, n_subdomains)
            self._dd = CMSSolver(self.L_ff, self.free, self.tets, part, cms_modes, cms_sweeps)
            self._solve = self._dd.solve
        else:
            raise ValueError(solver)
        self.last_info = {}
        self.energies = []

    def predictor(self, x, v):
        """y = x* + dt v* + dt^2 g on free vertices, rest position on pinned ones."""
        y = x + self.dt * v + self.dt * self.dt * self.g[None, :]
        y[self.fixed] = self.X[self.fixed]
        return y

    def rhs(self, y, P):
        """b = M y / dt^2 + sum_e B_e^T (D^T : P_e), restricted to free rows, minus L_fp x_p."""
        f = np.einsum("eij,eaj->eai", P, self.grads)        # P_e gradN_a per corner
        b = self.mass[:, None] * y / (self.dt * self.dt) + scatter_corners(self.nv, self.tets, f)
        return b[self.free] - self.L_fp @ self.X[self.fixed]

    def step(self, x, v, track_energy=False):
        """One time step (pd_iters local/global iterations).  Returns (x1, v1)."""
        x = np.asarray(x, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        y = self.predictor(x, v)
        xk = y.copy()
        info = {"inverted": 0, "det_ge2": 0, "no_plus_root": 0, "squash": 0, "clamped": 0}
        self.energies = []
        for _ in range(self.pd_iters):
            if track_energy:
                self.energies.append(pd_energy(xk, y, self.mass, self.dt, self.tets, self.grads,
                                               self.w_s, self.w_v))
            loc = local_step(xk, self.tets, self.grads, self.w_s, self.w_v)
            for k in info:
                info[k] += loc["info"][k]
            b = self.rhs(y, loc["P"])
            xk = xk.copy()
            if self.solver_kind == "cms":
                # an inexact solve corrects the current iterate (residual form)
                xf = xk[self.free]
                xk[self.free] = xf + self._solve(b - self.L_ff @ xf)
            else:
                xk[self.free] = self._solve(b)
        if track_energy:
            self.energies.append(pd_energy(xk, y, self.mass, self.dt, self.tets, self.grads,
                                           self.w_s, self.w_v))
        self.last_info = info
        v1 = (xk - x) / self.dt
        v1[self.fixed] = 0.0
        return xk, v1

    def run(self, x, v, frames):
        for _ in range(frames):
            x, v = self.step(x, v)
        return x, v

    @classmethod
    def from_problem(cls, p, solver="exact", n_subdomains=None):
        return cls(p.X, p.tets, p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt,
                   p.pd_iters, solver=solver,
                   n_subdomains=p.n_subdomains if n_subdomains is None else n_subdomains)
