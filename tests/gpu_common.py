"""Shared helpers of the GPU tests: build a library mesh from a synthetic problem
and the error measures of the parity bar."""

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_mesh(vhpd, ctx, p, n_subdomains=None, refine=0, pinned=None, gamma_s=None, gamma_v=None,
              gravity=None):
    m = vhpd.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s if gamma_s is None else gamma_s, p.gamma_v if gamma_v is None else gamma_v,
                 p.mass, p.pinned if pinned is None else pinned,
                 p.gravity if gravity is None else gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains if n_subdomains is None else n_subdomains, refine)
    return m


def rel_l2(a, b):
    """||a - b|| / ||b|| over all n_v x 3 absolute positions."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_disp(a, b, X):
    """Displacement-relative error ||(a - X) - (b - X)|| / ||b - X||."""
    d = np.linalg.norm(b - X)
    return float(np.linalg.norm(a - b) / d) if d > 0 else float(np.linalg.norm(a - b))


def deformed(p, amp=2e-3, seed=0):
    """A smooth, non-rigid deformation of the rest shape (pinned rows at rest)."""
    rng = np.random.default_rng(seed)
    k = rng.standard_normal((3, 3)) * 20.0
    ph = rng.uniform(0, 6.28, 3)
    x = p.X + amp * np.sin(p.X @ k.T + ph)
    x[p.pinned.astype(bool)] = p.X[p.pinned.astype(bool)]
    return x
