"""The inexact CMS global solve on the GPU (Sec. 7.2: interior eigenmodes,
boundary modes, the reduced solve of Eq. global_subspace on each PD
iteration's residual, Chebyshev-weighted Jacobi sweeps) against the FP64 CMS
oracle (oracle/cms.py) on the same partition (separators not thinned, so the
interfaces agree), and its error against the exact step.

Tolerances: as for the exact step (positions within 1e-5 relative L2 per
frame); the modes are stored in FP32, which moves a solve by about 1e-7 of
its size."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import rel_disp, rel_l2, say

pytestmark = pytest.mark.gpu

MODES, SWEEPS = 20, 10


@pytest.fixture(scope="module")
def vh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


@pytest.fixture(scope="module")
def ctx(vh):
    c = vh.Context(0)
    c.set_config(thin_separators=0, cms_modes=MODES, cms_sweeps=SWEEPS)
    yield c
    c.close()


def _mesh(vh, ctx, p):
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains)
    return m


def _oracle(p, sweeps=SWEEPS):
    return oracle.OracleSim(p.X, p.tets, p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters,
                            solver="cms", n_subdomains=p.n_subdomains, cms_modes=MODES, cms_sweeps=sweeps)


@pytest.mark.parametrize("name", ["box", "shell_small", "slab"])
def test_cms_solve_matches_oracle(vh, ctx, name):
    """One CMS solve of a random right-hand side (vh_debug_solve)."""
    say(f"[cms] solve {name}")
    p = synth.problem_by_name(name)
    m = _mesh(vh, ctx, p)
    sim = _oracle(p)
    rhs = np.random.default_rng(2).standard_normal((p.nv, 3))
    rhs[p.pinned.astype(bool)] = 0.0
    d = m.debug_solve(rhs)
    ref = np.zeros_like(rhs)
    ref[sim.free] = sim._solve(rhs[sim.free])
    e = rel_l2(d, ref)
    say(f"[cms] {name}: solve rel L2 vs the CMS oracle {e:.2e}")
    assert e <= 1e-6
    m.close()


@pytest.mark.parametrize("name,frames", [("box", 5), ("shell_small", 3)])
def test_cms_trajectory_matches_oracle(vh, ctx, name, frames):
    say(f"[cms] trajectory {name}")
    p = synth.problem_by_name(name)
    m = _mesh(vh, ctx, p)
    sim = _oracle(p)
    exact = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    xe, ve = p.initial_state()
    for f in range(frames):
        x, v = sim.step(x, v)
        xe, ve = exact.step(xe, ve)
    m.step(frames)
    xg, _ = m.read_state()
    e = rel_l2(xg, x)
    say(f"[cms] {name}: frame {frames} rel L2 vs the CMS oracle {e:.2e}; CMS vs exact: positions "
        f"{rel_l2(x, xe):.2e}, displacements {rel_disp(x, xe, p.X):.2e}")
    assert e <= 1e-5
    m.close()


def test_cms_misuse(vh, ctx):
    p = synth.problem_by_name("box")
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(p.n_subdomains, 1)                       # refinement with CMS
    assert ei.value.code == vh.VH_EINVAL
    m.prefactor(p.n_subdomains)
    x0, v0 = p.initial_state()
    with pytest.raises(vh.VHError) as ei:
        m.adjoint_forward(x0, v0, 2, 1)                       # the adjoint needs the exact solve
    assert ei.value.code == vh.VH_EINVAL
    with pytest.raises(vh.VHError) as ei:
        m.refactor(p.gamma_s, p.gamma_v)                      # the modes are rebuilt by prefactor
    assert ei.value.code == vh.VH_EINVAL
    with pytest.raises(vh.VHError) as ei:
        ctx.set_config(cms_modes=-1)
    assert ei.value.code == vh.VH_EINVAL
    m.close()
