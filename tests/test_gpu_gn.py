"""The adjoint Gauss-Newton direction on the GPU (vh_mesh_gn_direction through
the C ABI) against the FP64 oracle (oracle/gn.py, Sec. 6.2, Eq. gn / Eq. agn).

Both sides linearise at the oracle's equilibrium of one step from rest (the
GPU's own equilibrium, from a step of 400 PD iterations, is compared
separately).  Tolerances: the projection Jacobian and the (F - R) factor of B
are FP32 like the local step, and the GN solve amplifies their rounding by at
most the condition number of P + kappa I, about 10 here; measured 2e-5 to
3.5e-5 relative L2 for the gradient and the direction, the bars are 2e-4 and
3e-4."""

import numpy as np
import pytest

import oracle
import synth
from oracle import gn
from tests.gpu_common import make_mesh, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


def _problem(name):
    if name == "box_tiny":
        return synth.make_box_problem(seed=12, nx=3, ny=3, nz=2, n_subdomains=2, name="box_tiny")
    return synth.problem_by_name(name)


@pytest.mark.parametrize("name", ["box_tiny", "box"])
def test_gn_direction_matches_oracle(vh, name):
    p = _problem(name)
    sim = oracle.OracleSim.from_problem(p)
    x0, v0 = p.initial_state()
    xs, y, n_it = gn.equilibrium(sim, x0, v0)
    rng = np.random.default_rng(8)
    gs_true = p.gamma_s * np.exp(0.05 * rng.standard_normal(p.nt))
    st = oracle.OracleSim(p.X, p.tets, gs_true, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    xt, _, _ = gn.equilibrium(st, x0, v0)
    _, grad_ref, J = gn.gn_direction_dense(sim, xs, xt, 1.0)
    pn = np.linalg.norm(J.T @ J, 2)
    kappa = 0.1 * pn
    d_ref, _ = gn.gn_direction_agn(sim, xs, xt, kappa)
    ctx = vh.Context(0)
    m = make_mesh(vh, ctx, p)
    grad, d, stats = m.gn_direction(xs, xt, kappa, max_outer=200, outer_tol=1e-8)
    eg, ed = rel_l2(grad, grad_ref), rel_l2(d, d_ref)
    say(f"[gn] {name}: oracle equilibrium after {n_it} PD iterations; gradient rel L2 {eg:.2e}, "
        f"direction rel L2 {ed:.2e}, stats {stats}")
    assert eg < 2e-4
    assert ed < 3e-4
    assert d @ grad < 0
    assert stats["outer_rel_residual"] <= 1e-8
    # the GPU's own equilibrium: one step of 400 PD iterations from rest
    m2 = vh.Mesh(ctx, p.X, p.tets)
    m2.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, 400)
    m2.prefactor(p.n_subdomains)
    m2.step(1)
    xg, _ = m2.read_state()
    ex = rel_l2(xg, xs)
    say(f"[gn] {name}: GPU equilibrium rel L2 {ex:.2e}")
    assert ex < 1e-6
    grad2, d2, _ = m2.gn_direction(xg, xt, kappa, max_outer=200, outer_tol=1e-8)
    e2 = rel_l2(d2, d_ref)
    say(f"[gn] {name}: direction at the GPU's own equilibrium, rel L2 {e2:.2e}")
    assert e2 < 2e-3
    m.close()
    m2.close()
    ctx.close()


def test_gn_errors(vh):
    p = _problem("box_tiny")
    ctx = vh.Context(0)
    m = make_mesh(vh, ctx, p)
    x = p.X.copy()
    for kw in ({"kappa": -1.0}, {"kappa": float("nan")}, {"outer_tol": 0.0}, {"max_outer": -1}):
        args = dict(kappa=1.0, max_outer=10, outer_tol=1e-6)
        args.update(kw)
        with pytest.raises(vh.VHError) as ei:
            m.gn_direction(x, x, **args)
        assert ei.value.code == vh.VH_EINVAL
    # x_eq == x_target: zero gradient, zero direction
    g, d, st = m.gn_direction(x, x, kappa=1.0, max_outer=10, outer_tol=1e-6)
    assert np.all(g == 0) and np.all(d == 0) and st["outer_iters"] == 0
    m.close()
    ctx.close()
