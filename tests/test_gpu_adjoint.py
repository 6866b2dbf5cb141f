"""The discrete adjoint on the GPU (vh_mesh_adjoint_forward / _backward through
the C ABI, and the torch.autograd wrapper) against the FP64 oracle adjoint.

Tolerance: the local-step Jacobian and the interior solves run in FP32, and the
gamma_s term differences two O(1) FP32 matrices (R - F) whose difference is of
the order of the strain, so the gradient carries about 1e-4 relative error;
the bar is 2e-3 in relative L2 over all elements."""

import numpy as np
import pytest

import oracle
import synth
from oracle.adjoint import loss_and_grad
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


def _target(p, frames, seed=0):
    rng = np.random.default_rng(seed)
    gs_hidden = p.gamma_s * np.exp(0.3 * rng.standard_normal(p.nt))
    sim = oracle.OracleSim(p.X, p.tets, gs_hidden, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    x0, v0 = p.initial_state()
    xt, _ = sim.run(x0, v0, frames)
    return xt


@pytest.mark.parametrize("name,frames,every,refine", [("box", 4, 3, 0), ("shell_small", 3, 2, 0), ("box", 3, 2, 1)])
def test_adjoint_matches_oracle(vh, name, frames, every, refine):
    """refine > 0: the forward and its replay refine every solve against the
    FP64 residual; the reverse sweep reverses the exact-solve iteration."""
    say(f"[adjoint] {name} frames={frames} every={every} refine={refine}")
    p = synth.problem_by_name(name)
    xt = _target(p, frames)
    _, g_ref = loss_and_grad(p, p.gamma_s, xt, frames)
    ctx = vh.Context(0)
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains, refine)
    x0, v0 = p.initial_state()
    xf = m.adjoint_forward(x0, v0, frames, every)
    # same trajectory as plain stepping, bit for bit
    m2 = vh.Mesh(ctx, p.X, p.tets)
    m2.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m2.prefactor(p.n_subdomains, refine)
    m2.step(frames)
    assert np.array_equal(m2.read_state()[0], xf)
    d = xf - xt
    d[p.pinned.astype(bool)] = 0.0
    g = m.adjoint_backward(d)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    say(f"[adjoint] {name}: |g| {np.linalg.norm(g_ref):.3e}, rel L2 vs oracle adjoint {err:.2e}")
    assert err < 2e-3
    # a second backward of the same forward gives the same gradient
    g2 = m.adjoint_backward(d)
    assert np.array_equal(g, g2)
    m.close()
    m2.close()
    ctx.close()


def test_autograd_trajectory(vh):
    import torch
    from paper_2405_12484_amd.autograd import Trajectory
    p = synth.problem_by_name("box")
    frames = 3
    xt = _target(p, frames)
    ctx = vh.Context(0)
    traj = Trajectory(ctx, p.X, p.tets, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters,
                      n_subdomains=p.n_subdomains, frames=frames, ckpt_every=2)
    gs = torch.tensor(p.gamma_s, dtype=torch.float64, requires_grad=True)
    x = traj(gs)
    free = torch.tensor(~p.pinned.astype(bool))
    loss = 0.5 * (((x - torch.tensor(xt)) ** 2).sum(dim=1) * free).sum()
    loss.backward()
    _, g_ref = loss_and_grad(p, p.gamma_s, xt, frames)
    err = np.linalg.norm(gs.grad.numpy() - g_ref) / np.linalg.norm(g_ref)
    say(f"[adjoint] autograd box: rel L2 vs oracle adjoint {err:.2e}")
    assert err < 2e-3
    # two outputs before their backwards: each gradient belongs to its own gamma_s
    gs_b = torch.tensor(p.gamma_s * 1.5, dtype=torch.float64, requires_grad=True)
    gs_a = torch.tensor(p.gamma_s, dtype=torch.float64, requires_grad=True)
    xa = traj(gs_a)
    xb = traj(gs_b)
    la = 0.5 * (((xa - torch.tensor(xt)) ** 2).sum(dim=1) * free).sum()
    lb = 0.5 * (((xb - torch.tensor(xt)) ** 2).sum(dim=1) * free).sum()
    la.backward()
    assert np.allclose(gs_a.grad.numpy(), gs.grad.numpy(), rtol=1e-10, atol=0)
    lb.backward()
    _, g_ref_b = loss_and_grad(p, p.gamma_s * 1.5, xt, frames)
    err_b = np.linalg.norm(gs_b.grad.numpy() - g_ref_b) / np.linalg.norm(g_ref_b)
    say(f"[adjoint] autograd box, second output at 1.5 gamma_s: rel L2 vs oracle adjoint {err_b:.2e}")
    assert err_b < 2e-3
    with pytest.raises(vh.VHError):
        m = vh.Mesh(ctx, p.X, p.tets)
        m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
        m.prefactor(p.n_subdomains)
        m.adjoint_backward(np.zeros((p.nv, 3)))          # no forward yet
    traj.close()
    ctx.close()
