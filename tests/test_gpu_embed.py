"""Embedded points (Eq. m2y) on the GPU, through the C ABI, against the FP64
oracle (oracle/embed.py).

Tolerance: the shape-function values are stored in FP32 (relative rounding
6e-8 of values in [0, 1]) and multiply edge vectors x_a - x_0, so a point may
move by about 3 * 6e-8 of its tet's longest deformed edge; the bar is 1e-6 of
that edge, per point."""

import numpy as np
import pytest

import synth
from oracle.embed import embed, shape_values
from tests.gpu_common import make_mesh, say

pytestmark = pytest.mark.gpu


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
    yield c
    c.close()


def _edge(x, tets, tet):
    xt = x[np.asarray(tets, dtype=np.int64)[tet]]                       # [n, 4, 3]
    e = np.linalg.norm(xt[:, :, None, :] - xt[:, None, :, :], axis=3)   # [n, 4, 4]
    return e.max(axis=(1, 2))


def _check(got, x, p, tet, N):
    ref = embed(x, p.tets, tet, N)
    err = np.linalg.norm(got - ref, axis=1) / _edge(x, p.tets, tet)
    return float(err.max())


@pytest.mark.parametrize("name", ["box", "shell_small"])
def test_embed_matches_oracle(vh, ctx, name):
    import torch
    p = synth.problem_by_name(name)
    tet, P = synth.yarn_points(p.X, p.tets, per_tet=4, seed=3)
    say(f"[embed] {name}: {len(tet)} points")
    N = shape_values(p.X, p.tets, tet, P)
    m = make_mesh(vh, ctx, p)
    m.set_embedding(tet, P)
    got = m.embed()
    assert _check(got, p.X, p, tet, N) < 1e-6                 # at rest: the rest points
    m.step(3)
    x, _ = m.read_state()
    got = m.embed()
    err = _check(got, x, p, tet, N)
    say(f"[embed] {name} after 3 frames: max error / edge {err:.2e}")
    assert err < 1e-6
    # the device variant writes the same bits
    out = torch.empty((len(tet), 3), dtype=torch.float64, device="cuda")
    m.embed_device(out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), got)
    m.close()


def test_embed_edge_cases(vh, ctx):
    p = synth.problem_by_name("box")
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    tet = np.repeat(np.arange(6, dtype=np.int32), 4)
    corners = p.X[p.tets[tet, np.tile(np.arange(4), 6)]]
    m.set_embedding(tet, corners)
    with pytest.raises(vh.VHError):
        m.embed()                                             # not prefactored
    m.prefactor(p.n_subdomains)
    m.step(2)
    x, _ = m.read_state()
    got = m.embed()
    ref = x[p.tets[tet, np.tile(np.arange(4), 6)]]
    assert np.abs(got - ref).max() <= 4e-16 * np.abs(ref).max() + 1e-18   # corners follow their vertex
    # refactoring renumbers the vertices; the records are rebuilt
    P2 = synth.yarn_points(p.X, p.tets, per_tet=2, seed=8)
    m.set_embedding(*P2)
    a = m.embed()
    m.prefactor(1)
    m.write_state(x, np.zeros_like(x))
    b = m.embed()
    assert np.abs(a - b).max() < 1e-15
    # no points, bad indices
    m.set_embedding(np.zeros(0, dtype=np.int32), np.zeros((0, 3)))
    assert m.embed().shape == (0, 3)
    with pytest.raises(vh.VHError):
        m.set_embedding(np.array([p.nt], dtype=np.int32), np.zeros((1, 3)))
    with pytest.raises(vh.VHError):
        m.set_embedding(np.array([-1], dtype=np.int32), np.zeros((1, 3)))
    with pytest.raises(vh.VHError):
        m.set_embedding(np.array([0], dtype=np.int32), np.array([[0.0, np.nan, 0.0]]))
    m.close()
