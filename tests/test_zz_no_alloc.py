"""vh_mesh_step_noalloc (the step with its work buffers in the library's fixed
scratch array, for callers that cannot allocate device memory) against
vh_mesh_step on the same state: two calls in a row, the second on a smaller
mesh, each bitwise equal to the plain step (same kernels, same arguments but
the work-buffer addresses, which no result depends on)."""

import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_common import make_mesh, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


def _deformed_state(p, seed):
    rng = np.random.default_rng(seed)
    x = p.X + 1e-3 * rng.standard_normal(p.X.shape)
    v = 0.05 * rng.standard_normal(p.X.shape)
    pin = p.pinned.astype(bool)
    x[pin] = p.X[pin]
    v[pin] = 0.0
    return x, v


@pytest.mark.parametrize("first,second", [("shell", "box"), ("slab", "shell_small")])
def test_noalloc_step_equals_step(vh, first, second):
    import torch
    ctx = vh.Context(0)
    stream = torch.cuda.current_stream()
    for name, frames, seed in ((first, 3, 1), (second, 2, 2)):
        say(f"[noalloc] {name}, {frames} frames")
        p = synth.problem_by_name(name)
        a = make_mesh(vh, ctx, p, refine=1)
        b = make_mesh(vh, ctx, p, refine=1)
        x0, v0 = _deformed_state(p, seed)
        a.write_state(x0, v0)
        b.write_state(x0, v0)
        a.step(frames, stream)
        b.step_noalloc(frames, stream)
        xa, va = a.read_state(stream)
        xb, vb = b.read_state(stream)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), name
        a.close()
        b.close()
    ctx.close()


def test_noalloc_rejects_oversized_mesh(vh):
    """A 560,000-tet shell needs more step scratch (about 20 MB) than the
    array holds (16 MiB): the call fails with VH_EINVAL and changes nothing."""
    ctx = vh.Context(0)
    p = synth.make_shell_problem(seed=9, n_theta=400, n_z=140, n_subdomains=256, name="shell_560k")
    m = make_mesh(vh, ctx, p)
    x0, _ = m.read_state()
    with pytest.raises(vh.VHError) as ei:
        m.step_noalloc(1)
    assert ei.value.code == vh.VH_EINVAL and "scratch" in str(ei.value)
    assert np.array_equal(m.read_state()[0], x0)
    m.close()
    ctx.close()
