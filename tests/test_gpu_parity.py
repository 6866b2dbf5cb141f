"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: positions within 1e-5 relative L2 per step (FP32 bulk arithmetic);
per-kernel tolerances follow from FP32 rounding of O(1) quantities (the
deformation gradient, singular values) scaled by the element weights."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import deformed, make_mesh, rel_disp, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vh():
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


@pytest.fixture(scope="module")
def ctx(vh):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = vh.Context(0)
    yield c
    c.close()


# --- local step ----------------------------------------------------------------
@pytest.mark.parametrize("name", ["box", "shell_small"])
def test_local_step_matches_oracle(vh, ctx, name):
    say(f"[local] {name}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    for amp in (0.0, 1e-3, 5e-3):
        x = deformed(p, amp=amp, seed=1)
        T, sig, s = m.debug_local_step(x)
        loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
        Tref = loc["P"] - (sim.w_s + sim.w_v)[:, None, None] * loc["F"]
        w = (sim.w_s + sim.w_v)[:, None, None]
        err = np.abs(T - Tref) / w
        assert err.max() < 2e-5, (amp, err.max())
        assert np.abs(sig - loc["sigma"]).max() < 2e-6
        assert np.abs(s - loc["s"]).max() < 2e-6
        if amp == 0.0:
            assert np.abs(T).max() == 0.0          # F = I exactly at rest
    m.close()


def _shared_regime(S, s_ref):
    """Elements where the oracle's projection is the + branch root (Eq. vol_pre
    has one: always when det F <= 1, else when h(-sigma_min^2 / 4) <= 0) and
    the device keeps its Newton result (det F < 2, no clamp)."""
    det = S.prod(axis=1)
    smin = np.abs(S).min(axis=1)
    arg = np.maximum(S * S - smin[:, None] ** 2, 0.0)
    h_lo = np.log(np.maximum((S + np.sqrt(arg)) / 2, 1e-300)).sum(axis=1)
    plus_root = (det <= 1.0) | (h_lo <= 0.0)
    return plus_root & (det < 2.0) & (s_ref.min(axis=1) > 0.011)


@pytest.mark.parametrize("amp", [0.01, 0.02])
def test_local_step_large_strain_and_inverted(vh, ctx, amp):
    """Singular values from about 0.25 to 3.7, and (amp 0.02) inverted elements."""
    say(f"[local] large strain amp={amp}")
    p = synth.problem_by_name("box")
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    x = deformed(p, amp=amp, seed=1)
    T, sig, s = m.debug_local_step(x)
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    S = loc["sigma"]
    keep = _shared_regime(S, loc["s"])
    n_inv = int((S[:, 2] < 0).sum())
    say(f"[local] amp={amp}: {keep.sum()} of {len(S)} elements compared, {n_inv} inverted")
    assert keep.sum() > 0.9 * len(S)
    if amp >= 0.02:
        assert (keep & (S[:, 2] < 0)).sum() > 0      # inverted elements are in the comparison
    Tref = loc["P"] - (sim.w_s + sim.w_v)[:, None, None] * loc["F"]
    w = (sim.w_s + sim.w_v)[:, None, None]
    err = (np.abs(T - Tref) / w).max(axis=(1, 2))
    # the rotation's sensitivity to rounding of F grows like 2 / (sigma_i + sigma_j)
    pair = np.minimum.reduce([S[:, 0] + S[:, 1], S[:, 0] + S[:, 2], S[:, 1] + S[:, 2]])
    scale = np.maximum(1.0, np.abs(S).max(axis=1)) * np.maximum(1.0, 2.0 / np.abs(pair))
    assert (err[keep] / scale[keep]).max() < 2e-5, (err[keep] / scale[keep]).max()
    big = np.maximum(1.0, np.abs(S).max(axis=1))[:, None]
    assert (np.abs(sig - S) / big)[keep].max() < 4e-6
    assert (np.abs(s - loc["s"]) / big)[keep].max() < 4e-6
    m.close()


def test_local_step_rigid_rotation_zero_stress(vh, ctx):
    say("[local] rigid rotation")
    p = synth.problem_by_name("box")
    pins = np.zeros(p.nv, dtype=np.uint8)
    m = make_mesh(vh, ctx, p, pinned=pins)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    x = p.X @ Q.T + np.array([0.01, 0.02, -0.03])
    T, sig, s = m.debug_local_step(x)
    V, _ = oracle.element_geometry(p.X, p.tets)
    w = (V * (p.gamma_s + p.gamma_v))[:, None, None]
    # FP32 rounding of O(1) singular values: |T| / w is a few ulp of 1
    assert np.abs(T / w).max() < 2e-6
    assert np.abs(sig - 1).max() < 2e-6 and np.abs(s - 1).max() < 2e-6
    m.close()


# --- residual (local step + scatter) ------------------------------------------------
@pytest.mark.parametrize("name", ["box", "shell_small"])
def test_residual_matches_oracle(vh, ctx, name):
    say(f"[residual] {name}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    x = deformed(p, amp=2e-3, seed=2)
    y = deformed(p, amp=1e-3, seed=3)
    r = m.debug_residual(x, y)
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    rref = sim.rhs(y, loc["P"]) - sim.L_ff @ x[sim.free]
    assert np.linalg.norm(r[sim.free] - rref) <= 1e-5 * np.linalg.norm(rref)
    assert np.all(r[sim.fixed] == 0)
    m.close()


# --- decomposed solve ---------------------------------------------------------------
@pytest.mark.parametrize("name,D", [("box", 4), ("box", 1), ("shell_small", 8), ("slab", 8)])
def test_solve_matches_exact(vh, ctx, name, D):
    say(f"[solve] {name} D={D}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p, n_subdomains=D)
    sim = oracle.OracleSim.from_problem(p)
    rng = np.random.default_rng(4)
    rhs = rng.standard_normal((p.nv, 3))
    d = m.debug_solve(rhs)
    xe = sim._solve(rhs[sim.free])
    assert np.linalg.norm(d[sim.free] - xe) <= 5e-7 * np.linalg.norm(xe)
    assert np.all(d[sim.fixed] == 0)
    m.close()


# --- whole steps ---------------------------------------------------------------------
@pytest.mark.parametrize("name", ["box", "shell_small"])
def test_trajectory_matches_oracle(vh, ctx, name):
    """Free-running frames; every frame within 1e-5 relative L2 of the oracle,
    and lock-step (GPU started from the oracle's state) within 1e-5 too."""
    say(f"[trajectory] {name}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    worst = 0.0
    for f in range(p.frames):
        xo, vo = sim.step(x, v)
        m.step(1)
        xg, vg = m.read_state()
        e = rel_l2(xg, xo)
        worst = max(worst, e)
        assert e <= 1e-5, (f, e)
        # lock-step from the oracle state
        m.write_state(x, v)
        m.step(1)
        xl, _ = m.read_state()
        assert rel_l2(xl, xo) <= 1e-5
        m.write_state(xg, vg)
        x, v = xo, vo
    say(f"   worst rel L2 {worst:.3e}, displacement-relative {rel_disp(xg, xo, p.X):.3e}")
    m.close()


def test_box_matches_stored_oracle_frames(vh, ctx):
    """The 1,000-tet box workload (20 frames) against the oracle positions
    stored in tests/golden/box_oracle_frames.txt."""
    from tests.test_golden import load_box_frames
    ref = load_box_frames()
    p = synth.problem_by_name("box")
    m = make_mesh(vh, ctx, p)
    for f in range(1, 21):
        m.step(1)
        if f in ref:
            x, _ = m.read_state()
            e = rel_l2(x, ref[f])
            say(f"[golden] box frame {f}: rel L2 {e:.2e}")
            assert e <= 1e-5
    m.close()


def test_free_fall_without_stiffness(vh, ctx):
    say("[free fall]")
    p = synth.problem_by_name("box")
    z = np.zeros(p.nt)
    m = make_mesh(vh, ctx, p, gamma_s=z, gamma_v=z)
    rng = np.random.default_rng(5)
    v0 = 0.1 * rng.standard_normal(p.X.shape)
    v0[p.pinned.astype(bool)] = 0
    m.write_state(p.X, v0)
    m.step(1)
    x1, v1 = m.read_state()
    free = ~p.pinned.astype(bool)
    want = p.X + p.dt * (v0 + p.dt * p.gravity)
    assert np.abs(x1[free] - want[free]).max() < 1e-15
    m.close()


def test_rest_fixed_point(vh, ctx):
    say("[rest]")
    p = synth.problem_by_name("shell_small")
    m = make_mesh(vh, ctx, p, gravity=np.zeros(3))
    m.step(3)
    x, v = m.read_state()
    assert np.abs(x - p.X).max() == 0.0 and np.abs(v).max() == 0.0
    m.close()


def test_deterministic_and_resume(vh, ctx):
    """Two runs are bitwise equal; a run resumed from a read/written state equals
    the uninterrupted one bitwise."""
    say("[determinism]")
    p = synth.problem_by_name("shell_small")
    a = make_mesh(vh, ctx, p)
    b = make_mesh(vh, ctx, p)
    a.step(6)
    b.step(3)
    xs, vs = b.read_state()
    b.write_state(xs, vs)
    b.step(3)
    xa, va = a.read_state()
    xb, vb = b.read_state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    a.close()
    b.close()


def test_device_state_roundtrip(vh, ctx):
    import torch
    say("[device state]")
    p = synth.problem_by_name("box")
    m = make_mesh(vh, ctx, p)
    m.step(2)
    xh, vh_ = m.read_state()
    xt = torch.empty((p.nv, 3), dtype=torch.float64, device="cuda")
    vt = torch.empty_like(xt)
    s = torch.cuda.current_stream()
    m.read_state_device(xt, vt, s)
    torch.cuda.synchronize()
    assert np.array_equal(xt.cpu().numpy(), xh) and np.array_equal(vt.cpu().numpy(), vh_)
    m.write_state_device(xt, vt * 0, s)
    torch.cuda.synchronize()
    x2, v2 = m.read_state()
    assert np.array_equal(x2, xh) and np.abs(v2).max() == 0.0
    m.close()


def test_errors_are_reported(vh, ctx):
    say("[errors]")
    p = synth.problem_by_name("box")
    bad = p.tets.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]                        # inverted rest tet
    with pytest.raises(vh.VHError) as ei:
        vh.Mesh(ctx, p.X, bad)
    assert ei.value.code == vh.VH_EINVAL
    m = vh.Mesh(ctx, p.X, p.tets)
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(4)
    assert ei.value.code == vh.VH_ESTATE
    g = p.gamma_s.copy()
    g[3] = -1.0
    with pytest.raises(vh.VHError) as ei:
        m.set_params(g, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, 10)
    assert ei.value.code == vh.VH_EINVAL
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, 10)
    with pytest.raises(vh.VHError) as ei:
        m.step(1)
    assert ei.value.code == vh.VH_ESTATE
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(3)
    assert ei.value.code == vh.VH_EINVAL
    m.prefactor(4)
    x = p.X.copy()
    x[5, 0] = np.nan
    m.write_state(x, np.zeros_like(x))
    m.step(1)
    with pytest.raises(vh.VHError) as ei:
        m.read_state()
    assert ei.value.code == vh.VH_ENUMERIC
    m.close()


def test_degenerate_meshes(vh, ctx):
    """Every vertex pinned (no unknowns: the state stays at rest exactly), zero
    frames, and a single tet with one free vertex against the oracle."""
    say("[degenerate] all pinned")
    p = synth.problem_by_name("box")
    m = make_mesh(vh, ctx, p, pinned=np.ones(p.nv, dtype=np.uint8))
    assert m.info()["n_free"] == 0
    m.step(0)
    m.step(3)
    x, v = m.read_state()
    assert np.array_equal(x, p.X) and not np.any(v)
    m.close()
    say("[degenerate] single tet")
    X = np.array([[0.0, 0.0, 0.0], [0.01, 0.0, 0.0], [0.0, 0.01, 0.0], [0.003, 0.002, 0.01]])
    T = np.array([[0, 1, 2, 3]], dtype=np.int32)
    gs, gv = np.array([1e4]), np.array([3e3])
    mass = np.full(4, 1e-4)
    pins = np.array([1, 1, 1, 0], dtype=np.uint8)
    g = np.array([0.0, 0.0, -9.8])
    m = vh.Mesh(ctx, X, T)
    m.set_params(gs, gv, mass, pins, g, 1.0 / 150, 10)
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(2)                                    # more subdomains than elements
    assert ei.value.code == vh.VH_EINVAL
    m.prefactor(1)
    m.step(5)
    x, _ = m.read_state()
    sim = oracle.OracleSim(X, T, gs, gv, mass, pins, g, 1.0 / 150, 10)
    xo, vo = X.copy(), np.zeros_like(X)
    for _ in range(5):
        xo, vo = sim.step(xo, vo)
    err = rel_disp(x, xo, X)
    say(f"[degenerate] single tet after 5 frames: displacement-relative {err:.2e}")
    assert rel_l2(x, xo) < 1e-5 and err < 1e-4
    m.close()


def test_refinement_steps(vh, ctx):
    """Refinement against the FP64 residual (k_refine + further solves): the
    refined trajectory meets the same bar, differs from the plain one, and is
    bitwise the same when two copies of the garment are served batched."""
    say("[refine]")
    p = synth.problem_by_name("shell_small")
    sim = oracle.OracleSim.from_problem(p)
    xo, vo = p.initial_state()
    for _ in range(3):
        xo, vo = sim.step(xo, vo)
    res = {}
    for R in (0, 2):
        m = make_mesh(vh, ctx, p, refine=R)
        m.step(3)
        res[R] = m.read_state()[0]
        m.close()
        say(f"[refine] steps={R}: rel L2 vs oracle {rel_l2(res[R], xo):.2e}")
    assert rel_l2(res[2], xo) < 1e-5
    assert not np.array_equal(res[0], res[2])
    c2 = vh.Context(0)
    srv = vh.Server(c2, "batched", 2)
    ms = []
    for _ in range(2):
        mm = vh.Mesh(c2, p.X, p.tets)
        mm.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
        srv.add(mm, p.n_subdomains, 2)
        ms.append(mm)
    for mm in ms:
        srv.submit(mm, 3)
    srv.drain()
    assert srv.stats()["mean_batch"] > 1.0
    srv.close()
    for mm in ms:
        assert np.array_equal(mm.read_state()[0], res[2])
        mm.close()
    c2.close()


def test_budget_refuses(vh):
    say("[budget]")
    p = synth.problem_by_name("box")
    c = vh.Context(0, hbm_budget=4096)
    m = vh.Mesh(c, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, 10)
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(4)
    assert ei.value.code == vh.VH_ENOMEM
    assert c.hbm_in_use() == 0
    m.close()
    c.close()


def test_graph_replay_equals_direct_launches(vh, ctx):
    """The frame replayed as a HIP graph is bitwise equal to direct launches,
    on every replay."""
    import os
    say("[graph vs direct]")
    p = synth.problem_by_name("shell_small")
    a = make_mesh(vh, ctx, p)
    os.environ["VHPD_NO_GRAPH"] = "1"
    try:
        b = make_mesh(vh, ctx, p)
    finally:
        del os.environ["VHPD_NO_GRAPH"]
    for _ in range(4):
        a.step(1)
        b.step(1)
        xa, va = a.read_state()
        xb, vb = b.read_state()
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    a.close()
    b.close()


def test_full_shell_matches_oracle(vh, ctx):
    """The 390,400-tet shell with 128 subdomains (the benchmark configuration):
    the first frame from rest and one lock-step frame from the oracle's state,
    each within 1e-5 relative L2 of the FP64 oracle."""
    say("[full shell] building")
    p = synth.problem_by_name("shell")
    m = make_mesh(vh, ctx, p)
    say("[full shell] oracle setup")
    sim = oracle.OracleSim.from_problem(p)
    x0, v0 = p.initial_state()
    m.step(1)
    xg, _ = m.read_state()
    say("[full shell] oracle frame 1")
    x1, v1 = sim.step(x0, v0)
    e1 = rel_l2(xg, x1)
    say(f"   frame 1: rel L2 {e1:.3e}, displacement-relative {rel_disp(xg, x1, p.X):.3e}")
    assert e1 <= 1e-5
    m.write_state(x1, v1)
    m.step(1)
    xg2, _ = m.read_state()
    say("[full shell] oracle frame 2")
    x2, _ = sim.step(x1, v1)
    e2 = rel_l2(xg2, x2)
    say(f"   frame 2 (lock-step): rel L2 {e2:.3e}, displacement-relative {rel_disp(xg2, x2, p.X):.3e}")
    assert e2 <= 1e-5
    m.close()
