"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: positions within 1e-5 relative L2 per step (FP32 bulk arithmetic);
per-kernel tolerances follow from FP32 rounding of O(1) quantities (the
deformation gradient, singular values) scaled by the element weights."""

import dataclasses

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


def _stress_scale(S, s):
    """How much FP32 rounding of F moves the residual stress U diag(d) W^T per
    unit weight: the rotation's sensitivity grows like 2 / (sigma_i + sigma_j),
    and the volume projection's like the divided difference
    |s_i - s_j| / |sigma_i - sigma_j| (bounded on the + branch, large where a
    clamp or a minus-root axis separates two nearly equal singular values)."""
    big = np.maximum(1.0, np.abs(S).max(axis=1))
    rot = np.ones(len(S))
    dd = np.ones(len(S))
    for i, j in ((0, 1), (0, 2), (1, 2)):
        rot = np.maximum(rot, 2.0 / np.maximum(np.abs(S[:, i] + S[:, j]), 1e-30))
        dd = np.maximum(dd, np.abs(s[:, i] - s[:, j]) / np.maximum(np.abs(S[:, i] - S[:, j]), 1e-30))
    return big * rot * dd


def _check_projection(S, s_dev, tol=3e-6):
    """The device's projected singular values s_dev (Eq. vol_pre with the clamp
    of Sec. 7.1) against the FP64 oracle's projection of the same sigma S.

    The distance |s - sigma| of the nearest point is unique; the point is not
    where two stationary points lie at (nearly) equal distance, as for
    sigma = (c, c, c) with c > 2, whose mixed-branch candidates are each other's
    images under an axis swap.  So: the distance must agree everywhere; the
    point must agree where the device's point is not an equally near
    alternative; and every device point must be feasible (prod s = 1,
    s >= 0.01) and stationary (s_i (s_i - sigma_i) equal over the axes the
    clamp left free).  Returns the oracle's regime counts and the mask of
    elements whose point was compared directly."""
    s_ref, info = oracle.proj_sl3(S)
    big = np.maximum(1.0, np.abs(S).max(axis=1))
    d_dev = np.linalg.norm(s_dev - S, axis=1)
    d_ref = np.linalg.norm(s_ref - S, axis=1)
    assert (np.abs(d_dev - d_ref) / big).max() < tol, (np.abs(d_dev - d_ref) / big).max()
    assert np.abs(np.log(s_dev).sum(axis=1)).max() < 5 * tol
    assert s_dev.min() >= 0.01 * (1 - 1e-6)
    free = s_dev > 0.01 * (1 + 1e-5)
    mu = s_dev * (s_dev - S)
    for e in np.nonzero(free.sum(axis=1) >= 2)[0]:
        m = mu[e, free[e]]
        assert np.ptp(m) <= 20 * tol * big[e] ** 2, (e, S[e], s_dev[e], m)
    same = (np.abs(s_dev - s_ref) / big[:, None]).max(axis=1) < tol
    return info, same


@pytest.mark.parametrize("amp", [0.01, 0.02])
def test_local_step_large_strain_and_inverted(vh, ctx, amp):
    """Singular values from about 0.25 to 3.7, and (amp 0.02) inverted elements."""
    say(f"[local] large strain amp={amp}")
    p = synth.problem_by_name("box")
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    x = deformed(p, amp=amp, seed=1)
    m.regime_counts(reset=True)
    T, sig, s = m.debug_local_step(x)
    counts = m.regime_counts()
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    S = loc["sigma"]
    big = np.maximum(1.0, np.abs(S).max(axis=1))[:, None]
    assert (np.abs(sig - S) / big).max() < 4e-6
    info, same = _check_projection(sig, s)
    n_inv = int((S[:, 2] < 0).sum())
    say(f"[local] amp={amp}: {same.sum()} of {len(S)} points compared directly, {n_inv} inverted, "
        f"oracle {info}, device {counts}")
    assert same.mean() > 0.99
    for k in ("clamped", "inverted", "det_ge2", "squash", "no_plus_root"):
        assert abs(counts[k] - info[k]) <= 1, (k, counts, info)
    if amp >= 0.02:
        assert counts["inverted"] > 0 and counts["det_ge2"] > 0
    Tref = loc["P"] - (sim.w_s + sim.w_v)[:, None, None] * loc["F"]
    w = (sim.w_s + sim.w_v)[:, None, None]
    err = (np.abs(T - Tref) / w).max(axis=(1, 2))
    scale = _stress_scale(S, s)
    keep = same & np.all(np.abs(s - loc["s"]) / big < 4e-6, axis=1)
    assert (err[keep] / scale[keep]).max() < 2e-5, (err[keep] / scale[keep]).max()
    m.close()


# extreme affine deformations of a small box about its centre (plus seeded
# noise): two axes stretched 12x and the third flattened (every element
# clamped, then its pair re-solved on s1 s2 = 100), the same with the third
# axis inverted, a stretch about x2 (det F = 6.8: no + branch root, mixed
# points nearest) and (6, 3, 0.5) (det F = 9)
REGIME_CASES = {"flat": ((12.0, 12.0, 0.001), 2e-5), "flat_inverted": ((12.0, 12.0, -0.002), 2e-5),
                "stretch2": ((2.0, 1.9, 1.8), 1e-3), "mixed": ((6.0, 3.0, 0.5), 1e-3)}


@pytest.mark.parametrize("case", list(REGIME_CASES))
def test_local_step_projection_regimes(vh, ctx, case):
    """Clamped, inverted-and-clamped and det F >= 2 elements: the projection of
    Eq. vol_pre with Sec. 7.1's clamp and freeze, against the FP64 oracle, and
    the regime counters against the oracle's counts."""
    diag, noise = REGIME_CASES[case]
    say(f"[local regimes] {case}")
    p = synth.make_box_problem(seed=11, nx=4, ny=4, nz=2, n_subdomains=2, name="box_small")
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    c = p.X.mean(axis=0)
    rng = np.random.default_rng(5)
    x = (p.X - c) * np.asarray(diag) + c + noise * 0.01 * rng.standard_normal(p.X.shape)
    x[p.pinned.astype(bool)] = p.X[p.pinned.astype(bool)]      # the library keeps pinned rows at rest
    m.regime_counts(reset=True)
    T, sig, s = m.debug_local_step(x)
    counts = m.regime_counts()
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    S = loc["sigma"]
    big = np.maximum(1.0, np.abs(S).max(axis=1))[:, None]
    assert (np.abs(sig - S) / big).max() < 4e-6
    info, same = _check_projection(sig, s)
    say(f"[local regimes] {case}: {same.sum()} of {len(S)} points compared directly; oracle {loc['info']}, "
        f"device {counts}")
    for k in ("clamped", "inverted", "det_ge2", "squash", "no_plus_root"):
        assert abs(counts[k] - info[k]) <= 1, (k, counts, info)
    # the elements of the pinned row's layer are distorted differently
    if case.startswith("flat"):
        assert counts["clamped"] >= 0.8 * p.nt
    else:
        assert counts["det_ge2"] >= 0.7 * p.nt and counts["squash"] >= 0.7 * p.nt
    assert same.mean() >= 0.95
    # residual stress where the device's point is the oracle's
    keep = same & np.all(np.abs(s - loc["s"]) / big < 4e-6, axis=1)
    assert keep.sum() > 0
    Tref = loc["P"] - (sim.w_s + sim.w_v)[:, None, None] * loc["F"]
    w = (sim.w_s + sim.w_v)[:, None, None]
    err = (np.abs(T - Tref) / w).max(axis=(1, 2))
    scale = _stress_scale(S, s)
    assert (err[keep] / scale[keep]).max() < 2e-5, (err[keep] / scale[keep]).max()
    m.close()


def test_step_from_clamped_state_matches_oracle(vh, ctx):
    """One frame of the PD step (10 iterations) from a flattened state in which
    every element starts clamped: positions against the FP64 oracle, and the
    clamped evaluations counted by both."""
    say("[step regimes] flattened start")
    p = synth.make_box_problem(seed=12, nx=3, ny=3, nz=2, n_subdomains=2, name="box_tiny")
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    c = p.X.mean(axis=0)
    x0 = (p.X - c) * np.array([12.0, 12.0, 0.001]) + c
    x0[p.pinned.astype(bool)] = p.X[p.pinned.astype(bool)]
    v0 = np.zeros_like(x0)
    m.write_state(x0, v0)
    m.regime_counts(reset=True)
    m.step(1)
    xg, _ = m.read_state()
    counts = m.regime_counts()
    xo, _ = sim.step(x0, v0)
    info = sim.last_info
    e = rel_l2(xg, xo)
    say(f"[step regimes] rel L2 {e:.3e}, device {counts}, oracle {info}")
    assert counts["clamped"] > 0
    assert abs(counts["clamped"] - info["clamped"]) <= 2
    assert e <= 1e-5


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


@pytest.mark.parametrize("name,D", [("box", 4), ("box", 2), ("box", 1), ("shell_small", 8), ("slab", 8)])
def test_residual_in_solve_is_bitwise_standalone(vh, ctx, name, D):
    """The PD iterations form the residual inside the interior forward solve
    (each subdomain's workgroup its interior rows and a share of ceil(n_G / D)
    of the n_G interface rows, the last share shorter unless D divides n_G;
    D = 1 has no interface): bit for bit the residual of the gather's own
    launch, and within FP32 rounding of the oracle."""
    say(f"[residual in solve] {name} D={D}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p, n_subdomains=D)
    x = deformed(p, amp=2e-3, seed=4)
    y = deformed(p, amp=1e-3, seed=5)
    r_own = m.debug_residual(x, y)
    m.debug_residual(p.X, p.X)                    # another r in between
    r_in = m.debug_residual(x, y, in_solve=True)
    say(f"  interface rows {m.info()['n_interface']}, subdomains {D}")
    assert np.array_equal(r_in, r_own)
    sim = oracle.OracleSim.from_problem(p)
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    rref = sim.rhs(y, loc["P"]) - sim.L_ff @ x[sim.free]
    assert np.linalg.norm(r_in[sim.free] - rref) <= 1e-5 * np.linalg.norm(rref)
    m.close()


@pytest.mark.parametrize("name", ["box", "shell_small", "slab"])
def test_scatter_matches_element_colouring(vh, ctx, name):
    """The atomic-free scatter (per-workgroup LDS partial sums, then a gather
    per vertex) against the element-colouring scatter: the same corner forces
    summed in another order, so equal to FP32 summation rounding; both match
    the oracle's elastic forces."""
    say(f"[scatter colouring] {name}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p)
    sim = oracle.OracleSim.from_problem(p)
    x = deformed(p, amp=2e-3, seed=6)
    f_col, ncol = m.debug_scatter_colored(x)
    f_part = m.debug_residual(x, x)          # y = x: the inertial term vanishes
    scale = np.abs(f_part).max()
    assert 4 <= ncol <= 64
    assert np.abs(f_col - f_part).max() <= 1e-5 * scale
    assert np.all(f_col[p.pinned.astype(bool)] == 0)
    loc = oracle.local_step(x, sim.tets, sim.grads, sim.w_s, sim.w_v)
    fref = sim.rhs(x, loc["P"]) - sim.L_ff @ x[sim.free]   # residual at y = x
    assert np.linalg.norm(f_col[sim.free] - fref) <= 1e-5 * np.linalg.norm(fref)
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
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(4, 0, 1)                              # no such precision mode
    assert ei.value.code == vh.VH_EINVAL
    # M / dt^2 overflows: a pivot that is not a positive finite number
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, 1e-160, 10)
    with pytest.raises(vh.VHError) as ei:
        m.prefactor(4)
    assert ei.value.code == vh.VH_ENOTSPD
    with pytest.raises(vh.VHError) as ei:
        ctx.set_config(use_graphs=2)
    assert ei.value.code == vh.VH_EINVAL
    m.close()


@pytest.mark.parametrize("name,D", [("box", None), ("box", 1), ("shell_small", None)])
def test_refactor_matches_prefactor(vh, ctx, name, D):
    """vh_mesh_refactor with new stiffness gives the factor a fresh prefactor
    with that stiffness gives: solves and frames bitwise equal, also through
    the frame graph captured before the refactor; the state is kept.  (D = 1:
    one subdomain, no interface supernodes.)"""
    say(f"[refactor] {name} D={D}")
    p = synth.problem_by_name(name)
    if D is not None:
        p = dataclasses.replace(p, n_subdomains=D)
    rng = np.random.default_rng(13)
    gs2 = p.gamma_s * rng.uniform(0.5, 2.0, p.nt)
    gv2 = p.gamma_v * rng.uniform(0.5, 2.0, p.nt)
    a = make_mesh(vh, ctx, p)
    a.step(2)                                   # captures the frame graph
    xa, va = a.read_state()
    a.refactor(gs2, gv2)
    xk, vk = a.read_state()
    assert np.array_equal(xk, xa) and np.array_equal(vk, va)
    b = make_mesh(vh, ctx, p, gamma_s=gs2, gamma_v=gv2)
    rhs = rng.standard_normal((p.nv, 3))
    assert np.array_equal(a.debug_solve(rhs), b.debug_solve(rhs))
    a.write_state(*p.initial_state())
    a.step(3)
    b.step(3)
    xa, va = a.read_state()
    xb, vb = b.read_state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    sim = oracle.OracleSim.from_problem(dataclasses.replace(p, gamma_s=gs2, gamma_v=gv2))
    x, v = p.initial_state()
    for _ in range(3):
        x, v = sim.step(x, v)
    assert rel_l2(xa, x) <= 1e-5
    a.close()
    b.close()


@pytest.mark.parametrize("name,D", [("box", 4), ("shell_small", 8), ("slab", 8)])
def test_device_interface_factor_matches_host(vh, ctx, name, D):
    """The interface supernodes factored on the device (rocSOLVER / rocBLAS)
    against the host's FP64 multifrontal factorization of the same plan (the
    test library builds it with the host path): every stored value of the
    blocks the interface phases read, Ti, W_B and the root's Ti^T Ti."""
    import ctypes
    from tests.host import build as hbuild
    say(f"[device factor] {name} D={D}")
    p = synth.problem_by_name(name)
    m = make_mesh(vh, ctx, p, n_subdomains=D)
    dev = m.debug_interface_factor()
    m.close()
    hl = ctypes.CDLL(hbuild.ensure())
    vp, ci = ctypes.c_void_p, ctypes.c_int
    hl.vhp_build.restype = vp
    hl.vhp_build.argtypes = [vp, ci, vp, ci, vp, vp, vp, vp, vp, ctypes.c_double, ci, ci, ci, ci, vp, vp, ci]
    hl.vhp_dvals.restype = ctypes.c_longlong
    hl.vhp_dvals.argtypes = [vp, vp]
    hl.vhp_free.argtypes = [vp]
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    keep = [a(p.X, np.float64), a(p.tets, np.int32), a(p.gamma_s, np.float64), a(p.gamma_v, np.float64),
            a(p.mass, np.float64), a(p.pinned, np.uint8), a(p.gravity, np.float64)]
    rc = ctypes.c_int(0)
    msg = ctypes.create_string_buffer(256)
    h = hl.vhp_build(keep[0].ctypes.data, p.nv, keep[1].ctypes.data, p.nt, keep[2].ctypes.data,
                     keep[3].ctypes.data, keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data,
                     p.dt, p.pd_iters, D, 0, 32, ctypes.byref(rc), msg, 256)
    assert rc.value == 0, msg.value.decode()
    try:
        n = hl.vhp_dvals(h, None)
        host = np.empty(n)
        hl.vhp_dvals(h, host.ctypes.data)
    finally:
        hl.vhp_free(h)
    assert dev.shape == host.shape and dev.size > 0
    err = np.abs(dev - host).max() / np.abs(host).max()
    say(f"[device factor] {name}: {dev.size} values, max |device - host| / max |host| = {err:.2e}")
    assert err <= 1e-13


def test_refactor_misuse(vh, ctx):
    say("[refactor misuse]")
    p = synth.problem_by_name("box")
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, 10)
    with pytest.raises(vh.VHError) as ei:
        m.refactor(p.gamma_s, p.gamma_v)           # not prefactored
    assert ei.value.code == vh.VH_ESTATE
    m.prefactor(4)
    g = p.gamma_s.copy()
    g[7] = np.inf
    with pytest.raises(vh.VHError) as ei:
        m.refactor(g, p.gamma_v)
    assert ei.value.code == vh.VH_EINVAL
    m.refactor(p.gamma_s, p.gamma_v)               # still usable
    m.step(1)
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


@pytest.mark.parametrize("name,D", [("box", 4), ("box", 1), ("shell_small", 8)])
def test_chunk_descriptors_from_global_memory(vh, ctx, name, D):
    """The interior solves read the descriptors of program chunks past their
    LDS table from global memory.  With a table of one entry every chunk
    after a subdomain's first takes that path: the solve and three frames are
    bitwise those of the full table, and the solve is exact."""
    say(f"[descriptor table] {name} D={D}")
    p = synth.problem_by_name(name)
    rhs = np.random.default_rng(7).standard_normal((p.nv, 3))
    res = []
    for tab in (64, 1):
        c = vh.Context(0)
        c.set_config(interior_desc_table=tab)
        assert c.config()["interior_desc_table"] == tab
        m = make_mesh(vh, c, p, n_subdomains=D)
        d = m.debug_solve(rhs)
        m.step(3)
        x, v = m.read_state()
        res.append((d, x, v))
        m.close()
        c.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    sim = oracle.OracleSim.from_problem(p)
    xe = sim._solve(rhs[sim.free])
    assert np.linalg.norm(res[1][0][sim.free] - xe) <= 5e-7 * np.linalg.norm(xe)
    for bad in (0, 65):
        with pytest.raises(vh.VHError) as ei:
            ctx.set_config(interior_desc_table=bad)
        assert ei.value.code == vh.VH_EINVAL


def test_graph_replay_equals_direct_launches(vh, ctx):
    """The frame replayed as a HIP graph is bitwise equal to direct launches,
    on every replay."""
    say("[graph vs direct]")
    p = synth.problem_by_name("shell_small")
    a = make_mesh(vh, ctx, p)
    ctx_direct = vh.Context(0)
    ctx_direct.set_config(use_graphs=0)
    assert ctx_direct.config()["use_graphs"] == 0 and ctx.config()["use_graphs"] == 1
    b = make_mesh(vh, ctx_direct, p)
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
