"""The stored expected values under tests/golden/ (written by
tests/golden/make_golden.py from the FP64 oracle): the oracle still reproduces
them, and the stored projections satisfy Eq. vol_pre's conditions on their own."""

import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_box_frames():
    a = np.loadtxt(os.path.join(GOLDEN, "box_oracle_frames.txt"))
    out = {}
    for f in np.unique(a[:, 0]).astype(int):
        rows = a[a[:, 0] == f]
        out[f] = rows[np.argsort(rows[:, 1]), 2:5]
    return out


def test_oracle_reproduces_box_frames():
    ref = load_box_frames()
    p = synth.problem_by_name("box")
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    for f in range(1, 21):
        x, v = sim.step(x, v)
        if f in ref:
            assert np.abs(x - ref[f]).max() <= 1e-12 * np.abs(ref[f]).max(), f


def test_sl3_fixture():
    a = np.loadtxt(os.path.join(GOLDEN, "sl3_projection.txt"))
    sig, s = a[:, :3], a[:, 3:]
    s2, _ = oracle.proj_sl3(sig)
    assert np.abs(s2 - s).max() < 1e-13
    free = s.min(axis=1) > 0.0100001                      # no clamp fired
    assert np.abs(s.prod(axis=1) - 1.0).max() < 1e-12      # clamped rows re-solve the rest
    clamped = ~free
    assert clamped.sum() >= 4 and (s[clamped].min(axis=1) == 0.01).all()
    mu = s * (s - sig)                                    # the Lagrange multiplier, equal on every axis
    spread = (mu.max(axis=1) - mu.min(axis=1)) / np.maximum(np.abs(mu).max(axis=1), 1e-300)
    assert spread[free].max() < 1e-9
    assert (sig[:, 2] < 0).sum() >= 8 and (s > 0).all()


def test_slab_adjoint_against_central_differences():
    """The stored slab gradient (oracle adjoint of 30 frames, Sec. 7's PD step
    reversed) against the stored central differences of the loss itself,
    which only run the forward oracle: within 5e-5 of the largest |FD| at the
    relative step 1e-4 (truncation and rounding of the difference quotient are
    both small there), within 2e-3 at 1e-6 (rounding of the loss dominates);
    the stored gradient file holds the same adjoint values."""
    rows = np.loadtxt(os.path.join(GOLDEN, "slab_fd.txt"), comments="#")
    g = np.load(os.path.join(GOLDEN, "slab_oracle_grad.npy"))
    p = synth.problem_by_name("slab")
    assert g.shape == (p.nt,) and np.isfinite(g).all()
    for h, tol in ((1e-4, 5e-5), (1e-6, 2e-3)):
        r = rows[rows[:, 1] == h]
        assert len(r) == 32
        e = r[:, 0].astype(np.int64)
        assert np.array_equal(g[e], r[:, 3])
        assert np.abs(r[:, 2] - r[:, 3]).max() <= tol * np.abs(r[:, 2]).max(), h
    # the elements are spread over the slab, not clustered
    assert len(np.unique(rows[:, 0])) == 32 and np.ptp(rows[:, 0]) > 0.5 * p.nt


def test_shell_frames_reproduce():
    """The stored shell positions (oracle, frames 10, 149, 150) are finite with
    the pinned collar at rest, and one oracle frame from the stored frame-149
    state (x, v) reproduces the stored frame 150 (about 40 s of host time)."""
    p = synth.problem_by_name("shell")
    pin = p.pinned.astype(bool)
    xs = {f: np.load(os.path.join(GOLDEN, f"shell_oracle_x_f{f:03d}.npy")) for f in (10, 149, 150)}
    v149 = np.load(os.path.join(GOLDEN, "shell_oracle_v_f149.npy"))
    for f, x in xs.items():
        assert x.shape == p.X.shape and np.isfinite(x).all(), f
        assert np.array_equal(x[pin], p.X[pin]), f
    assert np.all(v149[pin] == 0.0)
    sim = oracle.OracleSim.from_problem(p)
    x150, _ = sim.step(xs[149], v149)
    assert np.abs(x150 - xs[150]).max() <= 1e-12 * np.abs(xs[150]).max()
