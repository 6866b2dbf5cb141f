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
