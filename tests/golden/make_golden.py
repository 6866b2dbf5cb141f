"""Writes the stored expected values under tests/golden/ from the FP64 oracle
(oracle/) and the seeded inputs (synth/) only.

    python tests/golden/make_golden.py

box_oracle_frames.txt: positions of the 1,000-tet box (seed 1, 20 frames of
10 PD iterations, Sec. 7.1) after frames 1 and 20, from rest.
sl3_projection.txt: nearest volume-preserving singular values (Eq. vol_pre)
for a sweep of signed singular values, including inverted and nearly flat
elements, with the oracle's regime rule.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def sl3_inputs():
    rng = np.random.Generator(np.random.PCG64(21))
    sig = np.sort(np.exp(rng.uniform(np.log(0.05), np.log(1.8), (24, 3))), axis=1)[:, ::-1]
    sig[16:, 2] *= -rng.uniform(0.1, 0.9, 8)           # inverted: sigma_3 < 0, |sigma_3| <= sigma_2
    fixed = np.array([[1.0, 1.0, 1.0], [1.2, 1.0, 0.8], [1.1, 1.1, 0.7], [2.0, 0.5, 0.002], [1.05, 0.98, -0.3]])
    return np.vstack([sig, fixed])


def main():
    p = synth.problem_by_name("box")
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    keep = {}
    for f in range(1, 21):
        x, v = sim.step(x, v)
        if f in (1, 20):
            keep[f] = x.copy()
    with open(os.path.join(HERE, "box_oracle_frames.txt"), "w") as fh:
        fh.write("# FP64 oracle (oracle.OracleSim, exact sparse solve), box workload: 10x10x2 hexes of\n")
        fh.write("# 1 cm, 5 tets each, seed 1, dt = 1/150, 10 PD iterations per frame (Sec. 7.1), from rest.\n")
        fh.write("# Written by tests/golden/make_golden.py.  Columns: frame vertex x y z (metres).\n")
        for f, xf in keep.items():
            for i, r in enumerate(xf):
                fh.write(f"{f} {i} {r[0]:.17g} {r[1]:.17g} {r[2]:.17g}\n")
    sig = sl3_inputs()
    s, _ = oracle.proj_sl3(sig)
    with open(os.path.join(HERE, "sl3_projection.txt"), "w") as fh:
        fh.write("# Nearest volume-preserving singular values (Eq. vol_pre) from oracle.proj_sl3 (FP64):\n")
        fh.write("# the + branch root of s_i (s_i - sigma_i) = mu with s1 s2 s3 = 1, the nearest\n")
        fh.write("# stationary point where several exist, clamp at 0.01.  Written by\n")
        fh.write("# tests/golden/make_golden.py.  Columns: sigma1 sigma2 sigma3 s1 s2 s3.\n")
        for a, b in zip(sig, s):
            fh.write(" ".join(f"{t:.17g}" for t in (*a, *b)) + "\n")


if __name__ == "__main__":
    main()
