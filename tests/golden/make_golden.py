"""Writes the stored expected values under tests/golden/ from the FP64 oracle
(oracle/) and the seeded inputs (synth/) only.

    python tests/golden/make_golden.py              (box frames, projections)
    python tests/golden/make_golden.py shell        (about an hour of host time)
    python tests/golden/make_golden.py slab --jobs 4

shell_oracle_*.npy: the 390,400-tet shell (seed 2, 128 subdomains, dt = 1/150,
10 PD iterations per frame) from rest, oracle exact solve: positions x after
frames 10 and 150, and (x, v) after frame 149, float64 [nv][3] in the
generator's vertex order.
slab_*: the 20,000-tet slab (40x25x4 hexes, seed 3): target positions
x_30(gamma_s_hidden) after 30 frames (slab_oracle_target_x30.npy), the oracle
adjoint gradient of 1/2 ||x_30(gamma_s) - target||^2 over the free vertices at
gamma_s = 1e4 everywhere (slab_oracle_grad.npy, [nt]), and central differences
of that loss on 32 seeded elements (seed 5) at relative steps 1e-6 and 1e-4
(slab_fd.txt).

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
    # clamp (Sec. 7.1): s_3 below 0.01 is frozen there and the pair re-solved;
    # twice-clamped; inverted and clamped; det F >= 2 with a squashed axis
    clamped = np.array([[50.0, 40.0, 1e-4], [30.0, 12.0, 2e-3], [25.0, 18.0, -1e-3], [1e5, 1e-3, 1e-3],
                        [10.0, 10.0, 10.0], [6.0, 3.0, 0.5], [4.0, 3.5, 3.0]])
    return np.vstack([sig, fixed, clamped])


def write_box():
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


def write_sl3():
    sig = sl3_inputs()
    s, _ = oracle.proj_sl3(sig)
    with open(os.path.join(HERE, "sl3_projection.txt"), "w") as fh:
        fh.write("# Nearest volume-preserving singular values (Eq. vol_pre) from oracle.proj_sl3 (FP64):\n")
        fh.write("# the + branch root of s_i (s_i - sigma_i) = mu with s1 s2 s3 = 1, the nearest\n")
        fh.write("# stationary point where several exist; a component below 0.01 is clamped to 0.01,\n")
        fh.write("# frozen, and the others re-solved on the remaining product.  Written by\n")
        fh.write("# tests/golden/make_golden.py.  Columns: sigma1 sigma2 sigma3 s1 s2 s3.\n")
        for a, b in zip(sig, s):
            fh.write(" ".join(f"{t:.17g}" for t in (*a, *b)) + "\n")


SHELL_FRAMES = (10, 149, 150)
SLAB_FRAMES, SLAB_GS0, SLAB_FD_STEPS = 30, 1e4, (1e-6, 1e-4)


def write_shell():
    import time
    p = synth.problem_by_name("shell")
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    t0 = time.perf_counter()
    counts = {}
    for f in range(1, max(SHELL_FRAMES) + 1):
        x, v = sim.step(x, v)
        for k, c in sim.last_info.items():
            counts[k] = counts.get(k, 0) + c
        if f in SHELL_FRAMES:
            np.save(os.path.join(HERE, f"shell_oracle_x_f{f:03d}.npy"), x)
            if f + 1 in SHELL_FRAMES:
                np.save(os.path.join(HERE, f"shell_oracle_v_f{f:03d}.npy"), v)
        print(f"shell frame {f}: {time.perf_counter() - t0:.0f} s {counts}", flush=True)


def slab_fd_elements(p, n=32, seed=5):
    return np.sort(np.random.Generator(np.random.PCG64(seed)).choice(p.nt, n, replace=False))


def _slab_loss(args):
    from oracle.adjoint import loss_only
    e, rel, sign, target = args
    p = synth.problem_by_name("slab")
    gs = np.full(p.nt, SLAB_GS0)
    gs[e] += sign * rel * SLAB_GS0
    return loss_only(p, gs, target, SLAB_FRAMES)


def write_slab(jobs):
    import multiprocessing as mp
    from oracle.adjoint import loss_and_grad
    p = synth.problem_by_name("slab")
    sim = oracle.OracleSim.from_problem(p)
    x0, v0 = p.initial_state()
    target, _ = sim.run(x0, v0, SLAB_FRAMES)
    np.save(os.path.join(HERE, "slab_oracle_target_x30.npy"), target)
    els = slab_fd_elements(p)
    tasks = [(int(e), rel, sg, target) for rel in SLAB_FD_STEPS for e in els for sg in (1.0, -1.0)]
    with mp.get_context("fork").Pool(jobs) as pool:
        res = pool.map_async(_slab_loss, tasks)
        loss, g = loss_and_grad(p, np.full(p.nt, SLAB_GS0), target, SLAB_FRAMES)
        np.save(os.path.join(HERE, "slab_oracle_grad.npy"), g)
        print(f"slab: loss {loss:.9e}, adjoint done", flush=True)
        vals = res.get()
    with open(os.path.join(HERE, "slab_fd.txt"), "w") as fh:
        fh.write("# Central differences of the slab loss 1/2 ||x_30(gamma_s) - x_30(gamma_s_hidden)||^2\n")
        fh.write("# (FP64 oracle, exact solve, 30 frames of 10 PD iterations from rest) at gamma_s = 1e4,\n")
        fh.write(f"# loss {loss:.17g}.  Written by tests/golden/make_golden.py.\n")
        fh.write("# Columns: element relative_step fd_gradient oracle_adjoint_gradient.\n")
        i = 0
        for rel in SLAB_FD_STEPS:
            for e in els:
                lp, lm = vals[i], vals[i + 1]
                i += 2
                h = rel * SLAB_GS0
                fh.write(f"{e} {rel:g} {(lp - lm) / (2 * h):.17g} {g[e]:.17g}\n")


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("targets", nargs="*", default=["box", "sl3"])
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    for t in a.targets:
        {"box": write_box, "sl3": write_sl3, "shell": write_shell,
         "slab": lambda: write_slab(a.jobs)}[t]()


if __name__ == "__main__":
    main()
