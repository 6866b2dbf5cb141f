"""Gradient of a trajectory loss with respect to gamma_s on the 20,000-tet slab:
the GPU adjoint against the FP64 oracle adjoint and central differences.

Loss: 1/2 ||x_30(gamma_s) - x_30(gamma_s_hidden)||^2 over the free vertices,
evaluated at gamma_s = 1e4 everywhere; the hidden stiffness is the slab's
seeded log-normal field; 30 frames of 10 iterations, checkpoints every 5.

    python tests/adjoint_check.py gpu --out G.npz      (GPU: gradient, timings)
    python tests/adjoint_check.py oracle --out O.npz   (host: oracle adjoint + FD)
    python tests/adjoint_check.py compare O.npz G.npz

Not collected by pytest (a measurement tool, not a test).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

FRAMES, EVERY, GS0 = 30, 5, 1e4


def fd_elements(p, n, seed=5):
    return np.sort(np.random.Generator(np.random.PCG64(seed)).choice(p.nt, n, replace=False))


def run_gpu(args):
    import torch
    from paper_2405_12484_amd import vhpd
    import synth
    p = synth.problem_by_name("slab")
    ctx = vhpd.Context(0)
    m = vhpd.Mesh(ctx, p.X, p.tets)
    x0, v0 = p.initial_state()
    # target: the hidden stiffness's trajectory
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains)
    xt = m.adjoint_forward(x0, v0, FRAMES, EVERY)
    gs0 = np.full(p.nt, GS0)
    m.set_params(gs0, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    t0 = time.perf_counter()
    m.prefactor(p.n_subdomains)
    t1 = time.perf_counter()
    xf = m.adjoint_forward(x0, v0, FRAMES, EVERY)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    d = xf - xt
    d[p.pinned.astype(bool)] = 0.0
    g = m.adjoint_backward(d)
    t3 = time.perf_counter()
    out = {"prefactor_s": t1 - t0, "forward_s": t2 - t1, "backward_s": t3 - t2,
           "loss": 0.5 * float((d * d).sum())}
    np.savez(args.out, grad=g, xt=xt, xf=xf, **out)
    print(json.dumps(out), flush=True)


def run_oracle(args):
    import oracle
    import synth
    from oracle.adjoint import loss_and_grad, loss_only
    p = synth.problem_by_name("slab")
    sim = oracle.OracleSim(p.X, p.tets, p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    x0, v0 = p.initial_state()
    xt, _ = sim.run(x0, v0, FRAMES)
    gs0 = np.full(p.nt, GS0)
    t0 = time.perf_counter()
    loss, g = loss_and_grad(p, gs0, xt, FRAMES)
    print(f"oracle adjoint {time.perf_counter() - t0:.0f} s, loss {loss:.6e}", flush=True)
    els = fd_elements(p, args.n_fd)
    fd = {}
    for rel in args.fd_steps:
        vals = []
        for e in els:
            h = rel * GS0
            gp = gs0.copy()
            gp[e] += h
            gm = gs0.copy()
            gm[e] -= h
            vals.append((loss_only(p, gp, xt, FRAMES) - loss_only(p, gm, xt, FRAMES)) / (2 * h))
            print(f"fd rel {rel:g} element {e}: {vals[-1]:.6e} (adjoint {g[e]:.6e})", flush=True)
        fd[f"fd_{rel:g}"] = np.array(vals)
    np.savez(args.out, grad=g, loss=loss, elements=els, **fd)


def compare(args):
    o = np.load(args.files[0])
    g = np.load(args.files[1])
    go, gg = o["grad"], g["grad"]
    res = {"rel_l2_gpu_vs_oracle_adjoint": float(np.linalg.norm(gg - go) / np.linalg.norm(go)),
           "loss_oracle": float(o["loss"]), "loss_gpu": float(g["loss"]),
           "gpu_forward_s": float(g["forward_s"]), "gpu_backward_s": float(g["backward_s"])}
    els = o["elements"]
    for k in o.files:
        if k.startswith("fd_"):
            fd = o[k]
            res[f"max_rel_err_oracle_adjoint_vs_{k}"] = float(np.abs(go[els] - fd).max() / np.abs(fd).max())
            res[f"max_rel_err_gpu_vs_{k}"] = float(np.abs(gg[els] - fd).max() / np.abs(fd).max())
    print(json.dumps(res, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["gpu", "oracle", "compare"])
    ap.add_argument("files", nargs="*")
    ap.add_argument("--out", default="")
    ap.add_argument("--n-fd", type=int, default=32)
    ap.add_argument("--fd-steps", type=float, nargs="*", default=[1e-6, 1e-4])
    args = ap.parse_args()
    {"gpu": run_gpu, "oracle": run_oracle, "compare": compare}[args.mode](args)


if __name__ == "__main__":
    main()
