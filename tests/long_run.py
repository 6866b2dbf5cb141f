"""Long free-running trajectories: the GPU path against the FP64 oracle.

The oracle side runs on the host (minutes per hundred frames of the 390K-tet
shell); the GPU side runs through the C ABI; both save the positions at the
same frames to .npz files, and `compare` prints the relative L2 errors.

    python tests/long_run.py oracle --workload shell --frames 150 --out O.npz
    python tests/long_run.py gpu --workload shell --frames 150 --refine 2 --out G.npz
    python tests/long_run.py compare O.npz G.npz

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


def checkpoints(frames):
    ks = sorted({1, 10, 50, 100, frames} | set(range(25, frames + 1, 25)))
    return [k for k in ks if k <= frames]


def run_oracle(args):
    import oracle
    import synth
    p = synth.problem_by_name(args.workload)
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    saved = {}
    ks = set(checkpoints(args.frames))
    t0 = time.perf_counter()
    for f in range(1, args.frames + 1):
        x, v = sim.step(x, v)
        if f in ks:
            saved[f"x{f}"] = x.copy()
            print(f"oracle frame {f}: {time.perf_counter() - t0:.0f} s", flush=True)
    np.savez(args.out, frames=np.array(sorted(ks)), **saved)


def run_gpu(args):
    import torch
    from paper_2405_12484_amd import vhpd
    import synth
    p = synth.problem_by_name(args.workload)
    ctx = vhpd.Context(0)
    m = vhpd.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains, args.refine)
    stream = torch.cuda.current_stream()
    ks = checkpoints(args.frames)
    saved = {}
    done = 0
    ms = 0.0
    for k in ks:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.step(k - done, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done = k
        x, _ = m.read_state(stream)
        saved[f"x{k}"] = x
        print(f"gpu frame {k}", flush=True)
    np.savez(args.out, frames=np.array(ks), ms_per_frame=ms / args.frames, refine=args.refine, **saved)
    print(json.dumps({"ms_per_frame": ms / args.frames, "refine": args.refine}), flush=True)
    m.close()
    ctx.close()


def compare(args):
    a = np.load(args.files[0])
    b = np.load(args.files[1])
    import synth
    X = synth.problem_by_name(args.workload).X
    out = {}
    for k in a["frames"]:
        if f"x{k}" not in b:
            continue
        xa, xb = a[f"x{k}"], b[f"x{k}"]
        out[int(k)] = {"positions": float(np.linalg.norm(xb - xa) / np.linalg.norm(xa)),
                       "displacements": float(np.linalg.norm(xb - xa) / np.linalg.norm(xa - X))}
    extra = {k: float(b[k]) for k in ("ms_per_frame", "refine") if k in b}
    print(json.dumps({"rel_l2": out, **extra}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["oracle", "gpu", "compare"])
    ap.add_argument("files", nargs="*")
    ap.add_argument("--workload", default="shell")
    ap.add_argument("--frames", type=int, default=150)
    ap.add_argument("--refine", type=int, default=0)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    {"oracle": run_oracle, "gpu": run_gpu, "compare": compare}[args.mode](args)


if __name__ == "__main__":
    main()
