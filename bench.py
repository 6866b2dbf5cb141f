#!/usr/bin/env python
"""Benchmark of the projective-dynamics step on one MI355X.

Workload: the 390,400-tet cylindrical shell (118,080 vertices, 128
subdomains, dt = 1/150 s, 10 local/global iterations per frame; the stand-in at
the scale of the paper's 389K-tet sweater scene).  One "step" is one frame:
predictor, 10 x (local step, decomposed solve whose first launch gathers the
residual), velocity.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line with:
  * ms/frame: HIP events around K frames replayed as a captured graph;
  * the roofline of every kernel class and of the dominant one: algorithmic
    bytes (vh_mesh_get_info) / average launch-group time, from HIP events on
    the bench stream around each launch group inside K more frames; the same
    from back-to-back launches of one class ("isolated", data warm in cache);
    HBM traffic per launch from the committed rocprofv3 counter summary while
    the kernel source is unchanged (else null);
  * the FP64 oracle timed on a bounded sample on the host (cpu_baseline) and
    the relative L2 error of the first frame against it;
  * serving: 64 uneven garments, batched against sequential plain stepping
    (saturated, Poisson arrivals at several rates, a 1 GB HBM budget);
  * the discrete adjoint with respect to gamma_s on the 20,000-tet slab
    (30 frames, checkpoints every 5): forward and backward wall times, and the
    gradient's relative L2 error against the stored FP64 oracle adjoint;
  * the 150-frame shell run at 2 refinement steps and without, each with
    ms/frame and its frame-150 error against the stored FP64 oracle frame;
  * the paper's inexact CMS solve (20 interior modes, 10 Chebyshev-weighted
    Jacobi sweeps) on the shell: ms/frame and its frame-10 distance from the
    exact solve.
`--no-legs` prints the step, roofline and cpu_baseline only.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def committed_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (scaled by the plain-copy calibration), valid only while the kernel
    source is the one those counters were taken on; otherwise {}."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pd_step_shell390k_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2405_12484_amd", "csrc", "kernels.hip")
    try:
        lines = open(path).read().splitlines()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return {}
    want = [l.split()[1] for l in lines if l.startswith("kernels_sha256 ")]
    if not want or want[0] != sha:
        return {}
    out = {}
    for l in lines:
        f = l.split()
        if len(f) == 3 and f[0] == "traffic":
            out[f[1]] = int(f[2])
    return out


def copy_calibration(torch, mb=512, reps=5):
    """A plain device copy of `mb` MB (torch's copy kernel): achieved GB/s,
    counting read + write bytes.  Also the reference dispatch for scaling the
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes."""
    n = mb * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    del a, b
    return {"bytes_per_copy": 2 * n * 4, "avg_us": round(ms * 1e3, 2), "GBps": round(gbs, 1)}


def run(args):
    import torch

    from paper_2405_12484_amd import vhpd
    import synth

    p = synth.problem_by_name(args.workload)
    if args.subdomains:
        p.n_subdomains = args.subdomains
    torch.cuda.init()
    dev = torch.device("cuda:0")
    copy_cal = copy_calibration(torch)
    stream = torch.cuda.current_stream(dev)
    ctx = vhpd.Context(0)
    mesh = vhpd.Mesh(ctx, p.X, p.tets)
    mesh.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    t0 = time.perf_counter()
    mesh.prefactor(p.n_subdomains, args.refine)
    prefactor_s = time.perf_counter() - t0
    info = mesh.info()
    print(f"# prefactor {prefactor_s:.2f} s, info {info}", file=sys.stderr, flush=True)
    # a stiffness change refactors over the same structure (as a fitting loop
    # does); the second refactor restores the benchmark's stiffness, bitwise
    # the factor the prefactor made
    t0 = time.perf_counter()
    mesh.refactor(p.gamma_s * 1.1, p.gamma_v)
    refactor_s = time.perf_counter() - t0
    mesh.refactor(p.gamma_s, p.gamma_v)
    print(f"# refactor {refactor_s:.2f} s", file=sys.stderr, flush=True)
    # the interface factor's entries without the merge of odd-depth separators
    # into their parents (the merge adds stored values to save launches): the
    # method's count of what the interface sweeps must read
    keep_cfg = ctx.config()
    ctx.set_config(iface_merge_max_cols=0)
    m_count = vhpd.Mesh(ctx, p.X, p.tets)
    m_count.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m_count.prefactor(p.n_subdomains, args.refine)
    nnz_coarse_unmerged = m_count.info()["nnz_coarse"]
    m_count.close()
    ctx.set_config(**keep_cfg)

    # first frame from rest, kept for the error against the oracle; frame 10
    # from rest, kept for the configuration's stored oracle frame and the CMS leg
    mesh.regime_counts(reset=True, stream=stream)
    mesh.step(1, stream)
    x1, v1 = mesh.read_state(stream)
    mesh.step(9, stream)
    x10, _ = mesh.read_state(stream)
    mesh.step(max(0, args.warmup - 1), stream)
    torch.cuda.synchronize()

    # timed region: K frames
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    mesh.step(args.steps, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_frame = ev0.elapsed_time(ev1) / args.steps

    # projection regimes met by every local step since the first frame (Eq.
    # vol_pre): the workload stays on the plain + branch root
    regimes = mesh.regime_counts(stream=stream)
    info = mesh.info()
    # the residual gather runs inside the interior forward launch (its prologue)
    classes = ("local", "interior_fwd", "interface", "interior_bwd")
    nbytes = {"local": info["bytes_local"],
              "interior_fwd": info["bytes_interior_fwd"] + info["bytes_residual"],
              "interface": info["bytes_interface"], "interior_bwd": info["bytes_interior_bwd"]}
    kname = {"local": "k_local", "interior_fwd": "k_interior_fwd", "interface": "k_coarse",
             "interior_bwd": "k_interior_bwd"}
    launches = {k: (info["interface_launches"] if k == "interface" else 1) for k in classes}

    # per-class durations inside real frames: a second timed region of K frames
    # with HIP events recorded on the bench stream around every launch group of
    # each class (frames launched directly, not as a graph)
    mesh.profile(list(vhpd.Mesh.PROFILE_CLASSES))
    mesh.step(args.steps, stream)
    br = mesh.profile_read()
    mesh.profile([])
    breakdown = {k: round(v[0] / args.steps, 4) for k, v in br.items()}   # ms per frame
    group_us = {k: br[k][0] * 1e3 / br[k][1] for k in classes}            # us per launch group

    # isolated: `reps` back-to-back launches of one class (its data warm in
    # cache); also the residual gather as a launch of its own, and the forward
    # solve without it
    reps = {"local": 40, "residual": 40, "interior_fwd": 10, "interior_fwd_plain": 10, "interface": 10,
            "interior_bwd": 10}
    iso_us = {}
    for k, n in reps.items():
        mesh.time_kernel(k, 2, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mesh.time_kernel(k, n, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        iso_us[k] = e0.elapsed_time(e1) / n * 1e3

    traffic = committed_traffic()
    mbytes = method_bytes(p, info, nnz_coarse_unmerged)
    rooflines = {}
    for k in classes:
        gbs = mbytes[k] / (group_us[k] * 1e-6) / 1e9
        iso = mbytes[k] / (iso_us[k] * 1e-6) / 1e9
        t = traffic.get(k)
        rooflines[k] = {"kernel": kname[k], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": t, "bytes_per_launch": int(mbytes[k] / launches[k]),
                        "representation_bytes_per_launch": int(nbytes[k] / launches[k]),
                        "representation_over_method": round(nbytes[k] / mbytes[k], 3),
                        "representation_frac": round(nbytes[k] / (group_us[k] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                        "avg_launch_us": round(group_us[k] / launches[k], 3),
                        "launches_per_group": launches[k],
                        "us_per_frame": round(breakdown[k] * 1e3, 1),
                        "isolated_avg_launch_us": round(iso_us[k] / launches[k], 3),
                        "isolated_achieved": round(iso, 1), "isolated_frac": round(iso / HBM_PEAK_GBS, 4)}
    rooflines["interface"]["nnz_factor_unmerged"] = int(nnz_coarse_unmerged)
    rooflines["interface"]["nnz_factor_stored"] = int(info["nnz_coarse"])
    dominant = max(classes, key=lambda k: breakdown[k])
    roofline = dict(rooflines[dominant])
    # local step + scatter: the local launch in the frame, plus what the
    # residual gather adds to the forward launch (isolated, with and without it)
    ls_b = mbytes["local"] + mbytes["residual"]
    gather_us = max(iso_us["interior_fwd"] - iso_us["interior_fwd_plain"], 0.0)
    ls_us = group_us["local"] + gather_us
    ls_iso = iso_us["local"] + gather_us
    local_scatter = {
        "kernels": "k_local + the residual gather in the k_interior_fwd prologue",
        "bytes_per_iteration": ls_b,
        "representation_bytes_per_iteration": info["bytes_local"] + info["bytes_residual"],
        "gather_us_in_forward_launch": round(gather_us, 3),
        "gather_us_as_own_launch_isolated": round(iso_us["residual"], 3),
        "us_per_iteration": round(ls_us, 3),
        "target_us_per_iteration": round(ls_b / (0.6 * HBM_PEAK_GBS * 1e9) * 1e6, 2),
        "achieved": round(ls_b / (ls_us * 1e-6) / 1e9, 1),
        "isolated_us_per_iteration": round(ls_iso, 3),
        "isolated_achieved": round(ls_b / (ls_iso * 1e-6) / 1e9, 1),
    }
    local_scatter["frac"] = round(local_scatter["achieved"] / HBM_PEAK_GBS, 4)
    local_scatter["isolated_frac"] = round(local_scatter["isolated_achieved"] / HBM_PEAK_GBS, 4)

    nt, nv, nf = p.nt, p.nv, info["n_free"]
    out = {
        "metric": "ms/frame on 390K-tet PD; batched frames/s + p99 step latency vs plain",
        "value": round(ms_per_frame, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_frame, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision": {"local_step": "f32", "residual": "f32 sums, f64 inertia", "interior_solve": "f32",
                      "interface_solve": "f64", "factorization": "f64 (host)", "state": "f64"},
        "data": "synthetic",
        "config": {"workload": f"{p.name}_{nt}tets_{p.n_subdomains}subdomains", "tets": nt, "verts": nv,
                   "free_verts": nf, "interface_verts": info["n_interface"], "subdomains": p.n_subdomains,
                   "dt": p.dt, "pd_iters": p.pd_iters, "refine_steps": args.refine},
        "roofline": roofline,
        "local_plus_scatter": local_scatter,
        "rooflines": rooflines,
        "breakdown_ms_per_frame": breakdown,
        "hbm_copy_calibration": copy_cal,
        "prefactor_s": round(prefactor_s, 3),
        "refactor_s": round(refactor_s, 3),
        "projection_regimes": dict(regimes, element_evaluations=nt * p.pd_iters * (args.warmup + args.steps + 9)),
    }
    ref10 = _golden(f"{p.name}_oracle_x_f010.npy") if p.name == "shell" else None
    if ref10 is not None:
        out["rel_l2_frame10_vs_oracle"] = {"positions": _rel(x10, ref10),
                                           "displacements": float(np.linalg.norm(x10 - ref10) /
                                                                  np.linalg.norm(ref10 - p.X))}

    if not args.no_embed:
        out["embed"] = embed_timing(mesh, p, stream, torch)
        print(f"# embed: {out['embed']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], err = cpu_baseline(p, x1, args)
        out["rel_l2_first_frame_vs_oracle"] = err
    mesh.close()
    ctx.close()
    if args.legs and p.name == "shell":
        out["precision_refine2_150frames"] = precision_leg(p, args, stream, torch)
        print(f"# precision leg: {out['precision_refine2_150frames']}", file=sys.stderr, flush=True)
        out["cms_solve"] = cms_leg(p, x10, args, stream, torch)
        print(f"# CMS leg: {out['cms_solve']}", file=sys.stderr, flush=True)
    if args.serving:
        out["serving"] = serving(args)
    if args.adjoint:
        out["adjoint"] = adjoint_timing(args)
    print(json.dumps(out), flush=True)


def method_bytes(p, info, nnz_coarse_unmerged):
    """Bytes each kernel class must move per launch group by the method's own
    count, independent of this library's storage:
      local step   per tet: 4 vertex ids (16 B), Dm^{-1} (36 B), two weights
                   (8 B), four corner forces out (48 B); each vertex's
                   displacement read once (12 B per vertex);
      scatter      per (tet, corner) incidence: a 4-byte slot index and the
                   12-byte force; per vertex 32 B (inertia term and the
                   residual out);
      interior     every FP32 entry of the interior factors once per sweep
                   (4 B), the interior rows' vectors in and out; the forward
                   launch also gathers the residual (the scatter's bytes);
      interface    every entry of the interface factor once per sweep, with
                   its index (8 + 4 B), two sweeps; the entries counted without
                   the merge fill."""
    nt, nv, nf, ni = p.nt, p.nv, info["n_free"], info["n_interior"]
    scatter = 4 * nt * (4 + 12) + nv * 32
    return {"local": nt * (16 + 36 + 8 + 48) + nv * 12,
            "residual": scatter,
            "interior_fwd": 4 * info["nnz_interior"] + ni * (24 + 12) + scatter,
            "interface": 2 * 12 * nnz_coarse_unmerged,
            "interior_bwd": 4 * info["nnz_interior"] + ni * 12 + nf * (24 + 24)}


def embed_timing(mesh, p, stream, torch, per_tet=4, reps=20):
    """Positions of points embedded in the shell (Eq. m2y) for the current
    state: `per_tet` seeded points per tet, one k_embed launch per call.
    Algorithmic bytes: a 32-byte record and a 24-byte output row per point,
    plus each vertex position (24 bytes) read once."""
    import synth
    tet, P = synth.yarn_points(p.X, p.tets, per_tet=per_tet)
    mesh.set_embedding(tet, P)
    n = len(tet)
    out_t = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    mesh.embed_device(out_t, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        mesh.embed_device(out_t, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    nbytes = 56 * n + 24 * p.nv
    gbs = nbytes / (us * 1e-6) / 1e9
    mesh.set_embedding(np.zeros(0, dtype=np.int32), np.zeros((0, 3)))
    return {"kernel": "k_embed", "points": n, "points_per_tet": per_tet, "bound": "hbm",
            "bytes_per_launch": nbytes, "avg_launch_us": round(us, 3), "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "mpoints_per_s": round(n / us, 1)}


def _serve_stats(st, extra=None):
    out = {"frames_per_s": round(st["frames_per_second"], 1),
           "p50_ms": round(st["latency_p50_s"] * 1e3, 3), "p99_ms": round(st["latency_p99_s"] * 1e3, 3),
           "max_ms": round(st["latency_max_s"] * 1e3, 3), "frames": st["frames_done"],
           "launches": st["launches"], "mean_batch": round(st["mean_batch"], 2),
           "span_s": round(st["span_s"], 3), "hbm_peak_bytes": st["hbm_peak"]}
    if extra:
        out.update(extra)
    return out


def _poisson(rate, n_req, frames_left, seed_arr=7, seed_assign=8):
    """Aggregate Poisson step arrivals at `rate`/s; each request (one frame) goes
    to a garment drawn uniformly among those with frames left."""
    ra = np.random.Generator(np.random.PCG64(seed_arr))
    rg = np.random.Generator(np.random.PCG64(seed_assign))
    left = np.array(frames_left, dtype=np.int64)
    t = np.cumsum(ra.exponential(1.0 / rate, n_req))
    out = []
    for k in range(n_req):
        cand = np.flatnonzero(left > 0)
        if cand.size == 0:
            break
        g = int(cand[rg.integers(0, cand.size)])
        left[g] -= 1
        out.append((float(t[k]), g))
    return out


def _drive(srv, meshes, arrivals, release_after=None):
    """Submit `arrivals` [(t, garment)] in real time on the server clock while
    ticking the server; optionally release a garment right after its last
    request (release_after[g] = index of that request)."""
    import time as _t
    t_base = srv.now()
    i = 0
    while i < len(arrivals):
        now = srv.now() - t_base
        while i < len(arrivals) and arrivals[i][0] <= now:
            g = arrivals[i][1]
            srv.submit(meshes[g], 1, t_base + arrivals[i][0])
            if release_after is not None and release_after.get(g) == i:
                srv.release(meshes[g])
            i += 1
        if srv.tick() == 0 and i < len(arrivals):
            wait = arrivals[i][0] - (srv.now() - t_base)
            if wait > 2e-4:
                _t.sleep(min(wait - 1e-4, 5e-4))
    srv.drain()


def serving(args):
    """Continuous batching of step requests from 64 uneven shell garments
    (5K-200K tets, log-uniform), batched launches against sequential plain
    stepping on the same GPU with the same kernels (bitwise the same results
    per garment), plus admission under a 1 GB HBM budget."""
    import torch
    from paper_2405_12484_amd import vhpd
    import synth

    sizes = synth.serving_garment_sizes()
    t0 = time.perf_counter()
    probs = [synth.serving_shell_problem(int(n), 100 + g) for g, n in enumerate(sizes)]
    gen_s = time.perf_counter() - t0
    torch.cuda.init()
    copy_cal = copy_calibration(torch)      # also the reference dispatch for scaling rocprofv3 counters
    ctx = vhpd.Context(0)
    meshes = []
    for p in probs:
        m = vhpd.Mesh(ctx, p.X, p.tets)
        m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
        meshes.append(m)
    ng = len(meshes)
    out = {"garments": ng, "tets_total": int(sum(p.nt for p in probs)),
           "tets_min": int(min(p.nt for p in probs)), "tets_max": int(max(p.nt for p in probs)),
           "subdomains": sorted({int(p.n_subdomains) for p in probs}), "dt": probs[0].dt,
           "pd_iters": probs[0].pd_iters, "generate_s": round(gen_s, 2), "hbm_copy_calibration": copy_cal}
    # host factorization + upload of every garment (outside every timed window)
    t0 = time.perf_counter()
    srv = vhpd.Server(ctx, "batched", args.serve_in_flight)
    for m, p in zip(meshes, probs):
        srv.add(m, p.n_subdomains)
    srv.tick()
    out["prefactor_s"] = round(time.perf_counter() - t0, 2)
    out["hbm_all_resident_bytes"] = ctx.hbm_in_use()
    print(f"# serving: {ng} garments, {out['tets_total']} tets, prefactor {out['prefactor_s']} s, "
          f"{out['hbm_all_resident_bytes'] / 2**30:.2f} GiB resident", file=sys.stderr, flush=True)
    # local step + residual gather of all 64 garments in one batched launch each:
    # a working set (about 400 MB) larger than the 256 MB MALL
    stream = torch.cuda.current_stream()
    infos = [m.info() for m in meshes]
    lb = sum(i["bytes_local"] for i in infos)
    rb = sum(i["bytes_residual"] for i in infos)
    us = {}
    for k, reps in (("local", 20), ("residual", 20)):
        srv.time_kernel(k, 2, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        srv.time_kernel(k, reps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us[k] = e0.elapsed_time(e1) / reps * 1e3
    ach = (lb + rb) / ((us["local"] + us["residual"]) * 1e-6) / 1e9
    out["batched_local_plus_scatter"] = {
        "kernels": "k_local + k_residual over 64 garments", "bytes_local": lb, "bytes_residual": rb,
        "local_us": round(us["local"], 2), "residual_us": round(us["residual"], 2),
        "local_GBps": round(lb / (us["local"] * 1e-6) / 1e9, 1),
        "residual_GBps": round(rb / (us["residual"] * 1e-6) / 1e9, 1),
        "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}
    print(f"# batched local+scatter: {out['batched_local_plus_scatter']}", file=sys.stderr, flush=True)
    srv.close()

    def session(mode, arrivals, warm=True):
        srv = vhpd.Server(ctx, mode, args.serve_in_flight)
        for m, p in zip(meshes, probs):
            srv.add(m, p.n_subdomains)
        if warm:                                  # graphs captured, clocks warm
            for m in meshes:
                srv.submit(m, 1)
            srv.drain()
            srv.reset_stats()
        _drive(srv, meshes, arrivals)
        st = srv.stats()
        srv.close()
        return st

    F = args.serve_frames
    res = {}
    # saturated: every garment asks for F single-frame steps at t = 0
    sat = [(0.0, g) for _ in range(F) for g in range(ng)]
    res["saturated"] = {"requests": len(sat)}
    for mode in ("batched", "sequential"):
        st = session(mode, sat)
        res["saturated"][mode] = _serve_stats(st)
        print(f"# serving saturated {mode}: {res['saturated'][mode]}", file=sys.stderr, flush=True)
    res["saturated"]["speedup_frames_per_s"] = round(
        res["saturated"]["batched"]["frames_per_s"] / max(res["saturated"]["sequential"]["frames_per_s"], 1e-9), 2)
    # Poisson arrivals at several aggregate rates
    res["poisson"] = {}
    for rate in args.serve_rates:
        arr = _poisson(rate, args.serve_requests, [F * 10] * ng)
        r = {"requests": len(arr), "rate_per_s": rate}
        for mode in ("batched", "sequential"):
            st = session(mode, arr)
            r[mode] = _serve_stats(st)
            print(f"# serving poisson {rate}/s {mode}: {r[mode]}", file=sys.stderr, flush=True)
        res["poisson"][str(rate)] = r
    if args.serve_full:
        # the whole stream: every garment asks for 150 frames, one per request,
        # at an aggregate 200 requests/s (9,600 requests, about 48 s per mode)
        arr = _poisson(200.0, ng * 150, [150] * ng)
        r = {"requests": len(arr), "rate_per_s": 200.0, "frames_per_garment": 150}
        for mode in ("batched", "sequential"):
            st = session(mode, arr)
            r[mode] = _serve_stats(st)
            print(f"# serving full stream 200/s {mode}: {r[mode]}", file=sys.stderr, flush=True)
        res["poisson_full_stream"] = r
    # admission under a budget: every garment leaves the device after its last
    # request, making room for the ones waiting in FIFO order
    srv = vhpd.Server(ctx, "batched", args.serve_in_flight)
    for m, p in zip(meshes, probs):               # release all: device memory freed, host plans kept
        srv.add(m, p.n_subdomains)
    for m in meshes:
        srv.release(m)
    srv.close()
    budget = int(args.serve_budget_gb * 2**30)
    ctx.set_hbm_budget(budget)
    arr = _poisson(args.serve_budget_rate, ng * args.serve_budget_frames, [args.serve_budget_frames] * ng)
    last = {}
    for k, (_, g) in enumerate(arr):
        last[g] = k
    srv = vhpd.Server(ctx, "batched", args.serve_in_flight)
    for m, p in zip(meshes, probs):
        srv.add(m, p.n_subdomains)
    _drive(srv, meshes, arr, release_after=last)
    st = srv.stats()
    srv.close()
    res["budget"] = _serve_stats(st, {"budget_bytes": budget, "rate_per_s": args.serve_budget_rate,
                                      "requests": len(arr), "frames_per_garment": args.serve_budget_frames})
    print(f"# serving budget: {res['budget']}", file=sys.stderr, flush=True)
    out.update(res)
    for m in meshes:
        m.close()
    ctx.close()
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    """A stored FP64 oracle value (tests/golden/, written from the oracle only),
    or None when it is not there."""
    path = os.path.join(GOLDEN, name)
    return np.load(path) if os.path.exists(path) else None


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def adjoint_timing(args):
    """Gradient of 1/2 ||x_30 - x_30(hidden)||^2 with respect to gamma_s on the
    20,000-tet slab (30 frames of 10 iterations, checkpoints every 5) with the
    GPU discrete adjoint: forward and backward wall times, and the gradient's
    error against the stored FP64 oracle adjoint (same loss: the oracle's own
    x_30(hidden) as the target)."""
    import torch
    from paper_2405_12484_amd import vhpd
    import synth
    p = synth.problem_by_name("slab")
    ctx = vhpd.Context(0)
    m = vhpd.Mesh(ctx, p.X, p.tets)
    x0, v0 = p.initial_state()
    xt = _golden("slab_oracle_target_x30.npy")
    target = "oracle x_30(hidden)"
    if xt is None:
        m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
        m.prefactor(p.n_subdomains)
        xt = m.adjoint_forward(x0, v0, 30, 5)
        target = "GPU x_30(hidden)"
    gs0 = np.full(p.nt, 1e4)
    m.set_params(gs0, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    m.prefactor(p.n_subdomains)
    m.adjoint_forward(x0, v0, 30, 5)            # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xf = m.adjoint_forward(x0, v0, 30, 5)
    t1 = time.perf_counter()
    d = xf - xt
    d[p.pinned.astype(bool)] = 0.0
    g = m.adjoint_backward(d)
    t2 = time.perf_counter()
    m.close()
    ctx.close()
    out = {"workload": "slab_20000tets_8subdomains_30frames_ckpt5", "target": target,
           "forward_ms": round((t1 - t0) * 1e3, 2), "backward_ms": round((t2 - t1) * 1e3, 2),
           "loss": 0.5 * float((d * d).sum()), "grad_norm": float(np.linalg.norm(g))}
    g_ref = _golden("slab_oracle_grad.npy")
    if g_ref is not None and target.startswith("oracle"):
        out["rel_l2_vs_oracle_adjoint"] = _rel(g, g_ref)
    return out


def precision_leg(p, args, stream, torch):
    """The shell run 150 frames from rest with 2 refinement steps per solve:
    ms/frame and the error after 150 frames against the stored FP64 oracle
    trajectory (free-running), beside the same error without refinement."""
    from paper_2405_12484_amd import vhpd
    x150 = _golden("shell_oracle_x_f150.npy")
    out = {"workload": f"{p.name}_{p.nt}tets_150frames", "frames": 150}
    ctx = vhpd.Context(0)
    for refine in (2, 0):
        m = vhpd.Mesh(ctx, p.X, p.tets)
        m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
        m.prefactor(p.n_subdomains, refine)
        m.step(1, stream)
        m.write_state(*p.initial_state(), stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.step(150, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        x, _ = m.read_state(stream)
        leg = {"ms_per_frame": round(e0.elapsed_time(e1) / 150, 4)}
        if x150 is not None:
            leg["rel_l2_vs_oracle_frame150"] = _rel(x, x150)
            leg["rel_disp_vs_oracle_frame150"] = float(np.linalg.norm(x - x150) / np.linalg.norm(x150 - p.X))
        out[f"refine_{refine}"] = leg
        m.close()
    ctx.close()
    return out


def cms_leg(p, x10_exact, args, stream, torch):
    """The paper's inexact CMS global solve (20 interior modes per subdomain,
    10 Chebyshev-weighted Jacobi sweeps) on the same shell: ms/frame and its
    error after 10 frames from rest against the exact solve (the library's
    exact path, and the stored FP64 oracle when present)."""
    from paper_2405_12484_amd import vhpd
    ctx = vhpd.Context(0)
    ctx.set_config(cms_modes=20, cms_sweeps=10)
    m = vhpd.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    t0 = time.perf_counter()
    m.prefactor(p.n_subdomains)
    pf = time.perf_counter() - t0
    m.step(10, stream)
    x10, _ = m.read_state(stream)
    m.step(3, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    m.step(args.steps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    m.profile(list(vhpd.Mesh.PROFILE_CLASSES))
    m.step(3, stream)
    br = m.profile_read()
    m.profile([])
    out = {"modes": 20, "sweeps": 10, "ms_per_frame": round(e0.elapsed_time(e1) / args.steps, 4),
           "breakdown_ms_per_frame": {("cms_back_and_sweeps" if k == "interior_bwd" else k): round(v[0] / 3, 4)
                                      for k, v in br.items()},
           "prefactor_s": round(pf, 2), "device_bytes": m.info()["device_bytes"],
           "rel_l2_vs_exact_gpu_frame10": _rel(x10, x10_exact),
           "rel_disp_vs_exact_gpu_frame10": float(np.linalg.norm(x10 - x10_exact) / np.linalg.norm(x10_exact - p.X))}
    ref = _golden("shell_oracle_x_f010.npy")
    if ref is not None:
        out["rel_l2_vs_oracle_exact_frame10"] = _rel(x10, ref)
    m.close()
    ctx.close()
    return out


def cpu_baseline(p, x1_gpu, args):
    """The FP64 oracle (as it stands) on a bounded sample: the first frame of the
    same workload from rest, single-threaded BLAS; its ms/frame, and the GPU's
    first-frame error against it."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:
        lim = None
    t0 = time.perf_counter()
    sim = oracle.OracleSim.from_problem(p)
    setup = time.perf_counter() - t0
    x, v = p.initial_state()
    t0 = time.perf_counter()
    xo, _ = sim.step(x, v)
    ms = (time.perf_counter() - t0) * 1e3
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    err = float(np.linalg.norm(x1_gpu - xo) / np.linalg.norm(xo))
    derr = float(np.linalg.norm(x1_gpu - xo) / max(np.linalg.norm(xo - p.X), 1e-300))
    return ({"value": round(ms, 1), "unit": "ms/frame", "cores": 1, "kind": "oracle",
             "sample": f"1 frame ({p.pd_iters} PD iterations) of the same workload from rest; "
                       f"oracle setup (assembly + sparse LU) {setup:.1f} s excluded"},
            {"positions": err, "displacements": derr})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="shell")
    ap.add_argument("--refine", type=int, default=0)
    ap.add_argument("--subdomains", type=int, default=0, help="override the workload's subdomain count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", dest="serving", action="store_false")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false")
    ap.add_argument("--serve-only", action="store_true", help="only the serving runs (one JSON object)")
    ap.add_argument("--serve-frames", type=int, default=10, help="frames per garment, saturated run")
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[200.0, 1000.0, 5000.0])
    ap.add_argument("--serve-requests", type=int, default=600, help="requests per Poisson run")
    ap.add_argument("--no-embed", action="store_true", help="skip the embedded-point timing")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="skip the 150-frame refinement leg and the CMS-solve leg")
    ap.add_argument("--serve-full", action="store_true",
                    help="also serve the whole 200/s stream (150 frames per garment; about 100 s)")
    ap.add_argument("--serve-in-flight", type=int, default=2)
    ap.add_argument("--serve-budget-gb", type=float, default=1.0)
    ap.add_argument("--serve-budget-rate", type=float, default=1000.0)
    ap.add_argument("--serve-budget-frames", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this "
              "path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    if args.serve_only:
        print(json.dumps({"serving": serving(args)}), flush=True)
        return
    run(args)


if __name__ == "__main__":
    main()
