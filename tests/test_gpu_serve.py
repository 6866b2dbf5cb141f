"""The step server on the GPU, through the C ABI: every garment's trajectory
is bitwise the same served alone, in a mix of uneven garments, sequentially,
and by plain stepping; admission under an HBM budget is first come, first
served; misuse is reported."""

import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import rel_l2, say

pytestmark = pytest.mark.gpu

# (tet-count target, material seed) of three uneven shell garments
GARMENTS = [(9000, 101), (5000, 100), (14000, 102)]
# per garment: frames of each successive request (6 frames in all)
REQUESTS = [[1, 2, 1, 2], [3, 1, 2], [1, 1, 1, 1, 2]]


@pytest.fixture(scope="module")
def vh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12484_amd import vhpd
    vhpd.load()
    return vhpd


@pytest.fixture(scope="module")
def probs():
    return [synth.serving_shell_problem(t, s) for t, s in GARMENTS]


def new_mesh(vh, ctx, p):
    m = vh.Mesh(ctx, p.X, p.tets)
    m.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters)
    return m


def serve(vh, probs, which, mode="batched", budget=0, in_flight=2, order_seed=None, release=()):
    """Serve the requests of garments `which` on a fresh context; returns the
    final states and the server stats."""
    ctx = vh.Context(0, budget)
    srv = vh.Server(ctx, mode, in_flight)
    ms = {}
    for g in which:
        ms[g] = new_mesh(vh, ctx, probs[g])
        srv.add(ms[g], probs[g].n_subdomains)
    reqs = [(g, n) for g in which for n in REQUESTS[g]]
    if order_seed is not None:
        # interleave the garments' requests in a random order, keeping each
        # garment's own order, and tick between submissions so launches form
        # around whatever has arrived
        rng = np.random.default_rng(order_seed)
        queues = {g: list(REQUESTS[g]) for g in which}
        reqs = []
        while any(queues.values()):
            g = rng.choice([k for k, q in queues.items() if q])
            reqs.append((g, queues[g].pop(0)))
    tickets = []
    for g, n in reqs:
        tickets.append(srv.submit(ms[g], n))
        if order_seed is not None:
            srv.tick()
    for g in release:
        srv.release(ms[g])
    srv.drain()
    for t in tickets:
        done, lat = srv.poll(t)
        assert done and lat > 0.0
    st = srv.stats()
    out = {g: ms[g].read_state() for g in which}
    srv.close()
    for m in ms.values():
        m.close()
    ctx.close()
    return out, st


def plain(vh, p, frames):
    ctx = vh.Context(0)
    m = new_mesh(vh, ctx, p)
    m.prefactor(p.n_subdomains)
    m.step(frames)
    x, v = m.read_state()
    m.close()
    ctx.close()
    return x, v


@pytest.fixture(scope="module")
def alone(vh, probs):
    res = {}
    for g in range(len(GARMENTS)):
        say(f"[serve] alone garment {g} ({probs[g].nt} tets, D={probs[g].n_subdomains})")
        out, st = serve(vh, probs, [g])
        res[g] = (out[g], st)
    return res


def test_alone_matches_plain_stepping_and_oracle(vh, probs, alone):
    for g, p in enumerate(probs):
        say(f"[serve] plain garment {g}")
        x, v = plain(vh, p, sum(REQUESTS[g]))
        xa, va = alone[g][0]
        assert np.array_equal(x, xa) and np.array_equal(v, va)
    # the smallest garment against the FP64 oracle, frame by frame
    p = probs[1]
    sim = oracle.OracleSim.from_problem(p)
    x, v = p.initial_state()
    for _ in range(sum(REQUESTS[1])):
        x, v = sim.step(x, v)
    err = rel_l2(alone[1][0][0], x)
    say(f"[serve] garment 1 after {sum(REQUESTS[1])} frames: rel L2 {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("in_flight,seed", [(1, 0), (2, 1), (4, 2)])
def test_mix_is_bitwise_alone(vh, probs, alone, in_flight, seed):
    say(f"[serve] mix in_flight={in_flight} seed={seed}")
    out, st = serve(vh, probs, [0, 1, 2], in_flight=in_flight, order_seed=seed)
    for g in range(3):
        xa, va = alone[g][0]
        assert np.array_equal(out[g][0], xa), g
        assert np.array_equal(out[g][1], va), g
    assert st["frames_done"] == sum(sum(r) for r in REQUESTS)
    assert st["requests_done"] == sum(len(r) for r in REQUESTS)
    assert st["mean_batch"] > 1.0            # frames of different garments shared launches


# interface lane-group thresholds per garment (mean task lengths from which
# 32 and 64 lanes are used): the default, 32 lanes everywhere, 64 everywhere
LANE_GROUPS = {0: None, 1: (1, 100000000), 2: (1, 1)}


def _add_with_groups(ctx, srv, m, p, spec):
    keep = ctx.config()
    if spec:
        ctx.set_config(iface_lanes32_min=spec[0], iface_lanes64_min=spec[1])
    try:
        srv.add(m, p.n_subdomains)
    finally:
        ctx.set_config(**keep)


def test_mix_of_lane_groups_is_bitwise_alone(vh, probs):
    """Phase j of the three garments has three lane-group sizes, so one
    interface phase index becomes several batched launches."""
    def run(which, seed):
        ctx = vh.Context(0)
        srv = vh.Server(ctx, "batched", 2)
        ms = {}
        for g in which:
            ms[g] = new_mesh(vh, ctx, probs[g])
            _add_with_groups(ctx, srv, ms[g], probs[g], LANE_GROUPS[g])
        rng = np.random.default_rng(seed)
        queues = {g: list(REQUESTS[g]) for g in which}
        while any(queues.values()):
            g = rng.choice([k for k, q in queues.items() if q])
            srv.submit(ms[g], queues[g].pop(0))
            srv.tick()
        srv.drain()
        st = srv.stats()
        out = {g: ms[g].read_state() for g in which}
        srv.close()
        for m in ms.values():
            m.close()
        ctx.close()
        return out, st

    say("[serve] lane groups alone")
    alone = {g: run([g], 0)[0][g] for g in range(3)}
    say("[serve] lane groups mixed")
    out, st = run([0, 1, 2], 7)
    for g in range(3):
        assert np.array_equal(out[g][0], alone[g][0]), g
        assert np.array_equal(out[g][1], alone[g][1]), g
    assert st["mean_batch"] > 1.0


def test_serving_sizes_span_is_bitwise_alone(vh):
    """The smallest, median and largest of the 64 serving garments (about 5K,
    31K and 191K tets; 2 to 64 subdomains), served together and alone: the
    same final states bit for bit."""
    sizes = synth.serving_garment_sizes()
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    ps = [synth.serving_shell_problem(int(sizes[g]), 100 + g) for g in pick]

    def run(which):
        ctx = vh.Context(0)
        srv = vh.Server(ctx, "batched", 2)
        ms = {}
        for i in which:
            ms[i] = new_mesh(vh, ctx, ps[i])
            srv.add(ms[i], ps[i].n_subdomains)
        for i in which:
            srv.submit(ms[i], 3)
        srv.drain()
        st = srv.stats()
        out = {i: ms[i].read_state()[0] for i in which}
        srv.close()
        for m in ms.values():
            m.close()
        ctx.close()
        return out, st

    say(f"[serve] sizes {[ps[i].nt for i in range(3)]}, subdomains {[ps[i].n_subdomains for i in range(3)]}")
    alone = {i: run([i])[0][i] for i in range(3)}
    mixed, st = run([0, 1, 2])
    assert st["mean_batch"] > 1.0
    for i in range(3):
        assert np.array_equal(mixed[i], alone[i]), i


def test_mix_with_refinement_is_bitwise_plain(vh, probs):
    """Two garments served together with one refinement step per PD
    iteration (the FP64 residual and a second decomposed solve inside the
    batched frame) end bitwise where plain stepping with the same refinement
    ends."""
    say("[serve] mix with refinement")
    which = [0, 1]
    ctx = vh.Context(0)
    srv = vh.Server(ctx, "batched", 2)
    ms = {}
    for g in which:
        ms[g] = new_mesh(vh, ctx, probs[g])
        srv.add(ms[g], probs[g].n_subdomains, 1)
    tickets = [srv.submit(ms[g], n) for g in which for n in REQUESTS[g]]
    srv.drain()
    assert all(srv.poll(t)[0] for t in tickets)
    out = {g: ms[g].read_state() for g in which}
    assert srv.stats()["mean_batch"] > 1.0
    srv.close()
    for m in ms.values():
        m.close()
    ctx.close()
    for g in which:
        p = probs[g]
        c2 = vh.Context(0)
        m = new_mesh(vh, c2, p)
        m.prefactor(p.n_subdomains, 1)
        m.step(sum(REQUESTS[g]))
        x, v = m.read_state()
        m.close()
        c2.close()
        assert np.array_equal(out[g][0], x), g
        assert np.array_equal(out[g][1], v), g


def test_mix_with_cms_solve_is_bitwise_plain(vh, probs):
    """Two garments served together with the inexact CMS global solve (8
    interior modes, 4 sweeps) end bitwise where plain stepping with the same
    solve ends."""
    say("[serve] mix with the CMS solve")
    which = [0, 1]
    ctx = vh.Context(0)
    ctx.set_config(cms_modes=8, cms_sweeps=4)
    srv = vh.Server(ctx, "batched", 2)
    ms = {}
    for g in which:
        ms[g] = new_mesh(vh, ctx, probs[g])
        srv.add(ms[g], probs[g].n_subdomains)
    tickets = [srv.submit(ms[g], n) for g in which for n in REQUESTS[g]]
    srv.drain()
    assert all(srv.poll(t)[0] for t in tickets)
    out = {g: ms[g].read_state() for g in which}
    srv.close()
    for m in ms.values():
        m.close()
    ctx.close()
    for g in which:
        p = probs[g]
        c2 = vh.Context(0)
        c2.set_config(cms_modes=8, cms_sweeps=4)
        m = new_mesh(vh, c2, p)
        m.prefactor(p.n_subdomains)
        m.step(sum(REQUESTS[g]))
        x, v = m.read_state()
        m.close()
        c2.close()
        assert np.array_equal(out[g][0], x), g
        assert np.array_equal(out[g][1], v), g


def test_sequential_mode_is_bitwise_alone(vh, probs, alone):
    say("[serve] sequential mix")
    out, st = serve(vh, probs, [0, 1, 2], mode="sequential", order_seed=5)
    for g in range(3):
        assert np.array_equal(out[g][0], alone[g][0][0])
    assert st["mean_batch"] == 1.0
    assert st["launches"] == sum(sum(r) for r in REQUESTS)


def test_admission_waits_for_budget(vh, probs, alone):
    # peak device bytes of each garment served alone
    peak = [alone[g][1]["hbm_peak"] for g in range(3)]
    # garments 0 and 1 fit together; garment 2 fits only once garment 0 has left
    budget = peak[2] + peak[1] + peak[0] // 2
    assert peak[0] + peak[1] <= budget < sum(peak)
    say(f"[serve] budget {budget} (alone peaks {peak})")
    ctx = vh.Context(0, budget)
    srv = vh.Server(ctx, "batched", 2)
    ms = [new_mesh(vh, ctx, p) for p in probs]
    for g in range(3):
        srv.add(ms[g], probs[g].n_subdomains)
    srv.tick()
    st = srv.stats()
    assert (st["meshes_resident"], st["meshes_waiting"]) == (2, 1)
    tk = {g: [srv.submit(ms[g], n) for n in REQUESTS[g]] for g in range(3)}
    # garment 2 waits: without a release nothing can admit it
    with pytest.raises(vh.VHError) as e:
        srv.drain()
    assert e.value.code == vh.VH_ESTATE
    assert all(srv.poll(t)[0] for t in tk[0] + tk[1])
    assert not any(srv.poll(t)[0] for t in tk[2])
    srv.release(ms[0])                       # leaves the device: garment 2 fits now
    srv.drain()
    assert all(srv.poll(t)[0] for t in tk[2])
    st = srv.stats()
    assert st["hbm_peak"] <= budget
    assert (st["meshes_resident"], st["meshes_waiting"]) == (2, 0)
    for g in range(3):
        x, v = ms[g].read_state()            # garment 0 from the state kept on release
        assert np.array_equal(x, alone[g][0][0]), g
    srv.close()
    for m in ms:
        m.close()
    ctx.close()


def test_serve_errors(vh, probs):
    ctx = vh.Context(0)
    srv = vh.Server(ctx, "batched")
    with pytest.raises(vh.VHError) as e:
        vh.Server(ctx, "batched")
    assert e.value.code == vh.VH_ESTATE
    a = new_mesh(vh, ctx, probs[1])
    with pytest.raises(vh.VHError) as e:
        srv.submit(a, 1)                     # not in the server
    assert e.value.code == vh.VH_EINVAL
    srv.add(a, probs[1].n_subdomains)
    with pytest.raises(vh.VHError) as e:
        a.step(1)                            # driven by the server
    assert e.value.code == vh.VH_ESTATE
    with pytest.raises(vh.VHError) as e:
        srv.submit(a, 0)
    assert e.value.code == vh.VH_EINVAL
    b = vh.Mesh(ctx, probs[1].X, probs[1].tets)
    p = probs[1]
    b.set_params(p.gamma_s, p.gamma_v, p.mass, p.pinned, p.gravity, p.dt, p.pd_iters + 1)
    with pytest.raises(vh.VHError) as e:
        srv.add(b, p.n_subdomains)           # a different iteration count
    assert e.value.code == vh.VH_EINVAL
    srv.submit(a, 2)
    srv.drain()
    srv.close()
    a.step(1)                                # out of the server: plain stepping again
    a.close()
    b.close()
    ctx.close()
    # a garment larger than the whole budget is refused at once
    ctx = vh.Context(0, 1 << 20)
    srv = vh.Server(ctx, "batched")
    c = new_mesh(vh, ctx, probs[0])
    with pytest.raises(vh.VHError) as e:
        srv.add(c, probs[0].n_subdomains)
    assert e.value.code == vh.VH_ENOMEM
    srv.close()
    c.close()
    ctx.close()
