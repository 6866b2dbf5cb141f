"""CPU checks of the library's host prefactor (partition, orderings, FP64
multifrontal factorization, solve programs) through a host emulation of the
device solve programs, against the oracle's exact sparse solve."""

import ctypes
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from tests.host import build as hbuild

_vp, _ci, _cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double


@pytest.fixture(scope="module")
def hl():
    lib = ctypes.CDLL(hbuild.ensure())
    lib.vhp_build.restype = _vp
    lib.vhp_build.argtypes = [_vp, _ci, _vp, _ci, _vp, _vp, _vp, _vp, _vp, _cd, _ci, _ci, _ci, _ci, _vp, _vp, _ci]
    lib.vhp_info.argtypes = [_vp, _vp]
    lib.vhp_solve.argtypes = [_vp, _vp, _vp]
    lib.vhp_free.argtypes = [_vp]
    lib.vhp_perm.argtypes = [_vp, _vp]
    return lib


def _build(hl, p, D, leaf=32, pinned=None):
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    keep = [a(p.X, np.float64), a(p.tets, np.int32), a(p.gamma_s, np.float64), a(p.gamma_v, np.float64),
            a(p.mass, np.float64), a(p.pinned if pinned is None else pinned, np.uint8), a(p.gravity, np.float64)]
    rc = ctypes.c_int(0)
    msg = ctypes.create_string_buffer(256)
    h = hl.vhp_build(keep[0].ctypes.data, p.nv, keep[1].ctypes.data, p.nt, keep[2].ctypes.data,
                     keep[3].ctypes.data, keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data,
                     p.dt, p.pd_iters, D, 0, leaf, ctypes.byref(rc), msg, 256)
    info = np.zeros(17, dtype=np.int64)
    if h:
        hl.vhp_info(h, info.ctypes.data)
    keys = ("n_free n_int n_gamma D n_sn n_clevels nnz_int nnz_coarse max_sub_phases n_chunks n_ctasks n_cslots "
            "max_sub_n max_cint max_nb max_fwd_chunks max_bwd_chunks")
    return h, rc.value, msg.value.decode(), dict(zip(keys.split(), info.tolist()))


@pytest.mark.parametrize("name,D,leaf", [("box", 4, 32), ("box", 1, 32), ("box", 2, 8), ("box", 8, 1000),
                                         ("shell_small", 8, 32), ("shell_small", 16, 16), ("slab", 8, 32)])
def test_emulated_solve_matches_exact(hl, name, D, leaf):
    p = synth.problem_by_name(name)
    h, rc, msg, info = _build(hl, p, D, leaf)
    assert rc == 0, msg
    try:
        sim = oracle.OracleSim.from_problem(p)
        assert info["n_free"] == sim.free.size
        assert info["n_int"] + info["n_gamma"] == info["n_free"]
        if D == 1:
            assert info["n_gamma"] == 0
        rng = np.random.default_rng(D)
        rhs = rng.standard_normal((p.nv, 3))
        d = np.zeros((p.nv, 3))
        hl.vhp_solve(h, rhs.ctypes.data, d.ctypes.data)
        xe = sim._solve(rhs[sim.free])
        # interior factor blocks are stored in FP32
        assert np.linalg.norm(d[sim.free] - xe) <= 2e-7 * np.linalg.norm(xe)
        assert np.all(d[sim.fixed] == 0)
    finally:
        hl.vhp_free(h)


def test_long_interior_program(hl):
    """A 10 x 10 x 22 hex box as one subdomain: its forward program has more
    chunks (65) than the interior kernels' 64-entry LDS table of chunk
    descriptors. The programs past the table still solve exactly. (The GPU
    refuses this subdomain: its contribution slots need more LDS than a CU has;
    no subdomain that fits LDS has reached 64 chunks in the meshes tried, so the
    kernels' global descriptor reads are not exercised on the GPU.)"""
    p = synth.meshes.make_box_problem(nx=10, ny=10, nz=22, name="box_long")
    h, rc, msg, info = _build(hl, p, 1)
    assert rc == 0, msg
    try:
        assert info["max_fwd_chunks"] > 64
        sim = oracle.OracleSim.from_problem(p)
        rhs = np.random.default_rng(5).standard_normal((p.nv, 3))
        d = np.zeros((p.nv, 3))
        hl.vhp_solve(h, rhs.ctypes.data, d.ctypes.data)
        xe = sim._solve(rhs[sim.free])
        assert np.linalg.norm(d[sim.free] - xe) <= 2e-7 * np.linalg.norm(xe)
    finally:
        hl.vhp_free(h)


@pytest.mark.parametrize("name,D,words", [("box", 1, 2048), ("box", 2, 2048), ("shell_small", 8, 4096)])
def test_small_chunks_solve_exactly(hl, name, D, words):
    """Interior programs cut into chunks of at most `words` 32-bit words
    instead of the kernels' 12,288 (more chunks, the same phases): the
    emulated solve is the one the full-size chunks give, to FP32 rounding, and
    exact; a chunk size that cannot hold a supernode's block is refused."""
    p = synth.problem_by_name(name)
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    keep = [a(p.X, np.float64), a(p.tets, np.int32), a(p.gamma_s, np.float64), a(p.gamma_v, np.float64),
            a(p.mass, np.float64), a(p.pinned, np.uint8), a(p.gravity, np.float64)]
    hl.vhp_build_chunks.restype = _vp
    hl.vhp_build_chunks.argtypes = [_vp, _ci, _vp, _ci, _vp, _vp, _vp, _vp, _vp, _cd, _ci, _ci, _ci, _ci, _vp, _vp,
                                    _ci]
    rhs = np.random.default_rng(3).standard_normal((p.nv, 3))
    sim = oracle.OracleSim.from_problem(p)
    xe = sim._solve(rhs[sim.free])
    out = {}
    for w in (12288, words, 256):
        rc = ctypes.c_int(0)
        msg = ctypes.create_string_buffer(256)
        h = hl.vhp_build_chunks(keep[0].ctypes.data, p.nv, keep[1].ctypes.data, p.nt, keep[2].ctypes.data,
                                keep[3].ctypes.data, keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data,
                                p.dt, p.pd_iters, D, 32, w, ctypes.byref(rc), msg, 256)
        if w == 256:
            assert not h and rc.value != 0 and "chunk" in msg.value.decode()
            continue
        assert h, msg.value.decode()
        try:
            info = np.zeros(17, dtype=np.int64)
            hl.vhp_info(h, info.ctypes.data)
            d = np.zeros((p.nv, 3))
            hl.vhp_solve(h, rhs.ctypes.data, d.ctypes.data)
            out[w] = (int(info[15]), d)
        finally:
            hl.vhp_free(h)
    assert out[words][0] > out[12288][0]
    d0, d1 = out[12288][1], out[words][1]
    assert np.linalg.norm(d1 - d0) <= 1e-7 * np.linalg.norm(d0)
    assert np.linalg.norm(d1[sim.free] - xe) <= 2e-7 * np.linalg.norm(xe)


def test_refactor_matches_fresh_plan(hl):
    """A plan refactored with new stiffness solves exactly as a plan built
    from scratch with that stiffness (bitwise: the same matrix assembly and
    numeric factorization over the same supernodes), and matches the oracle's
    exact solve with the new stiffness."""
    p = synth.problem_by_name("shell_small")
    rng = np.random.default_rng(11)
    gs2 = p.gamma_s * rng.uniform(0.5, 2.0, p.nt)
    gv2 = p.gamma_v * rng.uniform(0.5, 2.0, p.nt)
    p2 = dataclasses.replace(p, gamma_s=gs2, gamma_v=gv2)
    h1, rc, msg, _ = _build(hl, p, 8)
    assert rc == 0, msg
    h2, rc, msg, _ = _build(hl, p2, 8)
    assert rc == 0, msg
    try:
        hl.vhp_refactor.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _ci]
        X = np.ascontiguousarray(p.X, dtype=np.float64)
        T = np.ascontiguousarray(p.tets, dtype=np.int32)
        rcv = ctypes.c_int(0)
        m = ctypes.create_string_buffer(256)
        hl.vhp_refactor(h1, X.ctypes.data, T.ctypes.data, gs2.ctypes.data, gv2.ctypes.data, ctypes.byref(rcv), m, 256)
        assert rcv.value == 0, m.value.decode()
        rhs = np.random.default_rng(12).standard_normal((p.nv, 3))
        d1 = np.zeros((p.nv, 3))
        d2 = np.zeros((p.nv, 3))
        hl.vhp_solve(h1, rhs.ctypes.data, d1.ctypes.data)
        hl.vhp_solve(h2, rhs.ctypes.data, d2.ctypes.data)
        assert np.array_equal(d1, d2)
        sim = oracle.OracleSim.from_problem(p2)
        xe = sim._solve(rhs[sim.free])
        assert np.linalg.norm(d1[sim.free] - xe) <= 2e-7 * np.linalg.norm(xe)
    finally:
        hl.vhp_free(h1)
        hl.vhp_free(h2)


def test_permutation_is_bijection_free_first(hl):
    p = synth.problem_by_name("shell_small")
    h, rc, msg, info = _build(hl, p, 8)
    assert rc == 0, msg
    perm = np.zeros(p.nv, dtype=np.int32)
    hl.vhp_perm(h, perm.ctypes.data)
    hl.vhp_free(h)
    assert sorted(perm.tolist()) == list(range(p.nv))
    nf = info["n_free"]
    assert np.all(p.pinned[perm[:nf]] == 0) and np.all(p.pinned[perm[nf:]] == 1)


def test_non_power_of_two_rejected(hl):
    p = synth.problem_by_name("box")
    h, rc, msg, info = _build(hl, p, 3)
    assert h is None and rc == -1 and "power of two" in msg


def test_unpinned_mesh(hl):
    p = synth.problem_by_name("box")
    pins = np.zeros(p.nv, dtype=np.uint8)
    h, rc, msg, info = _build(hl, p, 4, pinned=pins)
    assert rc == 0, msg
    assert info["n_free"] == p.nv
    hl.vhp_free(h)


def test_non_finite_pivot_is_not_spd(hl):
    """dt = 1e-160 passes the argument checks (finite, positive) but M / dt^2
    overflows to inf, so the factorization meets a pivot that is not a positive
    finite number: the plan fails with VH_ENOTSPD (-3) and no plan is returned."""
    import dataclasses
    p = dataclasses.replace(synth.problem_by_name("box"), dt=1e-160)
    h, rc, msg, info = _build(hl, p, 4)
    assert h is None and rc == -3 and "pivot" in msg


def _build_opts(hl, p, D, thin, merge=3000):
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    keep = [a(p.X, np.float64), a(p.tets, np.int32), a(p.gamma_s, np.float64), a(p.gamma_v, np.float64),
            a(p.mass, np.float64), a(p.pinned, np.uint8), a(p.gravity, np.float64)]
    hl.vhp_build_opts.restype = _vp
    hl.vhp_build_opts.argtypes = [_vp, _ci, _vp, _ci, _vp, _vp, _vp, _vp, _vp, _cd, _ci, _ci, _ci, _ci, _vp, _vp, _ci]
    rc = ctypes.c_int(0)
    msg = ctypes.create_string_buffer(256)
    h = hl.vhp_build_opts(keep[0].ctypes.data, p.nv, keep[1].ctypes.data, p.nt, keep[2].ctypes.data,
                          keep[3].ctypes.data, keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data,
                          p.dt, p.pd_iters, D, thin, merge, ctypes.byref(rc), msg, 256)
    assert rc.value == 0, msg.value.decode()
    return h


@pytest.mark.parametrize("name", ["box", "shell_small", "slab"])
def test_cms_program_matches_oracle(hl, name):
    """The library's CMS data (host FP64 Lanczos modes and boundary modes,
    stored FP32) run as the device does (host emulation) against the FP64 CMS
    oracle on the same partition (separators not thinned: the oracle's
    interface is every vertex two subdomains share): 20 modes, 10 Chebyshev
    sweeps, the same spectral radius."""
    from oracle.cms import CMSSolver
    from oracle.dd import bisect_elements
    p = synth.problem_by_name(name)
    h = _build_opts(hl, p, p.n_subdomains, 0)
    try:
        perm = np.zeros(p.nv, dtype=np.int32)
        hl.vhp_perm(h, perm.ctypes.data)
        so = np.zeros(p.n_subdomains + 1, dtype=np.int32)
        hl.vhp_sub_off.argtypes = [_vp, _vp]
        hl.vhp_sub_off(h, so.ctypes.data)
        sim = oracle.OracleSim.from_problem(p)
        cms = CMSSolver(sim.L_ff, sim.free, sim.tets, bisect_elements(sim.tets, p.n_subdomains), 20, 10)
        assert [set(perm[so[d]:so[d + 1]].tolist()) for d in range(p.n_subdomains)] == \
            [set(sim.free[I].tolist()) for I in cms.interiors]
        rhs = np.random.default_rng(2).standard_normal((p.nv, 3))
        rhs[p.pinned.astype(bool)] = 0.0
        d = np.zeros((p.nv, 3))
        info = np.zeros(2)
        hl.vhp_cms_solve.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp]
        assert hl.vhp_cms_solve(h, 20, 10, rhs.ctypes.data, d.ctypes.data, info.ctypes.data) == 0
        assert abs(info[0] - cms.rho) <= 1e-10
        xo = np.zeros((p.nv, 3))
        xo[sim.free] = cms.solve(rhs[sim.free])
        assert np.linalg.norm(d - xo) <= 1e-7 * np.linalg.norm(xo)
    finally:
        hl.vhp_free(h)
