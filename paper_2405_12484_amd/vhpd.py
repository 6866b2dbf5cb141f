"""Python binding of libvhpd (ctypes; argument marshalling only).

Every step of the simulation runs in the HIP library; this module converts
numpy arrays and torch streams/tensors into the plain pointers and sizes of
the C ABI in ``include/vhpd.h`` and raises ``VHError`` on a nonzero return.
It fails loudly when the library has not been built: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvhpd.so")

VH_OK, VH_EINVAL, VH_ENOMEM, VH_ENOTSPD, VH_ESTATE, VH_ENUMERIC, VH_EDEVICE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {-1: "VH_EINVAL", -2: "VH_ENOMEM", -3: "VH_ENOTSPD", -4: "VH_ESTATE", -5: "VH_ENUMERIC",
          -6: "VH_EDEVICE"}

# Every symbol the header declares, with (restype, argtypes).
_vp, _i32, _dbl, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
_P = ctypes.POINTER


class MeshInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("nt", ctypes.c_int32), ("n_free", ctypes.c_int32),
                ("n_interior", ctypes.c_int32), ("n_interface", ctypes.c_int32),
                ("n_subdomains", ctypes.c_int32), ("n_supernodes", ctypes.c_int32),
                ("n_coarse_levels", ctypes.c_int32), ("max_interior_phases", ctypes.c_int32),
                ("nnz_interior", ctypes.c_int64), ("nnz_coarse", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t), ("prefactor_seconds", ctypes.c_double),
                ("n_partials", ctypes.c_int64),
                ("bytes_local", ctypes.c_int64), ("bytes_residual", ctypes.c_int64),
                ("bytes_interior_fwd", ctypes.c_int64), ("bytes_interface", ctypes.c_int64),
                ("bytes_interior_bwd", ctypes.c_int64), ("interface_launches", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServeStats(ctypes.Structure):
    _fields_ = [("frames_done", ctypes.c_int64), ("requests_done", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("span_s", ctypes.c_double),
                ("frames_per_second", ctypes.c_double), ("latency_p50_s", ctypes.c_double),
                ("latency_p99_s", ctypes.c_double), ("latency_max_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("meshes_resident", ctypes.c_int32), ("meshes_waiting", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Config(ctypes.Structure):
    _fields_ = [("use_graphs", ctypes.c_int32), ("iface_lanes32_min", ctypes.c_int32),
                ("iface_lanes64_min", ctypes.c_int32), ("thin_separators", ctypes.c_int32),
                ("iface_merge_max_cols", ctypes.c_int32), ("cms_modes", ctypes.c_int32),
                ("cms_sweeps", ctypes.c_int32), ("interior_desc_table", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RegimeCounts(ctypes.Structure):
    _fields_ = [("clamped", ctypes.c_uint64), ("inverted", ctypes.c_uint64), ("det_ge2", ctypes.c_uint64),
                ("squash", ctypes.c_uint64), ("no_plus_root", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


VH_PRECISION_MIXED = 0


class GNStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int64),
                ("outer_rel_residual", ctypes.c_double), ("inner_rel_residual_max", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

SIGNATURES = {
    "vh_last_error": (ctypes.c_char_p, []),
    "vh_ctx_create": (ctypes.c_int, [_P(_vp), ctypes.c_int, _sz]),
    "vh_ctx_destroy": (ctypes.c_int, [_vp]),
    "vh_ctx_hbm_in_use": (ctypes.c_int, [_vp, _P(_sz)]),
    "vh_ctx_set_hbm_budget": (ctypes.c_int, [_vp, _sz]),
    "vh_ctx_get_config": (ctypes.c_int, [_vp, _P(Config)]),
    "vh_ctx_set_config": (ctypes.c_int, [_vp, _P(Config)]),
    "vh_mesh_create": (ctypes.c_int, [_vp, _P(_vp), _vp, _i32, _vp, _i32]),
    "vh_mesh_destroy": (ctypes.c_int, [_vp]),
    "vh_mesh_set_params": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _dbl, _i32]),
    "vh_mesh_prefactor": (ctypes.c_int, [_vp, _i32, _i32, _i32]),
    "vh_mesh_refactor": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_mesh_regime_counts": (ctypes.c_int, [_vp, _P(RegimeCounts), _i32, _vp]),
    "vh_mesh_step": (ctypes.c_int, [_vp, _i32, _vp]),
    "vh_mesh_step_noalloc": (ctypes.c_int, [_vp, _i32, _vp]),
    "vh_mesh_read_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_mesh_write_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_mesh_read_state_device": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_mesh_write_state_device": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_mesh_get_info": (ctypes.c_int, [_vp, _P(MeshInfo)]),
    "vh_mesh_time_kernel": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "vh_mesh_profile": (ctypes.c_int, [_vp, ctypes.c_uint32]),
    "vh_mesh_profile_read": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_debug_local_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vh_debug_residual": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_debug_residual_in_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_debug_scatter_colored": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vh_debug_interface_factor": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_debug_solve": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_mesh_set_embedding": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "vh_mesh_embed": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_mesh_embed_device": (ctypes.c_int, [_vp, _vp, _vp]),
    "vh_mesh_adjoint_forward": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _vp, _vp]),
    "vh_mesh_adjoint_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vh_mesh_gn_direction": (ctypes.c_int, [_vp, _vp, _vp, _dbl, _i32, _dbl, _vp, _vp, _P(GNStats), _vp]),
    "vh_serve_open": (ctypes.c_int, [_vp, _i32, _i32, _i32]),
    "vh_serve_close": (ctypes.c_int, [_vp]),
    "vh_serve_add": (ctypes.c_int, [_vp, _vp, _i32, _i32]),
    "vh_serve_submit": (ctypes.c_int, [_vp, _vp, _i32, _dbl, _P(ctypes.c_uint64)]),
    "vh_serve_tick": (ctypes.c_int, [_vp, _i32, _P(_i32)]),
    "vh_serve_drain": (ctypes.c_int, [_vp]),
    "vh_serve_release": (ctypes.c_int, [_vp, _vp]),
    "vh_serve_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(_i32), _P(_dbl)]),
    "vh_serve_now": (ctypes.c_int, [_vp, _P(_dbl)]),
    "vh_serve_time_kernel": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "vh_serve_reset_stats": (ctypes.c_int, [_vp]),
    "vh_serve_get_stats": (ctypes.c_int, [_vp, _P(ServeStats)]),
}


class VHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libvhpd.so (built by paper_2405_12484_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python paper_2405_12484_amd/build.py`")
    # PyTorch's HIP runtime must be the one in the process (the library shares
    # its streams and device memory); loading torch first makes the library's
    # libamdhip64.so.7 dependency resolve to it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != VH_OK:
        raise VHError(rc, _lib.vh_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One GPU; ``hbm_budget`` bytes bound the device memory of all meshes (0 = none)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        load()
        h = ctypes.c_void_p()
        _check(_lib.vh_ctx_create(ctypes.byref(h), device, hbm_budget))
        self.h = h
        self._meshes = weakref.WeakSet()
        self._server = None

    def hbm_in_use(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.vh_ctx_hbm_in_use(self.h, ctypes.byref(b)))
        return b.value

    def set_hbm_budget(self, nbytes: int):
        _check(_lib.vh_ctx_set_hbm_budget(self.h, int(nbytes)))

    def config(self) -> dict:
        c = Config()
        _check(_lib.vh_ctx_get_config(self.h, ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, **kw):
        """Change some of the fields of vh_config (see include/vhpd.h)."""
        c = Config()
        _check(_lib.vh_ctx_get_config(self.h, ctypes.byref(c)))
        for k, v in kw.items():
            if k not in dict(Config._fields_):
                raise KeyError(k)
            setattr(c, k, int(v))
        _check(_lib.vh_ctx_set_config(self.h, ctypes.byref(c)))

    def close(self):
        """Destroy the context and every mesh still open on it."""
        if self.h:
            if self._server is not None:
                self._server.close()
            for m in list(self._meshes):
                m.close()
            _lib.vh_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """One garment: rest mesh, materials, factorization and device state."""

    def __init__(self, ctx: Context, X, tets):
        self.ctx = ctx
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.nv, self.nt = self.X.shape[0], self.tets.shape[0]
        if not ctx.h:
            raise VHError(VH_ESTATE, "context is closed")
        h = ctypes.c_void_p()
        _check(_lib.vh_mesh_create(ctx.h, ctypes.byref(h), _ptr(self.X), self.nv, _ptr(self.tets), self.nt))
        self.h = h
        ctx._meshes.add(self)

    def set_params(self, gamma_s, gamma_v, mass, pinned, gravity, dt, pd_iters=10):
        gs = np.ascontiguousarray(gamma_s, dtype=np.float64)
        gv = np.ascontiguousarray(gamma_v, dtype=np.float64)
        m = np.ascontiguousarray(mass, dtype=np.float64)
        pin = np.ascontiguousarray(pinned, dtype=np.uint8)
        g = np.ascontiguousarray(gravity, dtype=np.float64)
        if gs.shape != (self.nt,) or gv.shape != (self.nt,) or m.shape != (self.nv,) or pin.shape != (self.nv,) \
                or g.shape != (3,):
            raise ValueError("parameter array shapes do not match the mesh")
        _check(_lib.vh_mesh_set_params(self.h, _ptr(gs), _ptr(gv), _ptr(m), _ptr(pin), _ptr(g), float(dt),
                                       int(pd_iters)))

    def prefactor(self, n_subdomains: int, refine_steps: int = 0, precision_mode: int = VH_PRECISION_MIXED):
        _check(_lib.vh_mesh_prefactor(self.h, int(n_subdomains), int(refine_steps), int(precision_mode)))

    def refactor(self, gamma_s, gamma_v):
        """New per-element stiffness for the prefactored mesh (factor values
        redone, structure and state kept)."""
        gs = np.ascontiguousarray(gamma_s, dtype=np.float64)
        gv = np.ascontiguousarray(gamma_v, dtype=np.float64)
        if gs.shape != (self.nt,) or gv.shape != (self.nt,):
            raise ValueError("gamma_s and gamma_v must have shape (nt,)")
        _check(_lib.vh_mesh_refactor(self.h, _ptr(gs), _ptr(gv)))

    def regime_counts(self, reset: bool = False, stream=None) -> dict:
        """Projection regime counters of the local step since the last reset."""
        c = RegimeCounts()
        _check(_lib.vh_mesh_regime_counts(self.h, ctypes.byref(c), 1 if reset else 0, _stream_ptr(stream)))
        return c.as_dict()

    def step(self, n_frames: int = 1, stream=None):
        _check(_lib.vh_mesh_step(self.h, int(n_frames), _stream_ptr(stream)))

    def step_noalloc(self, n_frames: int = 1, stream=None):
        """The step with its work buffers in the library's fixed scratch array
        (allocates no device memory)."""
        _check(_lib.vh_mesh_step_noalloc(self.h, int(n_frames), _stream_ptr(stream)))

    def read_state(self, stream=None):
        x = np.empty((self.nv, 3))
        v = np.empty((self.nv, 3))
        _check(_lib.vh_mesh_read_state(self.h, _ptr(x), _ptr(v), _stream_ptr(stream)))
        return x, v

    def write_state(self, x, v, stream=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        if x.shape != (self.nv, 3) or v.shape != (self.nv, 3):
            raise ValueError("state arrays must be [nv, 3]")
        _check(_lib.vh_mesh_write_state(self.h, _ptr(x), _ptr(v), _stream_ptr(stream)))

    def read_state_device(self, x_t, v_t, stream=None):
        """Copy the state into float64 [nv, 3] device tensors (asynchronous)."""
        for t in (x_t, v_t):
            if t.dtype.__str__() != "torch.float64" or tuple(t.shape) != (self.nv, 3) or not t.is_contiguous():
                raise ValueError("state tensors must be contiguous float64 [nv, 3]")
        _check(_lib.vh_mesh_read_state_device(self.h, ctypes.c_void_p(x_t.data_ptr()),
                                              ctypes.c_void_p(v_t.data_ptr()), _stream_ptr(stream)))

    # -- embedded points (Eq. m2y) --
    def set_embedding(self, tet, rest_xyz):
        """Points carried by the mesh: tet[n] user element indices, rest_xyz[n, 3]."""
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        rest = np.ascontiguousarray(rest_xyz, dtype=np.float64)
        if tet.ndim != 1 or rest.shape != (tet.shape[0], 3):
            raise ValueError("tet must be [n] and rest_xyz [n, 3]")
        _check(_lib.vh_mesh_set_embedding(self.h, int(tet.shape[0]), _ptr(tet), _ptr(rest)))
        self.n_embedded = int(tet.shape[0])

    def embed(self, stream=None):
        """Positions of the embedded points for the current state, [n, 3] float64."""
        out = np.empty((getattr(self, "n_embedded", 0), 3))
        _check(_lib.vh_mesh_embed(self.h, _ptr(out), _stream_ptr(stream)))
        return out

    def embed_device(self, out_t, stream=None):
        """Same into a contiguous float64 [n, 3] device tensor (asynchronous)."""
        n = getattr(self, "n_embedded", 0)
        if out_t.dtype.__str__() != "torch.float64" or tuple(out_t.shape) != (n, 3) or not out_t.is_contiguous():
            raise ValueError("output must be a contiguous float64 [n, 3] tensor")
        _check(_lib.vh_mesh_embed_device(self.h, ctypes.c_void_p(out_t.data_ptr()), _stream_ptr(stream)))

    def write_state_device(self, x_t, v_t, stream=None):
        for t in (x_t, v_t):
            if t.dtype.__str__() != "torch.float64" or tuple(t.shape) != (self.nv, 3) or not t.is_contiguous():
                raise ValueError("state tensors must be contiguous float64 [nv, 3]")
        _check(_lib.vh_mesh_write_state_device(self.h, ctypes.c_void_p(x_t.data_ptr()),
                                               ctypes.c_void_p(v_t.data_ptr()), _stream_ptr(stream)))

    def info(self) -> dict:
        i = MeshInfo()
        _check(_lib.vh_mesh_get_info(self.h, ctypes.byref(i)))
        return i.as_dict()

    PROFILE_CLASSES = ("predictor", "local", "residual", "interior_fwd", "interface", "interior_bwd",
                       "refine", "velocity")

    def profile(self, classes=()):
        """Enable HIP-event timing for the named kernel classes (empty = off)."""
        mask = 0
        for c in classes:
            mask |= 1 << self.PROFILE_CLASSES.index(c)
        _check(_lib.vh_mesh_profile(self.h, mask))

    def time_kernel(self, kernel_class: str, reps: int, stream=None):
        """Launch one kernel class `reps` times back to back (for event timing)."""
        idx = {"local": 1, "residual": 2, "interior_fwd": 3, "interface": 4, "interior_bwd": 5,
               "interior_fwd_plain": 6}[kernel_class]
        _check(_lib.vh_mesh_time_kernel(self.h, idx, int(reps), _stream_ptr(stream)))

    def profile_read(self):
        """{class: (milliseconds, timed launch groups)} since profile() or the last read."""
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        _check(_lib.vh_mesh_profile_read(self.h, _ptr(ms), _ptr(n)))
        return {c: (float(ms[i]), int(n[i])) for i, c in enumerate(self.PROFILE_CLASSES) if n[i]}

    # -- discrete adjoint with respect to gamma_s --
    def adjoint_forward(self, x0, v0, n_frames, ckpt_every=5, stream=None):
        """Run n_frames from (x0, v0) keeping checkpoints; returns x_final."""
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        xf = np.empty((self.nv, 3))
        _check(_lib.vh_mesh_adjoint_forward(self.h, _ptr(x0), _ptr(v0), int(n_frames), int(ckpt_every),
                                            _ptr(xf), _stream_ptr(stream)))
        return xf

    def adjoint_backward(self, xbar, vbar=None, stream=None):
        """dLoss/dgamma_s [nt] for dLoss/dx_final = xbar (and dLoss/dv_final = vbar)."""
        xbar = np.ascontiguousarray(xbar, dtype=np.float64)
        vb = None if vbar is None else np.ascontiguousarray(vbar, dtype=np.float64)
        g = np.empty(self.nt)
        _check(_lib.vh_mesh_adjoint_backward(self.h, _ptr(xbar), None if vb is None else _ptr(vb), _ptr(g),
                                             _stream_ptr(stream)))
        return g

    # -- per-kernel entry points (clobber the state) --
    def gn_direction(self, x_eq, x_target, kappa, max_outer=200, outer_tol=1e-8, stream=None):
        """Adjoint Gauss-Newton direction for gamma_s at the equilibrium x_eq
        (returns gradient [nt], direction [nt], stats)."""
        xe = np.ascontiguousarray(x_eq, dtype=np.float64)
        xt = np.ascontiguousarray(x_target, dtype=np.float64)
        g = np.zeros(self.nt)
        d = np.zeros(self.nt)
        st = GNStats()
        _check(_lib.vh_mesh_gn_direction(self.h, _ptr(xe), _ptr(xt), float(kappa), int(max_outer), float(outer_tol),
                                         _ptr(g), _ptr(d), ctypes.byref(st), _stream_ptr(stream)))
        return g, d, st.as_dict()

    def debug_local_step(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        T = np.empty((self.nt, 9))
        sig = np.empty((self.nt, 3))
        s = np.empty((self.nt, 3))
        _check(_lib.vh_debug_local_step(self.h, _ptr(x), _ptr(T), _ptr(sig), _ptr(s)))
        return T.reshape(self.nt, 3, 3), sig, s

    def debug_residual(self, x, y, in_solve=False):
        """r = b(x) - K x [nv][3]; in_solve: formed as the PD iterations form it
        (inside the interior forward solve) instead of by its own launch."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        r = np.empty((self.nv, 3))
        fn = _lib.vh_debug_residual_in_solve if in_solve else _lib.vh_debug_residual
        _check(fn(self.h, _ptr(x), _ptr(y), _ptr(r)))
        return r

    def debug_scatter_colored(self, x):
        """Elastic forces at x [nv][3] assembled by element colouring, and the colour count."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        f = np.empty((self.nv, 3))
        nc = ctypes.c_int32(0)
        _check(_lib.vh_debug_scatter_colored(self.h, _ptr(x), _ptr(f), ctypes.byref(nc)))
        return f, int(nc.value)

    def debug_interface_factor(self):
        """The resident interface factor values (FP64), in the plan's layout."""
        n = ctypes.c_int64(0)
        _check(_lib.vh_debug_interface_factor(self.h, None, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.float64)
        _check(_lib.vh_debug_interface_factor(self.h, _ptr(out), ctypes.byref(n)))
        return out

    def debug_solve(self, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        d = np.empty((self.nv, 3))
        _check(_lib.vh_debug_solve(self.h, _ptr(rhs), _ptr(d)))
        return d

    def close(self):
        if getattr(self, "h", None):
            if self.ctx.h:                      # a closed context already destroyed it
                _lib.vh_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The context's step server (continuous batching of step requests).

    mode "batched": each launch steps one frame of every resident mesh with a
    request waiting; "sequential": one mesh's frame per launch (plain stepping).
    """

    MODES = {"batched": 0, "sequential": 1}

    def __init__(self, ctx: Context, mode: str = "batched", max_in_flight: int = 2, max_batch: int = 0):
        if not ctx.h:
            raise VHError(VH_ESTATE, "context is closed")
        _check(_lib.vh_serve_open(ctx.h, self.MODES[mode], int(max_in_flight), int(max_batch)))
        self.ctx = ctx
        self.mode = mode
        ctx._server = self

    def add(self, mesh: Mesh, n_subdomains: int, refine_steps: int = 0):
        _check(_lib.vh_serve_add(self.ctx.h, mesh.h, int(n_subdomains), int(refine_steps)))

    def submit(self, mesh: Mesh, n_frames: int = 1, t_arrival: float = -1.0) -> int:
        t = ctypes.c_uint64()
        _check(_lib.vh_serve_submit(self.ctx.h, mesh.h, int(n_frames), float(t_arrival), ctypes.byref(t)))
        return t.value

    def tick(self, wait: bool = False) -> int:
        n = ctypes.c_int32()
        _check(_lib.vh_serve_tick(self.ctx.h, 1 if wait else 0, ctypes.byref(n)))
        return n.value

    def drain(self):
        _check(_lib.vh_serve_drain(self.ctx.h))

    def release(self, mesh: Mesh):
        _check(_lib.vh_serve_release(self.ctx.h, mesh.h))

    def poll(self, ticket: int):
        """(done, latency seconds or None)."""
        d = ctypes.c_int32()
        lat = ctypes.c_double()
        _check(_lib.vh_serve_poll(self.ctx.h, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(lat)))
        return bool(d.value), (lat.value if d.value else None)

    def now(self) -> float:
        t = ctypes.c_double()
        _check(_lib.vh_serve_now(self.ctx.h, ctypes.byref(t)))
        return t.value

    def reset_stats(self):
        _check(_lib.vh_serve_reset_stats(self.ctx.h))

    def time_kernel(self, kernel_class: str, reps: int, stream=None):
        """Launch the batched local step or residual over every resident mesh
        `reps` times back to back (for event timing)."""
        idx = {"local": 1, "residual": 2}[kernel_class]
        _check(_lib.vh_serve_time_kernel(self.ctx.h, idx, int(reps), _stream_ptr(stream)))

    def stats(self) -> dict:
        st = ServeStats()
        _check(_lib.vh_serve_get_stats(self.ctx.h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.ctx is not None and self.ctx.h and self.ctx._server is self:
            rc = _lib.vh_serve_close(self.ctx.h)
            self.ctx._server = None
            self.ctx = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
