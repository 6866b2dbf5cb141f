"""Structured tetrahedral meshes and seeded per-element materials.

Workloads (all sizes in SI units):

* ``box``  -- an ``nx x ny x nz`` grid of cubic hex cells of edge ``h``, each
  split into 5 tetrahedra.  The default (10 x 10 x 2, h = 0.01 m) has 1,000 tets
  and 363 vertices; the row of vertices at the top (largest y) is pinned and
  gravity points along -y.
* ``shell`` -- a thin cylindrical shell (axis z, mid radius 0.25 m, height
  0.6 m) with ``n_theta`` cells around, ``n_z`` cells up and 2 radial cell
  layers, each hex split into 5 tetrahedra.  The default (320 x 122 x 2) has
  390,400 tets and 118,080 vertices, a stand-in at the scale of the paper's
  sweater scene (Table 1: 389K tets, dt = 1/150 s).  The ring of vertices at
  the top (the collar, z = 0.6 m) is pinned and gravity points along -z.

The 5-tet split alternates with the parity of the hex index so neighbouring
hexes share face diagonals (the paper splits voxels into tets, Sec. 4; the
5-tet variant is this workload's choice).  Hex corners are numbered
``dx + 2 dy + 4 dz``.  Every tet is oriented to positive volume.

Materials: ``gamma_s`` (strain weight) is log-normal, ``gamma_v`` (volume
weight) is uniform in [1e3, 1e4]; both are drawn from
``numpy.random.Generator(PCG64(seed))`` in tet order, gamma_s first.  Masses are
lumped as rho * V_e / 4 per corner with rho = 300 kg/m^3 (a bulk density for
knit fabric; the paper lumps yarn mass instead, Eq. mass_fit, which needs yarn
curves that these synthetic meshes do not have).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

RHO_DEFAULT = 300.0
GRAVITY = 9.81

# Corner tets of a hex for even and odd parity of (i + j + k); the fifth tet is
# the central one.  Corner numbering: dx + 2 dy + 4 dz.
_SPLIT_EVEN = np.array([[0, 1, 2, 4], [3, 1, 2, 7], [5, 1, 4, 7], [6, 2, 4, 7], [1, 2, 4, 7]])
_SPLIT_ODD = np.array([[1, 0, 3, 5], [2, 0, 3, 6], [4, 0, 5, 6], [7, 3, 5, 6], [0, 3, 5, 6]])


@dataclasses.dataclass
class Problem:
    """One garment: rest mesh, materials, masses, pins and the step settings."""

    name: str
    X: np.ndarray          # (nv, 3) float64 rest positions
    tets: np.ndarray       # (nt, 4) int32, positively oriented
    gamma_s: np.ndarray    # (nt,) float64
    gamma_v: np.ndarray    # (nt,) float64
    mass: np.ndarray       # (nv,) float64 lumped masses
    pinned: np.ndarray     # (nv,) uint8, 1 = Dirichlet at rest position
    gravity: np.ndarray    # (3,) float64
    dt: float
    pd_iters: int
    n_subdomains: int
    frames: int
    hex_index: np.ndarray | None = None  # (nt, 3) int32 (i, j, k) of the parent hex

    @property
    def nv(self) -> int:
        return int(self.X.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])

    def initial_state(self):
        """Rest positions and zero velocity."""
        return self.X.copy(), np.zeros_like(self.X)


def _signed_volume6(X, tets):
    a = X[tets[:, 1]] - X[tets[:, 0]]
    b = X[tets[:, 2]] - X[tets[:, 0]]
    c = X[tets[:, 3]] - X[tets[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def _split_hexes(corner_ids, parity):
    """corner_ids: (nh, 8) vertex ids of each hex; parity: (nh,) 0/1."""
    nh = corner_ids.shape[0]
    out = np.empty((nh, 5, 4), dtype=np.int64)
    even = parity == 0
    out[even] = corner_ids[even][:, _SPLIT_EVEN]
    out[~even] = corner_ids[~even][:, _SPLIT_ODD]
    return out.reshape(nh * 5, 4)


def _orient(X, tets):
    vol6 = _signed_volume6(X, tets)
    neg = vol6 < 0
    t = tets.copy()
    t[neg, 1], t[neg, 2] = tets[neg, 2], tets[neg, 1]
    return t


def _lumped_mass(X, tets, rho):
    vol = _signed_volume6(X, tets) / 6.0
    m = np.zeros(X.shape[0])
    for c in range(4):
        np.add.at(m, tets[:, c], rho * vol / 4.0)
    return m


def box_grid(nx=10, ny=10, nz=2, h=0.01):
    """Vertices (nv,3), tets (nt,4) and the parent hex index of each tet."""
    gx, gy, gz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    X = np.stack([gx, gy, gz], axis=-1).reshape(-1, 3).astype(np.float64) * h

    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    hi, hj, hk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    hi, hj, hk = hi.ravel(), hj.ravel(), hk.ravel()
    corners = np.stack(
        [vid(hi + dx, hj + dy, hk + dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], axis=1
    )
    parity = (hi + hj + hk) % 2
    tets = _orient(X, _split_hexes(corners, parity))
    hex_index = np.repeat(np.stack([hi, hj, hk], axis=1), 5, axis=0)
    return X, tets.astype(np.int32), hex_index.astype(np.int32)


def cylinder_shell(n_theta=320, n_z=122, n_r=2, radius=0.25, height=0.6):
    """Thin cylindrical shell around the z axis, base at z = 0.

    Radial cell size equals the circumferential one at mid radius; n_theta must
    be even so the 5-tet split parity matches across the seam.
    """
    if n_theta % 2:
        raise ValueError("n_theta must be even")
    dr = 2.0 * math.pi * radius / n_theta
    radii = radius + (np.arange(n_r + 1) - n_r / 2.0) * dr
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    zs = height * np.arange(n_z + 1) / n_z
    # vertex (it, jz, kr) -> id
    T, Z, R = np.meshgrid(th, zs, radii, indexing="ij")
    X = np.stack([R * np.cos(T), R * np.sin(T), Z], axis=-1).reshape(-1, 3)

    def vid(i, j, k):
        return ((i % n_theta) * (n_z + 1) + j) * (n_r + 1) + k

    hi, hj, hk = np.meshgrid(np.arange(n_theta), np.arange(n_z), np.arange(n_r), indexing="ij")
    hi, hj, hk = hi.ravel(), hj.ravel(), hk.ravel()
    # local hex axes: dx -> theta, dy -> z, dz -> r
    corners = np.stack(
        [vid(hi + dx, hj + dy, hk + dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], axis=1
    )
    parity = (hi + hj + hk) % 2
    tets = _orient(X, _split_hexes(corners, parity))
    hex_index = np.repeat(np.stack([hi, hj, hk], axis=1), 5, axis=0)
    return X, tets.astype(np.int32), hex_index.astype(np.int32)


def make_box_problem(seed=1, nx=10, ny=10, nz=2, h=0.01, rho=RHO_DEFAULT, dt=1.0 / 150.0,
                     pd_iters=10, n_subdomains=4, frames=20, name="box"):
    """Hex-grid slab with the top (max y) row of vertices pinned, gravity -y."""
    X, tets, hexi = box_grid(nx, ny, nz, h)
    rng = np.random.Generator(np.random.PCG64(seed))
    nt = tets.shape[0]
    gamma_s = np.exp(math.log(1e4) + 0.5 * rng.standard_normal(nt))
    gamma_v = rng.uniform(1e3, 1e4, nt)
    pinned = (np.abs(X[:, 1] - X[:, 1].max()) < 1e-12).astype(np.uint8)
    return Problem(name=name, X=X, tets=tets, gamma_s=gamma_s, gamma_v=gamma_v,
                   mass=_lumped_mass(X, tets, rho), pinned=pinned,
                   gravity=np.array([0.0, -GRAVITY, 0.0]), dt=dt, pd_iters=pd_iters,
                   n_subdomains=n_subdomains, frames=frames, hex_index=hexi)


def make_shell_problem(seed=2, n_theta=320, n_z=122, n_r=2, radius=0.25, height=0.6,
                       rho=RHO_DEFAULT, dt=1.0 / 150.0, pd_iters=10, n_subdomains=128,
                       frames=10, band_cells=20, name="shell"):
    """Cylindrical shell with vertical stripe bands of stiffness x{1,4,16},
    log-normal noise (sigma 0.3), collar ring pinned, gravity -z."""
    X, tets, hexi = cylinder_shell(n_theta, n_z, n_r, radius, height)
    rng = np.random.Generator(np.random.PCG64(seed))
    nt = tets.shape[0]
    level = np.array([1.0, 4.0, 16.0])[(hexi[:, 0] // band_cells) % 3]
    gamma_s = 1e4 * level * np.exp(0.3 * rng.standard_normal(nt))
    gamma_v = rng.uniform(1e3, 1e4, nt)
    pinned = (np.abs(X[:, 2] - height) < 1e-9).astype(np.uint8)
    return Problem(name=name, X=X, tets=tets, gamma_s=gamma_s, gamma_v=gamma_v,
                   mass=_lumped_mass(X, tets, rho), pinned=pinned,
                   gravity=np.array([0.0, 0.0, -GRAVITY]), dt=dt, pd_iters=pd_iters,
                   n_subdomains=n_subdomains, frames=frames, hex_index=hexi)


def serving_garment_sizes(n_garments=64, seed=6, lo=5e3, hi=2e5):
    """Tet-count targets, log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_garments))).astype(np.int64)


def serving_shell_problem(target_tets, seed, radius=0.25, height=0.6, leaf_verts=915):
    """A shell garment with about ``target_tets`` tets (10 tets per surface cell)."""
    h = math.sqrt(10.0 * 2.0 * math.pi * radius * height / float(target_tets))
    n_theta = max(4, 2 * int(round(math.pi * radius / h)))
    n_z = max(2, int(round(height / h)))
    p = make_shell_problem(seed=seed, n_theta=n_theta, n_z=n_z, radius=radius, height=height,
                           frames=150, name=f"shell{target_tets}")
    # the fewest power-of-two subdomains with at most about leaf_verts free
    # vertices each (the 390,400-tet shell's 128 subdomains hold 915)
    n_free = int((p.pinned == 0).sum())
    d = 2 ** max(0, int(math.ceil(math.log2(max(1.0, n_free / leaf_verts)))))
    p.n_subdomains = d
    return p


def problem_by_name(name: str) -> Problem:
    """The named workloads: 'box' (1,000 tets), 'shell' (390,400 tets),
    'slab' (20,000 tets), 'shell_small' (a 4,800-tet shell for quick GPU checks)."""
    if name == "box":
        return make_box_problem()
    if name == "shell":
        return make_shell_problem()
    if name == "slab":
        return make_box_problem(seed=3, nx=40, ny=25, nz=4, h=0.01, n_subdomains=8, frames=30,
                                name="slab")
    if name == "shell_small":
        return make_shell_problem(seed=4, n_theta=40, n_z=12, n_subdomains=8, frames=20,
                                  name="shell_small")
    raise KeyError(name)
