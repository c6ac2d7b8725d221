"""Seeded synthetic packings for the contact-force solve.

This module only draws inputs: particle positions, radii, masses, moments
of inertia, velocities, external forces and the confining walls.  It holds
none of the solver's arithmetic, so the CPU oracle and the HIP path can both
be fed from it.

The paper's own packings (dense 2D systems made by an unpublished
compression protocol, Sec. 4.1 and Fig. 10) are not available; the lattices
below stand in for them with the same structure: polydisperse disks or
spheres in a rigid box, densely packed, with a connected contact network.

Recipe (all FP64, numpy PCG64):
  * 2D: jittered triangular lattice, spacing s = 2.05,
        x = s (a + (b mod 2)/2), y = s (sqrt(3)/2) b, id = b*nx + a.
  * 3D: jittered simple-cubic lattice, x = s (a, b, c), id = (c*ny + b)*nx + a.
  * draw order: jitter U[-0.05, 0.05] per coordinate (N*d), radii
    U[0.8, 1.2] (N), velocities N(0, sigma_v^2) per component (N*d).
  * density 1: m = pi r^2 (2D) or 4/3 pi r^3 (3D); solid disk I = m r^2 / 2,
    solid sphere I = 2 m r^2 / 5; angular velocity 0.
  * external force F = -m g e_y (2D) or -m g e_z (3D), no external torque.
  * walls: one axis-aligned plane per box face, placed one mean radius
    outside the lattice extent; a wall is the plane {x : nu.x = o} with
    unit normal nu pointing into the box.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SPACING = 2.05
JITTER = 0.05
R_LO, R_HI = 0.8, 1.2
WALL_MARGIN = 1.0


@dataclasses.dataclass
class Packing:
    """A packing in structure-of-arrays form (component-major, a[k, i])."""

    dim: int
    x: np.ndarray        # (dim, N) positions
    v: np.ndarray        # (dim, N) velocities
    w: np.ndarray        # (dr, N) angular velocities (dr = 1 in 2D, 3 in 3D)
    r: np.ndarray        # (N,) radii
    m: np.ndarray        # (N,) masses
    inertia: np.ndarray  # (N,) moments of inertia
    f: np.ndarray        # (dim, N) external forces
    t: np.ndarray        # (dr, N) external torques
    wall_normal: np.ndarray    # (W, dim) unit normals into the box
    wall_offset: np.ndarray    # (W,) plane offsets: nu . x = o
    wall_velocity: np.ndarray  # (W, dim) translation velocities
    box_lo: np.ndarray   # (dim,) simulation box, the root region of the partition
    box_hi: np.ndarray   # (dim,)
    # benchmark boundary conditions (Sec. 4.1): bit k of `periodic` makes axis
    # k periodic over [box_lo_k, box_hi_k); a wall with wall_inv_mass > 0 is a
    # body of that inverse mass pushed with wall_force along its normal
    periodic: int = 0
    wall_inv_mass: Optional[np.ndarray] = None   # (W,)
    wall_force: Optional[np.ndarray] = None      # (W,)

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    @property
    def n_walls(self) -> int:
        return int(self.wall_offset.shape[0])

    def copy(self) -> "Packing":
        return Packing(**{f.name: (np.array(getattr(self, f.name), copy=True)
                                   if isinstance(getattr(self, f.name), np.ndarray)
                                   else getattr(self, f.name))
                          for f in dataclasses.fields(self)})


def _box_walls(lo: np.ndarray, hi: np.ndarray, top_velocity: Optional[np.ndarray]):
    """Axis-aligned walls: for each axis k a lower wall (nu = +e_k, o = lo_k)
    and an upper wall (nu = -e_k, o = -hi_k).  The upper wall of the last
    axis optionally moves with `top_velocity`."""
    dim = lo.shape[0]
    normals, offsets, vels = [], [], []
    for k in range(dim):
        e = np.zeros(dim)
        e[k] = 1.0
        normals.append(e.copy())
        offsets.append(lo[k])
        vels.append(np.zeros(dim))
        normals.append(-e)
        offsets.append(-hi[k])
        vels.append(np.zeros(dim))
    if top_velocity is not None:
        vels[-1] = np.asarray(top_velocity, dtype=np.float64)
    return (np.array(normals, dtype=np.float64), np.array(offsets, dtype=np.float64),
            np.array(vels, dtype=np.float64))


def lattice_2d(nx: int, ny: int, seed: int, *, n: Optional[int] = None,
               gravity: float = 1.0, sigma_v: float = 0.01) -> Packing:
    """Jittered triangular lattice of nx*ny disks (the first `n` sites if given)."""
    total = nx * ny
    n = total if n is None else int(n)
    assert 0 < n <= total
    rng = np.random.Generator(np.random.PCG64(seed))
    b, a = np.divmod(np.arange(n), nx)
    x = np.empty((2, n))
    x[0] = SPACING * (a + 0.5 * (b % 2))
    x[1] = SPACING * (math.sqrt(3.0) / 2.0) * b
    x += rng.uniform(-JITTER, JITTER, size=(n, 2)).T
    r = rng.uniform(R_LO, R_HI, size=n)
    v = rng.normal(0.0, sigma_v, size=(n, 2)).T.copy()
    m = math.pi * r * r
    inertia = 0.5 * m * r * r
    f = np.zeros((2, n))
    f[1] = -m * gravity
    rows = (n + nx - 1) // nx
    lo = np.array([-WALL_MARGIN, -WALL_MARGIN])
    hi = np.array([SPACING * (nx - 0.5) + WALL_MARGIN,
                   SPACING * (math.sqrt(3.0) / 2.0) * (rows - 1) + WALL_MARGIN])
    wn, wo, wv = _box_walls(lo, hi, None)
    return Packing(2, np.ascontiguousarray(x), np.ascontiguousarray(v), np.zeros((1, n)),
                   r, m, inertia, f, np.zeros((1, n)), wn, wo, wv, lo, hi)


def sheared_box_2d(nx: int, ny: int, seed: int, *, pressure: float = 0.25,
                   shear_velocity: float = 0.0, sigma_v: float = 0.01) -> Packing:
    """The setup of the paper's performance and physics tests (Sec. 4.1,
    Fig. 10; Sec. 4.4): a jittered triangular lattice of nx*ny disks
    (generator of lattice_2d, no gravity) periodic in x over nx spacings,
    between a bottom and a top wall that each push with `pressure` times the
    box width along their normal (walls of finite mass: one row of disks of
    the mean radius, nx pi) and slide along x at -shear_velocity (bottom) and
    +shear_velocity (top)."""
    pk = lattice_2d(nx, ny, seed, gravity=0.0, sigma_v=sigma_v)
    Lx = SPACING * nx
    lo = np.array([0.0, pk.box_lo[1]])
    hi = np.array([Lx, pk.box_hi[1]])
    x = pk.x.copy()
    x[0] = np.mod(x[0] - lo[0], Lx) + lo[0]     # the row offsets wrap into [0, Lx)
    wn = np.array([[0.0, 1.0], [0.0, -1.0]])
    wo = np.array([lo[1], -hi[1]])
    wv = np.array([[-shear_velocity, 0.0], [shear_velocity, 0.0]])
    mass = nx * math.pi
    return Packing(2, np.ascontiguousarray(x), pk.v, pk.w, pk.r, pk.m, pk.inertia, pk.f, pk.t,
                   wn, wo, wv, lo, hi, periodic=1,
                   wall_inv_mass=np.array([1.0 / mass, 1.0 / mass]),
                   wall_force=np.array([pressure * Lx, pressure * Lx]))


def lattice_3d(nx: int, ny: int, nz: int, seed: int, *, gravity: float = 0.0,
               sigma_v: float = 0.01, top_velocity: float = 0.0) -> Packing:
    """Jittered simple-cubic lattice of nx*ny*nz spheres; the top (z) wall
    moves with velocity (0, 0, -top_velocity)."""
    n = nx * ny * nz
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.arange(n)
    c, rem = np.divmod(idx, nx * ny)
    b, a = np.divmod(rem, nx)
    x = np.empty((3, n))
    x[0] = SPACING * a
    x[1] = SPACING * b
    x[2] = SPACING * c
    x += rng.uniform(-JITTER, JITTER, size=(n, 3)).T
    r = rng.uniform(R_LO, R_HI, size=n)
    v = rng.normal(0.0, sigma_v, size=(n, 3)).T.copy()
    m = (4.0 / 3.0) * math.pi * r ** 3
    inertia = 0.4 * m * r * r
    f = np.zeros((3, n))
    f[2] = -m * gravity
    lo = np.full(3, -WALL_MARGIN)
    hi = np.array([SPACING * (nx - 1), SPACING * (ny - 1), SPACING * (nz - 1)]) + WALL_MARGIN
    wn, wo, wv = _box_walls(lo, hi, np.array([0.0, 0.0, -top_velocity]))
    return Packing(3, np.ascontiguousarray(x), np.ascontiguousarray(v), np.zeros((3, n)),
                   r, m, inertia, f, np.zeros((3, n)), wn, wo, wv, lo, hi)


def uneven_batch(count: int, seed: int = 3, n_lo: int = 256, n_hi: int = 65536,
                 mu_lo: float = 0.1, mu_hi: float = 0.6, base_seed: int = 3000):
    """`count` independent 2D packings with N log-uniform in [n_lo, n_hi] and a
    friction coefficient uniform in [mu_lo, mu_hi] each.  Packing b is a
    triangular lattice with ceil(sqrt(N_b)) sites per row, filled row by row
    to N_b sites, drawn with seed base_seed + b."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    mus = rng.uniform(mu_lo, mu_hi, size=count)
    packs: List[Packing] = []
    for b in range(count):
        nb = int(sizes[b])
        nx = int(math.ceil(math.sqrt(nb)))
        ny = (nb + nx - 1) // nx
        packs.append(lattice_2d(nx, ny, base_seed + b, n=nb))
    return packs, mus


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def pair_mu(seed: int, ci: np.ndarray, cj: np.ndarray, lo: float = 0.2, hi: float = 0.4):
    """Friction coefficient of each contact pair (i, j), uniform in [lo, hi),
    from a stateless hash of (seed, i, j): the same pair gets the same value
    whatever list it appears in."""
    ci = np.asarray(ci, dtype=np.uint64)
    cj = np.asarray(cj, dtype=np.uint64)
    h = _splitmix64(_splitmix64(_splitmix64(np.full(ci.shape, seed, dtype=np.uint64)) ^ ci) ^ cj)
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def chain_2d(n: int, force: float, radius: float = 1.0) -> Packing:
    """n touching equal disks on the x axis between two walls; the first disk
    is pushed with `force` towards the fixed wall at the far end (Fig. 13a
    setup).  No gravity, all velocities zero."""
    x = np.zeros((2, n))
    x[0] = radius + 2.0 * radius * np.arange(n)
    r = np.full(n, radius)
    m = math.pi * r * r
    inertia = 0.5 * m * r * r
    f = np.zeros((2, n))
    f[0, 0] = force
    lo = np.array([0.0, -radius])
    hi = np.array([2.0 * radius * n, radius])
    # only the two end walls (x); no floor, so the chain is the whole network
    wn = np.array([[1.0, 0.0], [-1.0, 0.0]])
    wo = np.array([lo[0], -hi[0]])
    wv = np.zeros((2, 2))
    return Packing(2, x, np.zeros((2, n)), np.zeros((1, n)), r, m, inertia, f,
                   np.zeros((1, n)), wn, wo, wv, lo, hi)


def column_2d(n: int, gravity: float = 1.0, radius: float = 1.0) -> Packing:
    """A vertical column of n touching equal disks resting on the floor."""
    x = np.zeros((2, n))
    x[0] = 0.0
    x[1] = radius + 2.0 * radius * np.arange(n)
    r = np.full(n, radius)
    m = math.pi * r * r
    inertia = 0.5 * m * r * r
    f = np.zeros((2, n))
    f[1] = -m * gravity
    lo = np.array([-2.0 * radius, 0.0])
    hi = np.array([2.0 * radius, 2.0 * radius * n + 1.0])
    wn = np.array([[0.0, 1.0]])
    wo = np.array([0.0])
    wv = np.zeros((1, 2))
    return Packing(2, x, np.zeros((2, n)), np.zeros((1, n)), r, m, inertia, f,
                   np.zeros((1, n)), wn, wo, wv, lo, hi)


def config(name: str) -> Packing:
    """The named workloads (the bench's and the tests' large cases)."""
    if name == "disks_1k":
        return lattice_2d(32, 32, 1000)
    if name == "disks_262k":
        return lattice_2d(512, 512, 1001)
    if name == "spheres_1m":
        return lattice_3d(128, 128, 64, 1002, gravity=0.0, top_velocity=1e-3)
    if name == "disks_65k":
        return lattice_2d(256, 256, 1004)
    raise KeyError(name)
