"""Seeded synthetic inputs: meshes, materials and initial states.

This module holds no arithmetic of the solver.  It builds the procedural
stand-ins for the paper's meshes (its Armadillo, puffer balls, letters ...
are not available): Kuhn-split hexahedral beams and voxelised spheres, their
per-tetrahedron materials, and seeded initial positions and velocities.  The
oracle and the HIP library both consume these inputs; neither shares any
other code.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the n-th output (n >= 0) of a
generator whose state is ``s`` is ``fin(s + (n + 1) * GAMMA)`` with the
finaliser ``fin`` below.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def sm64_fin(z: int) -> int:
    """SplitMix64 output finaliser (variant 13 of Stafford's mix)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sm64(x: int) -> int:
    """One SplitMix64 step from state ``x``: returns the output."""
    return sm64_fin((x + GAMMA) & MASK64)


class SplitMix64:
    """Sequential SplitMix64 stream."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        return sm64_fin(self.state)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def randint(self, lo: int, hi: int) -> int:
        """Integer in [lo, hi] by the multiply-high map of the top 32 bits."""
        n = hi - lo + 1
        return lo + (((self.next_u64() >> 32) * n) >> 32)

    def uniform_array(self, n: int, lo: float, hi: float) -> np.ndarray:
        return np.array([self.uniform_range(lo, hi) for _ in range(n)], dtype=np.float64)


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

# The six tetrahedra of the Kuhn (Freudenthal) split of a unit cube: each is
# the monotone corner path 000 -> +e_p0 -> +e_p0+e_p1 -> 111 for one
# permutation p of the three axes, taken in lexicographic order.
def _kuhn_corner_paths():
    paths = []
    for p in itertools.permutations(range(3)):
        c = [0, 0, 0]
        path = [tuple(c)]
        for ax in p:
            c[ax] = 1
            path.append(tuple(c))
        paths.append(path)
    return paths


KUHN_PATHS = _kuhn_corner_paths()


def _orient(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap the last two corners of every tet with a negative signed volume."""
    d = X[tets[:, 1:]] - X[tets[:, :1]]
    det = np.linalg.det(d)
    neg = det < 0
    t = tets.copy()
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


@dataclass
class Mesh:
    X: np.ndarray          # (V, 3) float64 rest positions
    tets: np.ndarray       # (T, 4) int32, positive orientation
    pinned: np.ndarray     # (V,) uint8
    name: str = ""
    body: np.ndarray | None = None  # (V,) int32 body id

    @property
    def nV(self) -> int:
        return self.X.shape[0]

    @property
    def nT(self) -> int:
        return self.tets.shape[0]


def beam_mesh(n_long: int, n_a: int, n_b: int, cell: float = 0.05) -> Mesh:
    """Hexahedral beam of n_long x n_a x n_b cubes, long axis along world x.

    Vertex (ix, iy, iz) has id ``iz + (n_b+1)*(iy + (n_a+1)*ix)`` so that the
    long axis varies slowest; cube (ix, iy, iz) owns tets
    ``6*((ix*n_a + iy)*n_b + iz) + p``.  Vertices at x = 0 are pinned.
    """
    nx, ny, nz = n_long, n_a, n_b
    ix, iy, iz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    X = np.stack([ix, iy, iz], axis=-1).reshape(-1, 3).astype(np.float64) * cell

    def vid(a, b, c):
        return c + (nz + 1) * (b + (ny + 1) * a)

    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    tets = np.empty((cx.size, 6, 4), dtype=np.int64)
    for p, path in enumerate(KUHN_PATHS):
        for c, (dx, dy, dz) in enumerate(path):
            tets[:, p, c] = vid(cx + dx, cy + dy, cz + dz)
    tets = tets.reshape(-1, 4)
    tets = _orient(X, tets).astype(np.int32)
    pinned = (X[:, 0] == 0.0).astype(np.uint8)
    return Mesh(X=X, tets=tets, pinned=pinned, name=f"beam{nx}x{ny}x{nz}")


def sphere_mesh(radius: float, cell: float) -> Mesh:
    """Solid sphere voxelised on a ``cell`` grid (a cube is kept when its
    centre lies strictly inside the sphere), each cube Kuhn-split.  Vertices
    are the used cube corners, numbered lexicographically (x slowest).
    Coordinates are in the sphere's local frame (centre at the origin)."""
    n = int(math.ceil(radius / cell))
    r = np.arange(-n, n)
    cx, cy, cz = np.meshgrid(r, r, r, indexing="ij")
    cen = (np.stack([cx, cy, cz], -1) + 0.5) * cell
    keep = (cen ** 2).sum(-1) < radius * radius
    cx, cy, cz = cx[keep], cy[keep], cz[keep]
    m = 2 * n + 1  # corner index range [-n, n]

    def cid(a, b, c):
        return ((a + n) * m + (b + n)) * m + (c + n)

    tets = np.empty((cx.size, 6, 4), dtype=np.int64)
    for p, path in enumerate(KUHN_PATHS):
        for c, (dx, dy, dz) in enumerate(path):
            tets[:, p, c] = cid(cx + dx, cy + dy, cz + dz)
    tets = tets.reshape(-1, 4)
    used = np.unique(tets)
    remap = np.full(m ** 3, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    tets = remap[tets]
    a = used // (m * m) - n
    b = (used // m) % m - n
    c = used % m - n
    X = np.stack([a, b, c], -1).astype(np.float64) * cell
    tets = _orient(X, tets).astype(np.int32)
    return Mesh(X=X, tets=tets, pinned=np.zeros(X.shape[0], np.uint8), name=f"sphere_r{radius}_c{cell}")


def concat_meshes(meshes: list[Mesh], offsets: list[np.ndarray] | None = None) -> Mesh:
    """Disjoint union; body[v] records which input mesh vertex v came from."""
    Xs, Ts, Ps, Bs = [], [], [], []
    base = 0
    for k, m in enumerate(meshes):
        X = m.X + (offsets[k] if offsets is not None else 0.0)
        Xs.append(X)
        Ts.append(m.tets.astype(np.int64) + base)
        Ps.append(m.pinned)
        Bs.append(np.full(m.nV, k, np.int32))
        base += m.nV
    return Mesh(X=np.concatenate(Xs), tets=np.concatenate(Ts).astype(np.int32),
                pinned=np.concatenate(Ps), name="+".join(m.name for m in meshes),
                body=np.concatenate(Bs))


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------

@dataclass
class Scene:
    mesh: Mesh
    E: np.ndarray            # (T,) Young's modulus [Pa]
    nu: np.ndarray           # (T,) Poisson ratio
    rho: np.ndarray          # (T,) density [kg/m^3]
    x0: np.ndarray           # (V, 3) positions at the start of step 1
    v0: np.ndarray           # (V, 3) velocities at the start of step 1
    dt: float = 1.0 / 120.0
    gravity: tuple = (0.0, -9.8, 0.0)
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # rows (n, c): n.x >= c
    d_hat: float = 1e-3
    kappa: float = 1e4
    steps: int = 1
    name: str = ""


def _per_tet(val, nT):
    return np.full(nT, float(val), dtype=np.float64)


def jitter(mesh: Mesh, amp: float, seed: int) -> np.ndarray:
    """Rest positions plus U(-amp, amp) on every coordinate of free vertices,
    drawn vertex-major (x, y, z) from one SplitMix64 stream."""
    g = SplitMix64(seed)
    x = mesh.X.copy()
    for v in range(mesh.nV):
        if mesh.pinned[v]:
            continue
        for d in range(3):
            x[v, d] += g.uniform_range(-amp, amp)
    return x


def twist_velocity(mesh: Mesh, amplitude: float = 2.0) -> np.ndarray:
    """Velocity of a torsion about the beam's long axis: angular rate
    amplitude * sin(pi s / (2 L)) at distance s from the pinned end."""
    X = mesh.X
    L = X[:, 0].max()
    cy = 0.5 * (X[:, 1].min() + X[:, 1].max())
    cz = 0.5 * (X[:, 2].min() + X[:, 2].max())
    om = amplitude * np.sin(np.pi * X[:, 0] / (2.0 * L))
    v = np.zeros_like(X)
    # omega e_x cross (0, y - cy, z - cz) = (0, -(z - cz), (y - cy)) * omega
    v[:, 1] = -om * (X[:, 2] - cz)
    v[:, 2] = om * (X[:, 1] - cy)
    v[mesh.pinned.astype(bool)] = 0.0
    return v


def twisted_positions(mesh: Mesh, total_angle: float = 0.3) -> np.ndarray:
    """Positions of the beam with each cross-section at distance s from the
    pinned end turned by total_angle * s / L about the long axis (a prescribed
    deformed configuration, no solve)."""
    X = mesh.X
    L = X[:, 0].max()
    cy = 0.5 * (X[:, 1].min() + X[:, 1].max())
    cz = 0.5 * (X[:, 2].min() + X[:, 2].max())
    th = total_angle * X[:, 0] / L
    c, s = np.cos(th), np.sin(th)
    x = X.copy()
    x[:, 1] = cy + c * (X[:, 1] - cy) - s * (X[:, 2] - cz)
    x[:, 2] = cz + s * (X[:, 1] - cy) + c * (X[:, 2] - cz)
    return x


def tiny_beam(seed: int = 0, E: float = 1e6, nu: float = 0.4) -> Scene:
    """4x4 cross-section, 16 long, 0.05 m cells (425 vertices, 1536 tets),
    one step from rest with a 1e-6 m jitter on the free vertices."""
    m = beam_mesh(16, 4, 4, 0.05)
    return Scene(mesh=m, E=_per_tet(E, m.nT), nu=_per_tet(nu, m.nT), rho=_per_tet(1000.0, m.nT),
                 x0=jitter(m, 1e-6, seed), v0=np.zeros_like(m.X), steps=1, name="tiny_beam_4x4x16")


def beam_scene(n_long: int, n_a: int, n_b: int, E: float, nu: float = 0.45, twist: float = 2.0,
               steps: int = 10, cell: float = 0.05) -> Scene:
    """Pinned beam with an initial sinusoidal twist about its long axis."""
    m = beam_mesh(n_long, n_a, n_b, cell)
    return Scene(mesh=m, E=_per_tet(E, m.nT), nu=_per_tet(nu, m.nT), rho=_per_tet(1000.0, m.nT),
                 x0=m.X.copy(), v0=twist_velocity(m, twist), steps=steps,
                 name=f"beam_{n_a}x{n_b}x{n_long}_E{E:g}")


def single_beam(E: float = 1e5) -> Scene:
    """16x16 cross-section, 128 long (37,281 vertices, 196,608 tets)."""
    return beam_scene(128, 16, 16, E)


def diff_beam(seed: int = 0):
    """16x16x64 beam (18,785 vertices, 98,304 tets) with per-tet log E drawn
    as log(1e6) + U(-0.3, 0.3), plus a seeded tip target.  Returns
    (scene, log_E, target)."""
    m = beam_mesh(64, 16, 16, 0.05)
    g = SplitMix64(seed)
    logE = math.log(1e6) + g.uniform_array(m.nT, -0.3, 0.3)
    L = m.X[:, 0].max()
    tip = m.X[m.X[:, 0] == L].mean(0)
    target = tip + g.uniform_array(3, -0.1, 0.1) * L
    sc = Scene(mesh=m, E=np.exp(logE), nu=_per_tet(0.45, m.nT), rho=_per_tet(1000.0, m.nT),
               x0=m.X.copy(), v0=np.zeros_like(m.X), steps=30, name="diff_beam_16x16x64")
    return sc, logE, target


def batched_beams(n: int = 256, seed: int = 0):
    """n independent beams; per beam (in draw order) cross-section a, b in
    U{4..24}, length in U{16..96}, E log-uniform in [1e4, 1e7], nu in
    U[0.3, 0.48].  Returns a list of (n_long, n_a, n_b, E, nu)."""
    g = SplitMix64(seed)
    out = []
    for _ in range(n):
        a = g.randint(4, 24)
        b = g.randint(4, 24)
        L = g.randint(16, 96)
        E = math.exp(g.uniform_range(math.log(1e4), math.log(1e7)))
        nu = g.uniform_range(0.3, 0.48)
        out.append((L, a, b, E, nu))
    return out


def contact_scene(seed: int = 0, radius: float = 0.3, cell: float = 0.01, n_spheres: int = 10) -> Scene:
    """Spheres dropped into a 2 x 2 x 4 m box (z up) with a floor and four
    walls; the first half stiff (E = 2e6), the second half 20x softer."""
    g = SplitMix64(seed)
    lo = radius + 0.01
    cents = []
    while len(cents) < n_spheres:
        c = np.array([g.uniform_range(lo, 2.0 - lo), g.uniform_range(lo, 2.0 - lo),
                      g.uniform_range(lo, 4.0 - lo)])
        if all(np.linalg.norm(c - d) >= 2 * radius + 0.01 for d in cents):
            cents.append(c)
    sph = sphere_mesh(radius, cell)
    m = concat_meshes([sph] * n_spheres, offsets=cents)
    body_t = m.body[m.tets[:, 0]]
    E = np.where(body_t < n_spheres // 2, 2e6, 1e5)
    planes = np.array([[0, 0, 1, 0.0], [1, 0, 0, 0.0], [-1, 0, 0, -2.0],
                       [0, 1, 0, 0.0], [0, -1, 0, -2.0]], dtype=np.float64)
    return Scene(mesh=m, E=E.astype(np.float64), nu=_per_tet(0.45, m.nT), rho=_per_tet(1000.0, m.nT),
                 x0=m.X.copy(), v0=np.zeros_like(m.X), gravity=(0.0, 0.0, -9.8), planes=planes,
                 steps=120, name="spheres_in_box")


def sphere_on_floor(radius: float = 0.05, cell: float = 0.01, gap: float = 6e-4, speed: float = 1.0,
                    E: float = 1e5, nu: float = 0.45) -> Scene:
    """One voxel sphere whose lowest vertex sits `gap` above the plane z = 0,
    moving down at `speed`; gravity along -z, IPC barrier d_hat 1e-3."""
    m = sphere_mesh(radius, cell)
    X = m.X.copy()
    X[:, 2] += gap - X[:, 2].min()
    m = Mesh(X=X, tets=m.tets, pinned=m.pinned, name=m.name + "_on_floor")
    v0 = np.zeros_like(X)
    v0[:, 2] = -speed
    return Scene(mesh=m, E=_per_tet(E, m.nT), nu=_per_tet(nu, m.nT), rho=_per_tet(1000.0, m.nT),
                 x0=X.copy(), v0=v0, gravity=(0.0, 0.0, -9.8),
                 planes=np.array([[0.0, 0.0, 1.0, 0.0]]), steps=1, name="sphere_on_floor")
