"""Seeded synthetic tetrahedral meshes and states.

This module is the one input generator shared by the GPU path, its tests,
the benchmark and the CPU oracle.  It holds no finite-element arithmetic:
only lattice bookkeeping, seeded random draws and permutations.  The
paper's own meshes (Vega's dragon/hose/turtle, the FreeFem++ sphere and
bunny; Performance Evaluation, Vega and FreeFem++ subsections) are not
available, so unit cubes split into Kuhn tetrahedra stand in for them.

Mesh conventions (numpy arrays, row-major, the form the oracle takes):
  X       (nv, 3) float64   rest positions
  tets    (nt, 4) int32     the tets.v[4] key-field (Runtime Implementation,
                            Relational Primitives Implementations)
  pinned  (nv,)   uint8     1 on the bottom face (lattice layer k = 0)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Axis permutations of a Kuhn (Freudenthal) split in lexicographic order, and
# whether each is odd.  Tet p of a cell walks v000 -> +e_a -> +e_b -> v111.
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
KUHN_ODD = (False, True, True, False, False, True)

STVK = 0
NH = 1


@dataclass
class Mesh:
    X: np.ndarray
    tets: np.ndarray
    pinned: np.ndarray
    n: int = 0           # cells per side (0 for non-lattice meshes)
    h: float = 0.0       # lattice spacing

    @property
    def nv(self) -> int:
        return int(self.X.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])


def vid(i, j, k, n):
    """Lattice vertex id of (i, j, k) on an n-cell cube."""
    return i + (n + 1) * (j + (n + 1) * k)


def kuhn_cube(n: int, size: float = 1.0) -> Mesh:
    """[0,size]^3 split into n^3 cells of 6 tets each.

    Cell c = i + n(j + n k) owns tets 6c .. 6c+5, one per axis permutation
    in KUHN_PERMS order.  The split is conforming and every tet has volume
    h^3/6.  For odd permutations corners 2 and 3 are swapped so that every
    tet is positively oriented (the orientation of [e_a, e_a+e_b, e_a+e_b+e_c]
    is the sign of the permutation).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = size / n
    m = n + 1
    g = np.arange(m, dtype=np.float64) * h
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([g[ii.ravel()], g[jj.ravel()], g[kk.ravel()]], axis=1)

    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel().astype(np.int64)
    cj = cj.ravel().astype(np.int64)
    ck = ck.ravel().astype(np.int64)
    base = vid(ci, cj, ck, n)
    step = (1, m, m * m)
    v111 = base + step[0] + step[1] + step[2]
    nc = n ** 3
    tets = np.empty((nc, 6, 4), dtype=np.int64)
    for p, (a, b, _c) in enumerate(KUHN_PERMS):
        c1 = base + step[a]
        c2 = c1 + step[b]
        if KUHN_ODD[p]:
            tets[:, p] = np.stack([base, c1, v111, c2], axis=1)
        else:
            tets[:, p] = np.stack([base, c1, c2, v111], axis=1)
    tets = tets.reshape(nc * 6, 4).astype(np.int32)
    pinned = (kk.ravel() == 0).astype(np.uint8)
    return Mesh(X=X, tets=tets, pinned=pinned, n=n, h=h)


def single_tet(X4=None) -> Mesh:
    """One tet; by default the unit right-corner tet (Dm = I)."""
    if X4 is None:
        X4 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    X4 = np.ascontiguousarray(X4, dtype=np.float64)
    return Mesh(X=X4, tets=np.array([[0, 1, 2, 3]], dtype=np.int32),
                pinned=np.zeros(4, dtype=np.uint8), n=0, h=1.0)


def jitter(mesh: Mesh, frac: float = 0.01, seed: int = 0) -> Mesh:
    """Uniform +-frac*h per component on every vertex, in vertex-id order."""
    rng = np.random.default_rng(seed)
    amp = frac * mesh.h
    X = mesh.X + rng.uniform(-amp, amp, size=mesh.X.shape)
    return Mesh(X=X, tets=mesh.tets.copy(), pinned=mesh.pinned.copy(), n=mesh.n, h=mesh.h)


def scramble(mesh: Mesh, seed: int = 1):
    """Randomly renumber vertices and shuffle tet rows (corner order kept).

    Returns (mesh', pv, pt): pv[new] = old vertex id, pt[new] = old tet row.
    """
    rng = np.random.default_rng(seed)
    pv = rng.permutation(mesh.nv)
    pt = rng.permutation(mesh.nt)
    inv = np.empty_like(pv)
    inv[pv] = np.arange(mesh.nv)
    tets = inv[mesh.tets.astype(np.int64)][pt].astype(np.int32)
    out = Mesh(X=np.ascontiguousarray(mesh.X[pv]), tets=tets,
               pinned=np.ascontiguousarray(mesh.pinned[pv]), n=mesh.n, h=mesh.h)
    return out, pv, pt


def perturbed_state(mesh: Mesh, amp: float = 0.02, seed: int = 10) -> np.ndarray:
    """A nontrivial displacement: uniform +-amp*h per component."""
    rng = np.random.default_rng(seed)
    a = amp * mesh.h
    return rng.uniform(-a, a, size=(mesh.nv, 3))


def direction(mesh: Mesh, seed: int = 11) -> np.ndarray:
    """A unit-scale direction field u ~ U(-1, 1) per component."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(mesh.nv, 3))


def rotation(seed: int = 20) -> np.ndarray:
    """A random proper rotation (QR of a Gaussian matrix, sign-fixed)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# --------------------------------------------------------------------------
# Workload recipes.  Each returns the mesh and the parameters that a
# workload fixes; unstated values are filled with the readings listed in the
# design notes (rho = 1000, g = (0,0,-9.81), bottom face pinned).
# --------------------------------------------------------------------------

GRAVITY = (0.0, 0.0, -9.81)


@dataclass
class Workload:
    name: str
    mesh: Mesh
    model: int
    prec: str                  # element arithmetic: "f32" or "f64"
    E: float
    nu: float
    rho: float = 1000.0
    dt: float = 1e-3
    maxit: int = 100
    tol: float = 0.0
    extra: dict = field(default_factory=dict)


def workload_small() -> Workload:
    """8^3 cells (3,072 tets, 729 verts), jittered +-1% h (seed 0), StVK, FP64,
    E=1e5, nu=0.3, rho=1000, dt=1e-3, 50 CG iterations."""
    m = jitter(kuhn_cube(8), 0.01, seed=0)
    return Workload("cube8_stvk_f64", m, STVK, "f64", 1e5, 0.3, maxit=50)


def workload_plain(n: int = 64) -> Workload:
    """64^3 cells (1,572,864 tets, 274,625 verts), neo-Hookean, FP32 element
    math with FP64 vertex vectors, E=1e6, nu=0.45, dt=1e-3, 100 CG iterations."""
    return Workload(f"cube{n}_nh_f32", kuhn_cube(n), NH, "f32", 1e6, 0.45, maxit=100)


def workload_locality(n: int = 128) -> Workload:
    """128^3 cells (12,582,912 tets, 2,146,689 verts), StVK, FP64, vertex ids
    and tet rows scrambled (seed 1); E=1e5, nu=0.3."""
    m, pv, pt = scramble(kuhn_cube(n), seed=1)
    return Workload(f"cube{n}_stvk_f64_scrambled", m, STVK, "f64", 1e5, 0.3,
                    extra={"pv": pv, "pt": pt})


def batch_recipe(count: int = 256, seed: int = 3, nmin: int = 8, nmax: int = 40):
    """Per-mesh sides n ~ U{nmin..nmax}, log10 E ~ U(4,6), nu ~ U(0.3,0.45),
    drawn in that order from one generator."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    E = 10.0 ** rng.uniform(4.0, 6.0, size=count)
    nu = rng.uniform(0.3, 0.45, size=count)
    return ns.astype(np.int64), E, nu


@dataclass
class MeshUnion:
    """Meshes concatenated into one vertex set and one tet set, each sorted by
    mesh: the layout of a batch (vertex and tet ids offset per mesh)."""
    X: np.ndarray            # (sum nv, 3)
    tets: np.ndarray         # (sum nt, 4) int32, global vertex ids
    pinned: np.ndarray       # (sum nv,) uint8
    vert_mesh: np.ndarray    # (sum nv,) int32
    tet_mesh: np.ndarray     # (sum nt,) int32
    vptr: np.ndarray         # (count + 1,) vertex offsets
    tptr: np.ndarray         # (count + 1,) tet offsets

    @property
    def nv(self) -> int:
        return int(self.X.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])


def union(meshes) -> MeshUnion:
    nvs = np.array([m.nv for m in meshes], dtype=np.int64)
    nts = np.array([m.nt for m in meshes], dtype=np.int64)
    vptr = np.concatenate([[0], np.cumsum(nvs)])
    tptr = np.concatenate([[0], np.cumsum(nts)])
    if vptr[-1] >= 2 ** 31 or tptr[-1] >= 2 ** 31:
        raise ValueError("union too large for int32 ids")
    X = np.concatenate([m.X for m in meshes]).astype(np.float64, copy=False)
    tets = np.concatenate([m.tets for m in meshes]).astype(np.int32, copy=False)
    tets += np.repeat(vptr[:-1], nts).astype(np.int32)[:, None]
    pinned = np.concatenate([m.pinned for m in meshes]).astype(np.uint8, copy=False)
    vert_mesh = np.repeat(np.arange(len(meshes), dtype=np.int32), nvs)
    tet_mesh = np.repeat(np.arange(len(meshes), dtype=np.int32), nts)
    return MeshUnion(X, tets, pinned, vert_mesh, tet_mesh, vptr, tptr)


def workload_batch(count: int = 256, seed: int = 3, nmin: int = 8, nmax: int = 40):
    """Batched workload: `count` Kuhn cubes with sides from batch_recipe,
    compressible neo-Hookean, per-mesh E and nu, dt = 1e-3, CG to 1e-8,
    at most 1000 iterations.  Returns (meshes, E, nu)."""
    ns, E, nu = batch_recipe(count, seed, nmin, nmax)
    return [kuhn_cube(int(n)) for n in ns], E, nu


def adjoint_recipe(mesh: Mesh, seed: int = 2, n_fd: int = 32):
    """Per-tet E = 1e5 exp(0.5 z), target = X + 1e-3 N(0,1), and n_fd
    distinct tets for finite-difference checks, in that draw order."""
    rng = np.random.default_rng(seed)
    E = 1e5 * np.exp(0.5 * rng.standard_normal(mesh.nt))
    target = mesh.X + 1e-3 * rng.standard_normal((mesh.nv, 3))
    fd_tets = rng.choice(mesh.nt, size=min(n_fd, mesh.nt), replace=False)
    return E, target, fd_tets


def directed_edges(tets: np.ndarray, nv: int):
    """The edges relation of a tet mesh as the spring-mass example uses it: every
    ordered pair (tail, head) of distinct corners of some tet, without repeats,
    sorted by tail, then head.  Returns (tail, head) int32 arrays."""
    t = np.asarray(tets, dtype=np.int64)
    a = np.repeat(t, 4, axis=1).ravel()
    b = np.tile(t, (1, 4)).ravel()
    keep = a != b
    key = np.unique(a[keep] * nv + b[keep])
    return (key // nv).astype(np.int32), (key % nv).astype(np.int32)


@dataclass
class SpringWorkload:
    name: str
    mesh: Mesh
    tail: np.ndarray
    head: np.ndarray
    mass: np.ndarray      # (nv,) per-vertex mass
    q0: np.ndarray        # (nv, 3) initial positions
    qd0: np.ndarray       # (nv, 3) initial velocities
    K: float
    dt: float


def workload_springs(n: int = 64, seed: int = 5) -> SpringWorkload:
    """Spring-mass example on the n^3 Kuhn cube: springs on its directed edges
    (rest lengths from the rest positions), masses (1 +- 0.5 uniform) / nv,
    positions perturbed by up to 0.1 h and velocities up to 0.05 per axis
    (uniform), K = 1, dt = 1e-4, in that draw order."""
    m = kuhn_cube(n)
    tail, head = directed_edges(m.tets, m.nv)
    rng = np.random.default_rng(seed)
    mass = (1.0 + 0.5 * rng.uniform(-1.0, 1.0, m.nv)) / m.nv
    q0 = m.X + (0.1 / n) * rng.uniform(-1.0, 1.0, (m.nv, 3))
    qd0 = 0.05 * rng.uniform(-1.0, 1.0, (m.nv, 3))
    return SpringWorkload(f"springs_cube{n}", m, tail, head, mass, q0, qd0, 1.0, 1e-4)


def soa(a: np.ndarray) -> np.ndarray:
    """(n, k) row-major -> (k, n) contiguous: the column-store layout."""
    return np.ascontiguousarray(np.asarray(a).T)
