"""ctypes binding of the plain FP64 CPU oracle (ebb_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU product path never does.

All arrays are numpy, row-major AoS: X, d, u, v: (nv, 3) float64; tets:
(nt, 4) int32; B: (nt, 3, 3); V0, mu, lam, E: (nt,); mass: (nv,).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libebboracle.so")

STVK = 0
NH = 1
OK = 0
E_DEGENERATE = -8
E_INVERTED = -9
E_NOT_SPD = -10
E_NOT_CONVERGED = -11
PRECOND_NONE = 0
PRECOND_JACOBI = 1

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    I64 = C.c_int64
    D = C.c_double
    I32 = C.c_int32
    lib.orc_lame.argtypes = [D, D, P, P]
    lib.orc_precompute.argtypes = [I64, I64, P, P, D, P, D, P, P, P, P, P, P]
    for name in ("orc_stress",):
        getattr(lib, name).argtypes = [C.c_int, D, D, P, P]
    lib.orc_dstress.argtypes = [C.c_int, D, D, P, P, P]
    lib.orc_d2stress.argtypes = [C.c_int, D, D, P, P, P, P]
    lib.orc_energy_density.argtypes = [C.c_int, D, D, P, P]
    base = [C.c_int, I64, I64, P, P, P, P, P]
    lib.orc_forces.argtypes = base + [P, P]
    lib.orc_kmul.argtypes = base + [P, P, P]
    lib.orc_tmul.argtypes = base + [P, P, P, P]
    lib.orc_energy.argtypes = base + [P, P]
    lib.orc_jacobi_diag.argtypes = base + [P, D, P, P]
    lib.orc_implicit_step.argtypes = base + [P, P, D, P, D, D, D, I32, I32, P, P, P, P]
    lib.orc_step_vjp.argtypes = base + [P, P, P, D, D, D, D, I32, I32, P, P, P, P, P, P, P, P]
    lib.orc_group_by.argtypes = [I64, I64, P, P, P]
    lib.orc_edges.argtypes = [I64, I64, P, P, P, I64, P]
    lib.orc_assemble.argtypes = base + [P, P, P, P]
    lib.orc_spmv.argtypes = [I64, P, P, P, P, P]
    lib.orc_spring_rest.argtypes = [I64, P, P, P, P]
    lib.orc_spring_forces.argtypes = [I64, I64, P, P, P, D, P, P]
    lib.orc_spring_apply.argtypes = [I64, P, D, P, P, P]
    lib.orc_kinetic_energy.argtypes = [I64, P, P]
    lib.orc_kinetic_energy.restype = D
    lib.orc_morton.argtypes = [I64, I64, P, P, P, P, P]
    lib.orc_morton_seg.argtypes = [I64, I64, P, P, P, P, P, P]
    lib.orc_forces_mt.argtypes = base + [P, P, P, P, P, C.c_int]
    lib.orc_kmul_mt.argtypes = base + [P, P, P, P, P, P, C.c_int]
    for f in ("orc_precompute", "orc_stress", "orc_dstress", "orc_d2stress",
              "orc_energy_density", "orc_forces", "orc_kmul", "orc_tmul", "orc_energy",
              "orc_jacobi_diag", "orc_implicit_step", "orc_step_vjp", "orc_group_by",
              "orc_morton", "orc_morton_seg", "orc_edges", "orc_assemble", "orc_spmv", "orc_spring_rest",
              "orc_spring_forces", "orc_spring_apply", "orc_forces_mt", "orc_kmul_mt"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def lame(E: float, nu: float):
    mu = C.c_double()
    lam = C.c_double()
    _load().orc_lame(E, nu, C.byref(mu), C.byref(lam))
    return mu.value, lam.value


def _chk(st: int, what: str, allow=(OK,)):
    if st not in allow:
        raise OracleError(st, what)
    return st


def stress(model, mu, lam, G):
    G = _f64(G, (3, 3))
    P = np.zeros((3, 3))
    _chk(_load().orc_stress(model, mu, lam, _p(G), _p(P)), "stress")
    return P


def dstress(model, mu, lam, G, dF):
    G = _f64(G, (3, 3))
    dF = _f64(dF, (3, 3))
    dP = np.zeros((3, 3))
    _chk(_load().orc_dstress(model, mu, lam, _p(G), _p(dF), _p(dP)), "dstress")
    return dP


def d2stress(model, mu, lam, G, A, W):
    G, A, W = _f64(G, (3, 3)), _f64(A, (3, 3)), _f64(W, (3, 3))
    Q = np.zeros((3, 3))
    _chk(_load().orc_d2stress(model, mu, lam, _p(G), _p(A), _p(W), _p(Q)), "d2stress")
    return Q


def energy_density(model, mu, lam, G):
    G = _f64(G, (3, 3))
    psi = C.c_double()
    _chk(_load().orc_energy_density(model, mu, lam, _p(G), C.byref(psi)), "energy_density")
    return psi.value


def group_by(nv: int, tets: np.ndarray):
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    nt = tets.shape[0]
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    inc = np.zeros(4 * nt, dtype=np.int32)
    _chk(_load().orc_group_by(nv, nt, _p(tets), _p(row_ptr), _p(inc)), "group_by")
    return row_ptr, inc


def edges(nv: int, tets: np.ndarray):
    """Directed edges grouped by tail: (row_ptr (nv+1) int64, col int32)."""
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    nt = tets.shape[0]
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    cap = 16 * nt
    col = np.zeros(max(cap, 1), dtype=np.int32)
    n = C.c_int64()
    _chk(_load().orc_edges(nv, nt, _p(tets), _p(row_ptr), _p(col), cap, C.byref(n)), "edges")
    return row_ptr, col[: n.value].copy()


def spmv(row_ptr, col, blocks, u):
    """y_i = sum_j K_ij u_j over the assembled blocks ((n_edges, 3, 3))."""
    nv = len(row_ptr) - 1
    u = _f64(u, (nv, 3))
    y = np.zeros((nv, 3))
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    bl = _f64(blocks)
    _chk(_load().orc_spmv(nv, _p(rp), _p(cl), _p(bl), _p(u), _p(y)), "spmv")
    return y


class Springs:
    """Spring-mass workload on directed edges (tail, head): rest lengths from X."""

    def __init__(self, X, tail, head, mass, K):
        self.X = _f64(X)
        self.nv = self.X.shape[0]
        self.tail = np.ascontiguousarray(tail, dtype=np.int32)
        self.head = np.ascontiguousarray(head, dtype=np.int32)
        self.ne = len(self.tail)
        self.mass = _f64(mass)
        self.K = float(K)
        self.rest = np.zeros(max(self.ne, 1))
        _chk(_load().orc_spring_rest(self.ne, _p(self.tail), _p(self.head), _p(self.X), _p(self.rest)),
             "spring_rest")

    def forces(self, q):
        q = _f64(q, (self.nv, 3))
        f = np.zeros((self.nv, 3))
        _chk(_load().orc_spring_forces(self.nv, self.ne, _p(self.tail), _p(self.head), _p(self.rest), self.K,
                                       _p(q), _p(f)), "spring_forces")
        return f

    def step(self, q, qd, dt):
        """One step (forces, then the exclusive update); returns (q', qd')."""
        q = _f64(q, (self.nv, 3)).copy()
        qd = _f64(qd, (self.nv, 3)).copy()
        f = self.forces(q)
        _chk(_load().orc_spring_apply(self.nv, _p(self.mass), float(dt), _p(q), _p(qd), _p(f)), "spring_apply")
        return q, qd

    def kinetic_energy(self, qd):
        qd = _f64(qd, (self.nv, 3))
        return _load().orc_kinetic_energy(self.nv, _p(self.mass), _p(qd))


def morton(X: np.ndarray, tets: np.ndarray, seg=None):
    """Morton order (codes, vperm, tperm); with seg (one int label per vertex) the vertices are
    ordered by (seg, code, id), a Morton order within each segment."""
    X = _f64(X)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    nv, nt = X.shape[0], tets.shape[0]
    codes = np.zeros(nv, dtype=np.uint64)
    vperm = np.zeros(nv, dtype=np.int32)
    tperm = np.zeros(nt, dtype=np.int32)
    if seg is None:
        _chk(_load().orc_morton(nv, nt, _p(X), _p(tets), _p(codes), _p(vperm), _p(tperm)), "morton")
    else:
        seg = np.ascontiguousarray(seg, dtype=np.int32)
        assert seg.shape == (nv,)
        _chk(_load().orc_morton_seg(nv, nt, _p(X), _p(tets), _p(seg), _p(codes), _p(vperm), _p(tperm)), "morton")
    return codes, vperm, tperm


@dataclass
class FEM:
    """Rest-shape data of one mesh plus the material, as the oracle sees it."""
    model: int
    tets: np.ndarray
    B: np.ndarray
    V0: np.ndarray
    mu: np.ndarray
    lam: np.ndarray
    E: np.ndarray
    mass: np.ndarray
    pinned: np.ndarray
    nu: float

    @property
    def nv(self):
        return self.mass.shape[0]

    @property
    def nt(self):
        return self.tets.shape[0]

    @classmethod
    def create(cls, model, X, tets, E, nu, rho=1000.0, pinned=None):
        X = _f64(X)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        nv, nt = X.shape[0], tets.shape[0]
        Et = _f64(np.broadcast_to(np.asarray(E, dtype=np.float64), (nt,)))
        B = np.zeros((nt, 3, 3))
        V0 = np.zeros(nt)
        mu = np.zeros(nt)
        lam = np.zeros(nt)
        mass = np.zeros(nv)
        bad = C.c_int64(-1)
        st = _load().orc_precompute(nv, nt, _p(X), _p(tets), rho, _p(Et), nu, _p(B), _p(V0),
                                    _p(mu), _p(lam), _p(mass), C.byref(bad))
        _chk(st, f"precompute (tet {bad.value})")
        if pinned is None:
            pinned = np.zeros(nv, dtype=np.uint8)
        pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        return cls(model, tets, B, V0, mu, lam, Et, mass, pinned, nu)

    def _base(self):
        return [self.model, self.nv, self.nt, _p(self.tets), _p(self.B), _p(self.V0),
                _p(self.mu), _p(self.lam)]

    def forces(self, d):
        d = _f64(d, (self.nv, 3))
        f = np.zeros((self.nv, 3))
        _chk(_load().orc_forces(*self._base(), _p(d), _p(f)), "forces")
        return f

    def kmul(self, d, u):
        d = _f64(d, (self.nv, 3))
        u = _f64(u, (self.nv, 3))
        y = np.zeros((self.nv, 3))
        _chk(_load().orc_kmul(*self._base(), _p(d), _p(u), _p(y)), "kmul")
        return y

    def _mt_buffers(self):
        if getattr(self, "_grp", None) is None:
            self._grp = group_by(self.nv, self.tets)
            self._part = np.zeros((max(self.nt, 1), 12))
        return self._grp[0], self._grp[1], self._part

    def forces_mt(self, d, threads):
        """orc_forces on `threads` OpenMP threads (timing; equal bit for bit to forces)."""
        d = _f64(d, (self.nv, 3))
        f = np.zeros((self.nv, 3))
        rp, inc, part = self._mt_buffers()
        _chk(_load().orc_forces_mt(*self._base(), _p(d), _p(f), _p(rp), _p(inc), _p(part), int(threads)),
             "forces_mt")
        return f

    def kmul_mt(self, d, u, threads):
        """orc_kmul on `threads` OpenMP threads (timing; equal bit for bit to kmul)."""
        d = _f64(d, (self.nv, 3))
        u = _f64(u, (self.nv, 3))
        y = np.zeros((self.nv, 3))
        rp, inc, part = self._mt_buffers()
        _chk(_load().orc_kmul_mt(*self._base(), _p(d), _p(u), _p(y), _p(rp), _p(inc), _p(part), int(threads)),
             "kmul_mt")
        return y

    def assemble(self, d, row_ptr, col):
        """Per-edge 3x3 stiffness blocks K_ij = df_i/dd_j at d: (n_edges, 3, 3)."""
        d = _f64(d, (self.nv, 3))
        blocks = np.zeros((max(len(col), 1), 3, 3))
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        _chk(_load().orc_assemble(*self._base(), _p(d), _p(rp), _p(cl), _p(blocks)), "assemble")
        return blocks[: len(col)]

    def tmul(self, d, a, w):
        d, a, w = (_f64(x, (self.nv, 3)) for x in (d, a, w))
        out = np.zeros((self.nv, 3))
        _chk(_load().orc_tmul(*self._base(), _p(d), _p(a), _p(w), _p(out)), "tmul")
        return out

    def energy(self, d):
        d = _f64(d, (self.nv, 3))
        W = C.c_double()
        _chk(_load().orc_energy(*self._base(), _p(d), C.byref(W)), "energy")
        return W.value

    def jacobi_diag(self, d, dt):
        d = _f64(d, (self.nv, 3))
        diag = np.zeros((self.nv, 3))
        _chk(_load().orc_jacobi_diag(*self._base(), _p(self.mass), dt, _p(d), _p(diag)),
             "jacobi_diag")
        return diag

    def implicit_step(self, d, v, dt, g=(0.0, 0.0, -9.81), tol=0.0, maxit=100,
                      precond=PRECOND_JACOBI, allow_not_converged=True, alpha=0.0, beta=0.0):
        """Returns (d', v', dv, stats) without touching the inputs.

        alpha, beta: Rayleigh damping D = alpha M - beta K (Vega's step computes
        damping with the forces and the stiffness: Performance Evaluation)."""
        d = _f64(d, (self.nv, 3)).copy()
        v = _f64(v, (self.nv, 3)).copy()
        g = _f64(g)
        dv = np.zeros((self.nv, 3))
        st = Stats()
        rc = _load().orc_implicit_step(*self._base(), _p(self.mass), _p(self.pinned), dt, _p(g),
                                       alpha, beta, tol, maxit, precond, _p(d), _p(v), _p(dv),
                                       C.byref(st))
        allow = (OK, E_NOT_CONVERGED) if allow_not_converged else (OK,)
        _chk(rc, "implicit_step", allow)
        return d, v, dv, st

    def step_vjp(self, d_n, v_np1, gx, gv, dt, tol=1e-12, maxit=10000,
                 precond=PRECOND_JACOBI, alpha=0.0, beta=0.0):
        """Returns (d_bar, v_bar, E_bar, stats) of one implicit step."""
        d_n, v_np1, gx, gv = (_f64(x, (self.nv, 3)) for x in (d_n, v_np1, gx, gv))
        d_bar = np.zeros((self.nv, 3))
        v_bar = np.zeros((self.nv, 3))
        E_bar = np.zeros(self.nt)
        st = Stats()
        rc = _load().orc_step_vjp(*self._base(), _p(self.E), _p(self.mass), _p(self.pinned),
                                  dt, alpha, beta, tol, maxit, precond, _p(d_n), _p(v_np1),
                                  _p(gx), _p(gv),
                                  _p(d_bar), _p(v_bar), _p(E_bar), C.byref(st))
        _chk(rc, "step_vjp", (OK, E_NOT_CONVERGED))
        return d_bar, v_bar, E_bar, st


def trajectory(fem: FEM, d0, v0, steps, dt, tol, maxit, g=(0.0, 0.0, -9.81),
               precond=PRECOND_JACOBI, alpha=0.0, beta=0.0):
    """Run `steps` implicit steps; returns the list of (d, v) states 0..steps."""
    states = [(np.array(d0, dtype=np.float64), np.array(v0, dtype=np.float64))]
    d, v = states[0]
    for _ in range(steps):
        d, v, _dv, _st = fem.implicit_step(d, v, dt, g=g, tol=tol, maxit=maxit, precond=precond,
                                           alpha=alpha, beta=beta)
        states.append((d, v))
    return states


def trajectory_grad(fem: FEM, d0, v0, steps, dt, tol, maxit, target, X,
                    g=(0.0, 0.0, -9.81), precond=PRECOND_JACOBI, checkpoint_every=0,
                    alpha=0.0, beta=0.0):
    """Loss L = ||x_T - target||^2 with x = X + d; returns (L, dL/dd0, dL/dE).

    checkpoint_every = k > 0 keeps only every k-th state and recomputes each
    segment forward before reversing it; 0 keeps every state.
    """
    k = checkpoint_every if checkpoint_every > 0 else steps
    ckpt = {0: (np.array(d0, dtype=np.float64), np.array(v0, dtype=np.float64))}
    d, v = ckpt[0]
    for n in range(steps):
        d, v, _dv, _st = fem.implicit_step(d, v, dt, g=g, tol=tol, maxit=maxit, precond=precond,
                                           alpha=alpha, beta=beta)
        if (n + 1) % k == 0 and n + 1 < steps:
            ckpt[n + 1] = (d, v)
    xT = X + d
    L = float(np.sum((xT - target) ** 2))
    gx = 2.0 * (xT - target)
    gv = np.zeros_like(gx)
    E_bar = np.zeros(fem.nt)
    seg_starts = sorted(ckpt.keys(), reverse=True)
    end = steps
    for s0 in seg_starts:
        # recompute the states of this segment
        states = [ckpt[s0]]
        d, v = ckpt[s0]
        for _ in range(s0, end - 1):
            d, v, _dv, _st = fem.implicit_step(d, v, dt, g=g, tol=tol, maxit=maxit,
                                               precond=precond, alpha=alpha, beta=beta)
            states.append((d, v))
        # reverse the steps s0 .. end-1; step n maps states[n-s0] -> n+1
        for n in range(end - 1, s0 - 1, -1):
            d_n, v_n = states[n - s0]
            _d1, v_np1, _dv, _st = fem.implicit_step(d_n, v_n, dt, g=g, tol=tol, maxit=maxit,
                                                     precond=precond, alpha=alpha, beta=beta)
            d_bar, v_bar, eb, _ = fem.step_vjp(d_n, v_np1, gx, gv, dt, tol=tol, maxit=maxit,
                                               precond=precond, alpha=alpha, beta=beta)
            E_bar += eb
            gx, gv = d_bar, v_bar
        end = s0
    return L, gx, E_bar
