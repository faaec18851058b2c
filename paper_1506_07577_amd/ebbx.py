"""Thin ctypes binding of libebbx.so (the C-ABI in include/ebbx.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
supplies device memory (tensors are passed as raw pointers; the library's
hidden fields come from torch's caching allocator through the allocator
hook) and streams.  Importing this module does not load the library; the
first call does, and raises if libebbx.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebbx.so")

OK = 0
E_ARG, E_DTYPE, E_SHAPE, E_LAYOUT, E_KEY_RANGE, E_PHASE, E_NOT_GROUPED = -1, -2, -3, -4, -5, -6, -7
E_DEGENERATE, E_INVERTED, E_NOT_SPD, E_NOT_CONVERGED, E_HIP, E_OOM, E_STATE, E_NOT_FOUND = (
    -8, -9, -10, -11, -12, -13, -14, -15)
F32, F64, I32, U8, I64 = 0, 1, 2, 3, 4
STVK, NH = 0, 1
STRAT_AUTO, STRAT_ATOMIC, STRAT_SEG, STRAT_BLOCK, STRAT_BLOCK_LDS, STRAT_OWNER, STRAT_PIPE, STRAT_LANES = (
    0, 1, 2, 3, 4, 5, 6, 7)
BLOCK_TPT2 = 0x10000   # or-ed into a BLOCK / BLOCK_LDS block size: two tets per thread
PRECOND_NONE, PRECOND_JACOBI = 0, 1

_DT = {torch.float32: F32, torch.float64: F64, torch.int32: I32, torch.uint8: U8, torch.int64: I64}


class EbbxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ebbx status {code}: {msg}")
        self.code = code


class FemParams(C.Structure):
    _fields_ = [("model", C.c_int32), ("elem_prec", C.c_int32), ("rho", C.c_double), ("E", C.c_double),
                ("nu", C.c_double), ("E_field", C.c_char_p), ("strategy", C.c_int32), ("block", C.c_int32)]


class StepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double * 3), ("tol", C.c_double), ("maxit", C.c_int32),
                ("precond", C.c_int32), ("alpha", C.c_double), ("beta", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("n_inverted", C.c_int64)]


class TuneEntry(C.Structure):
    _fields_ = [("strategy", C.c_int32), ("block", C.c_int32), ("us", C.c_double)]


class BatchFields(C.Structure):
    _fields_ = [(n, C.c_char_p) for n in ("tet_verts", "tet_mesh", "vert_mesh", "pos", "pinned", "E", "nu")]


_lib = None
_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_hooks = []


def _torch_alloc(nbytes, _ctx, stream):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream or None)
    except Exception:   # out of memory: the library reports EBBX_E_OOM
        return None


def _torch_free(ptr, _ctx):
    torch.cuda.caching_allocator_delete(ptr)


def lib():
    """Load libebbx.so (once).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the GPU path has no fallback)")
    L = C.CDLL(LIB_PATH)
    P, I32_, I64_, D, S = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_char_p
    sig = {
        "ebbx_last_error": ([], C.c_char_p),
        "ebbx_version": ([], C.c_int32),
        "ebbx_set_allocator": ([_ALLOC_T, _FREE_T, P], I32_),
        "ebbx_relation_create": ([S, I64_, C.POINTER(P)], I32_),
        "ebbx_relation_destroy": ([P], I32_),
        "ebbx_relation_size": ([P, C.POINTER(I64_)], I32_),
        "ebbx_field_bind": ([P, S, C.c_int, I32_, P], I32_),
        "ebbx_keyfield_bind": ([P, S, P, I32_, P], I32_),
        "ebbx_relation_group_by": ([P, S], I32_),
        "ebbx_group_export": ([P, S, P, P], I32_),
        "ebbx_morton_order": ([P, S, S, P, S, P, P, P], I32_),
        "ebbx_relation_reorder": ([P, P], I32_),
        "ebbx_fem_create": ([P, S, P, S, S, C.POINTER(FemParams), C.POINTER(P)], I32_),
        "ebbx_fem_destroy": ([P], I32_),
        "ebbx_fem_set_strategy": ([P, I32_, I32_], I32_),
        "ebbx_fem_get_strategy": ([P, C.POINTER(I32_), C.POINTER(I32_)], I32_),
        "ebbx_fem_forces": ([P, P, P, I32_, P], I32_),
        "ebbx_fem_Kmul": ([P, P, P, P, I32_, P], I32_),
        "ebbx_fem_Kmul_noalloc": ([P, P, P, P, I32_, P], I32_),
        "ebbx_fem_energy": ([P, P, P, P], I32_),
        "ebbx_fem_jacobi_diag": ([P, P, D, P, P], I32_),
        "ebbx_fem_mass": ([P, P, P], I32_),
        "ebbx_fem_status": ([P, C.POINTER(I64_), I32_, P], I32_),
        "ebbx_implicit_step": ([P, P, P, C.POINTER(StepParams), P, P], I32_),
        "ebbx_stats_fetch": ([P, C.POINTER(StepStats), P], I32_),
        "ebbx_cache_flush": ([C.c_size_t, P], I32_),
        "ebbx_fem_Tmul": ([P, P, P, P, P, I32_, P], I32_),
        "ebbx_fem_E_grad": ([P, P, P, P, D, P, P], I32_),
        "ebbx_fem_set_material": ([P, P, P, D, D, P], I32_),
        "ebbx_fem_forces_vjp": ([P, P, P, P, P, P], I32_),
        "ebbx_fem_Kmul_vjp": ([P, P, P, P, P, P, P, P], I32_),
        "ebbx_implicit_step_vjp": ([P, P, P, C.POINTER(StepParams), P, P, P, P, P, P, P], I32_),
        "ebbx_fem_autotune": ([P, P, P, S, C.POINTER(TuneEntry), I32_, C.POINTER(I32_), P], I32_),
        "ebbx_batch_create": ([P, P, P, C.POINTER(BatchFields), C.POINTER(FemParams), C.POINTER(P)], I32_),
        "ebbx_batch_destroy": ([P], I32_),
        "ebbx_batch_fem": ([P, C.POINTER(P)], I32_),
        "ebbx_batch_implicit_step": ([P, P, P, C.POINTER(StepParams), P, P], I32_),
        "ebbx_fem_assemble": ([P, P, P], I32_),
        "ebbx_fem_spmv": ([P, P, P, I32_, P], I32_),
        "ebbx_fem_edge_count": ([P, C.POINTER(I64_)], I32_),
        "ebbx_fem_edges_get": ([P, P, P, P, P], I32_),
        "ebbx_springs_create": ([P, S, S, P, S, D, C.POINTER(P)], I32_),
        "ebbx_springs_destroy": ([P], I32_),
        "ebbx_springs_rest": ([P, P, P], I32_),
        "ebbx_springs_forces": ([P, P, P, I32_, P], I32_),
        "ebbx_springs_apply": ([P, P, D, P, P, P, P], I32_),
        "ebbx_springs_kinetic_energy": ([P, P, P, P, P], I32_),
        "ebbx_springs_run": ([P, P, D, I32_, P, P, P, P], I32_),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    use_torch_allocator(True)
    return L


def use_torch_allocator(on: bool = True):
    """Route the library's hidden-field allocations through torch's caching allocator."""
    L = lib()
    if on:
        a, f = _ALLOC_T(_torch_alloc), _FREE_T(_torch_free)
        _hooks[:] = [a, f]
        _check(L.ebbx_set_allocator(a, f, None))
    else:
        _check(L.ebbx_set_allocator(_ALLOC_T(), _FREE_T(), None))


def _check(st):
    if st != OK:
        raise EbbxError(st, lib().ebbx_last_error().decode(errors="replace"))
    return st


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t: torch.Tensor, dtype, what) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous (column store)")
    return t


class Relation:
    """A relation (table).  Bound tensors are kept alive by this object."""

    def __init__(self, name: str, size: int):
        h = C.c_void_p()
        _check(lib().ebbx_relation_create(name.encode(), int(size), C.byref(h)))
        self.h = h
        self.name = name
        self.size = int(size)
        self._keep = {}

    def bind_field(self, name: str, t: torch.Tensor):
        """t: (ncomp, size) or (size,) CUDA tensor, column store."""
        if t.dtype not in _DT:
            raise TypeError(f"unsupported dtype {t.dtype}")
        ncomp = 1 if t.dim() == 1 else t.shape[0]
        if t.shape[-1] != self.size:
            raise ValueError(f"field {name}: last dim {t.shape[-1]} != relation size {self.size}")
        _dev(t, t.dtype, name)
        _check(lib().ebbx_field_bind(self.h, name.encode(), _DT[t.dtype], int(ncomp), _ptr(t)))
        self._keep[name] = t

    def bind_keyfield(self, name: str, target: "Relation", t: torch.Tensor):
        """t: (arity, size) int32 CUDA tensor of keys into target."""
        _dev(t, torch.int32, name)
        arity = 1 if t.dim() == 1 else t.shape[0]
        if t.shape[-1] != self.size:
            raise ValueError(f"key-field {name}: last dim {t.shape[-1]} != relation size {self.size}")
        _check(lib().ebbx_keyfield_bind(self.h, name.encode(), target.h, int(arity), _ptr(t)))
        self._keep[name] = t
        self._keep["__target_" + name] = target

    def group_by(self, keyfield: str):
        _check(lib().ebbx_relation_group_by(self.h, keyfield.encode()))

    def group_export(self, keyfield: str, n_target: int, arity: int):
        rp = torch.empty(n_target + 1, dtype=torch.int64, device="cuda")
        inc = torch.empty(max(arity * self.size, 1), dtype=torch.int32, device="cuda")
        _check(lib().ebbx_group_export(self.h, keyfield.encode(), _ptr(rp), _ptr(inc)))
        return rp, inc[: arity * self.size]

    def reorder(self, new_to_old: torch.Tensor):
        _dev(new_to_old, torch.int32, "permutation")
        _check(lib().ebbx_relation_reorder(self.h, _ptr(new_to_old)))

    def close(self):
        if self.h:
            _check(lib().ebbx_relation_destroy(self.h))
            self.h = None


def morton_order(verts: Relation, pos_field: str, rel: Relation, keyfield: str, seg: Optional[str] = None):
    """Returns (codes uint64-as-int64, vperm int32, tperm int32), each new -> old.  seg: an
    arity-1 key-field of verts whose segments (e.g. a batch's meshes) the order keeps apart."""
    codes = torch.empty(max(verts.size, 1), dtype=torch.int64, device="cuda")
    vperm = torch.empty(max(verts.size, 1), dtype=torch.int32, device="cuda")
    tperm = torch.empty(max(rel.size, 1), dtype=torch.int32, device="cuda")
    _check(lib().ebbx_morton_order(verts.h, pos_field.encode(), seg.encode() if seg else None, rel.h,
                                   keyfield.encode(), _ptr(codes), _ptr(vperm), _ptr(tperm)))
    return codes[: verts.size], vperm[: verts.size], tperm[: rel.size]


class Fem:
    """The tet-FEM domain over (tets, verts); see ebbx_fem_create."""

    def __init__(self, tets: Relation, keyfield: str, verts: Relation, pos_field: str,
                 pinned_field: Optional[str], model: int, elem_prec: int, E: float, nu: float,
                 rho: float = 1000.0, E_field: Optional[str] = None, strategy: int = STRAT_ATOMIC,
                 block: int = 0):
        p = FemParams(model, elem_prec, rho, E, nu, E_field.encode() if E_field else None, strategy, block)
        h = C.c_void_p()
        _check(lib().ebbx_fem_create(tets.h, keyfield.encode(), verts.h, pos_field.encode(),
                                     pinned_field.encode() if pinned_field else None, C.byref(p),
                                     C.byref(h)))
        self.h = h
        self.tets, self.verts = tets, verts
        self.nt, self.nv = tets.size, verts.size
        self.model, self.elem_prec = model, elem_prec
        self.E, self.nu = float(E), float(nu)

    @classmethod
    def _borrowed(cls, h, tets: Relation, verts: Relation, model: int, elem_prec: int):
        """A view of a domain owned by something else (a batch's union)."""
        self = cls.__new__(cls)
        self.h = h
        self.tets, self.verts = tets, verts
        self.nt, self.nv = tets.size, verts.size
        self.model, self.elem_prec = model, elem_prec
        self.E, self.nu = 0.0, 0.0
        self._owned = False
        return self

    def close(self):
        if self.h and getattr(self, "_owned", True):
            _check(lib().ebbx_fem_destroy(self.h))
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_strategy(self, strategy: int, block: int = 0):
        _check(lib().ebbx_fem_set_strategy(self.h, int(strategy), int(block)))

    def get_strategy(self):
        s, b = C.c_int32(), C.c_int32()
        _check(lib().ebbx_fem_get_strategy(self.h, C.byref(s), C.byref(b)))
        return s.value, b.value

    def autotune(self, d=None, u=None, cache: Optional[str] = None, stream=None):
        """Time the stiffness product under each strategy/block size and keep the fastest.
        Returns [(strategy, block, us)] (empty on a cache hit)."""
        if d is not None:
            self._vec(d, "d")
        if u is not None:
            self._vec(u, "u")
        cap = 64
        arr = (TuneEntry * cap)()
        n = C.c_int32()
        _check(lib().ebbx_fem_autotune(self.h, _ptr(d), _ptr(u), cache.encode() if cache else None, arr, cap,
                                       C.byref(n), _stream(stream)))
        return [(arr[i].strategy, arr[i].block, arr[i].us) for i in range(min(n.value, cap))]

    def _vec(self, t, what):
        _dev(t, torch.float64, what)
        if tuple(t.shape) != (3, self.nv):
            raise ValueError(f"{what}: expected shape (3, {self.nv}), got {tuple(t.shape)}")
        return t

    def forces(self, d, f=None, accumulate=False, stream=None):
        self._vec(d, "d")
        if f is None:
            f = torch.empty_like(d)
        self._vec(f, "f")
        _check(lib().ebbx_fem_forces(self.h, _ptr(d), _ptr(f), int(bool(accumulate)), _stream(stream)))
        return f

    def kmul(self, d, u, y=None, accumulate=False, stream=None):
        self._vec(d, "d")
        self._vec(u, "u")
        if y is None:
            y = torch.empty_like(d)
        self._vec(y, "y")
        _check(lib().ebbx_fem_Kmul(self.h, _ptr(d), _ptr(u), _ptr(y), int(bool(accumulate)),
                                   _stream(stream)))
        return y

    def kmul_noalloc(self, d, u, y, accumulate=False, stream=None):
        """kmul through the allocation-free entry point: y must be given (nothing is allocated)."""
        self._vec(d, "d")
        self._vec(u, "u")
        self._vec(y, "y")
        _check(lib().ebbx_fem_Kmul_noalloc(self.h, _ptr(d), _ptr(u), _ptr(y), int(bool(accumulate)),
                                           _stream(stream)))
        return y

    def assemble(self, d, stream=None):
        """Assemble K(d) into the per-edge 3x3 blocks (the edges relation is built on first use)."""
        self._vec(d, "d")
        _check(lib().ebbx_fem_assemble(self.h, _ptr(d), _stream(stream)))

    def spmv(self, u, y=None, accumulate=False, stream=None):
        """y (+)= K u with the blocks of the last assemble()."""
        self._vec(u, "u")
        if y is None:
            y = torch.empty_like(u)
        self._vec(y, "y")
        _check(lib().ebbx_fem_spmv(self.h, _ptr(u), _ptr(y), int(bool(accumulate)), _stream(stream)))
        return y

    def edge_count(self):
        n = C.c_int64()
        _check(lib().ebbx_fem_edge_count(self.h, C.byref(n)))
        return n.value

    def edges(self, blocks=True, stream=None):
        """(row_ptr (nv+1) int32, col (n_edges) int32, blocks (9, n_edges) FP64 or None), library order."""
        n = self.edge_count()
        row = torch.empty(self.nv + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        blk = torch.empty(9, max(n, 1), dtype=torch.float64, device="cuda") if blocks else None
        _check(lib().ebbx_fem_edges_get(self.h, _ptr(row), _ptr(col), _ptr(blk), _stream(stream)))
        return row, col[:n], (blk[:, :n] if blk is not None else None)

    def energy(self, d, stream=None):
        self._vec(d, "d")
        out = torch.empty(1, dtype=torch.float64, device=d.device)
        _check(lib().ebbx_fem_energy(self.h, _ptr(d), _ptr(out), _stream(stream)))
        return out

    def jacobi_diag(self, d, dt, stream=None):
        self._vec(d, "d")
        out = torch.empty_like(d)
        _check(lib().ebbx_fem_jacobi_diag(self.h, _ptr(d), float(dt), _ptr(out), _stream(stream)))
        return out

    def mass(self, stream=None):
        out = torch.empty(self.nv, dtype=torch.float64, device="cuda")
        _check(lib().ebbx_fem_mass(self.h, _ptr(out), _stream(stream)))
        return out

    def n_inverted(self, reset=False, stream=None):
        n = C.c_int64()
        _check(lib().ebbx_fem_status(self.h, C.byref(n), int(bool(reset)), _stream(stream)))
        return n.value

    def tmul(self, d, a, w, out=None, accumulate=False, stream=None):
        for t, n in ((d, "d"), (a, "a"), (w, "w")):
            self._vec(t, n)
        if out is None:
            out = torch.empty_like(d)
        self._vec(out, "out")
        _check(lib().ebbx_fem_Tmul(self.h, _ptr(d), _ptr(a), _ptr(w), _ptr(out), int(bool(accumulate)),
                                   _stream(stream)))
        return out

    def E_grad(self, d, v, w, dt, E_bar, stream=None):
        for t, n in ((d, "d"), (v, "v"), (w, "w")):
            self._vec(t, n)
        _dev(E_bar, torch.float64, "E_bar")
        _check(lib().ebbx_fem_E_grad(self.h, _ptr(d), _ptr(v), _ptr(w), float(dt), _ptr(E_bar),
                                     _stream(stream)))
        return E_bar

    def forces_vjp(self, d, w, d_bar=None, E_bar=None, stream=None):
        """d_bar += K(d) w; E_bar += per-tet w.f_t/E_t (outputs accumulate, nullable)."""
        self._vec(d, "d")
        self._vec(w, "w")
        if d_bar is not None:
            self._vec(d_bar, "d_bar")
        if E_bar is not None:
            _dev(E_bar, torch.float64, "E_bar")
        _check(lib().ebbx_fem_forces_vjp(self.h, _ptr(d), _ptr(w), _ptr(d_bar), _ptr(E_bar), _stream(stream)))
        return d_bar, E_bar

    def kmul_vjp(self, d, u, w, d_bar=None, u_bar=None, E_bar=None, stream=None):
        """d_bar += T[u, w]; u_bar += K(d) w; E_bar += per-tet w.K_t u/E_t (accumulate, nullable)."""
        for t, n in ((d, "d"), (u, "u"), (w, "w")):
            self._vec(t, n)
        for t, n in ((d_bar, "d_bar"), (u_bar, "u_bar")):
            if t is not None:
                self._vec(t, n)
        if E_bar is not None:
            _dev(E_bar, torch.float64, "E_bar")
        _check(lib().ebbx_fem_Kmul_vjp(self.h, _ptr(d), _ptr(u), _ptr(w), _ptr(d_bar), _ptr(u_bar), _ptr(E_bar),
                                       _stream(stream)))
        return d_bar, u_bar, E_bar

    def set_material(self, E_tet=None, nu_tet=None, E=0.0, nu=0.3, stream=None):
        """Per-tet (nt,) FP64 CUDA tensors or uniform values.  The tensors are borrowed."""
        if E_tet is not None:
            _dev(E_tet, torch.float64, "E_tet")
        if nu_tet is not None:
            _dev(nu_tet, torch.float64, "nu_tet")
        self._material = (E_tet, nu_tet)
        _check(lib().ebbx_fem_set_material(self.h, _ptr(E_tet), _ptr(nu_tet), float(E), float(nu),
                                           _stream(stream)))

    def step_vjp(self, d_n, v_np1, gx, gv, dt, tol=1e-10, maxit=1000, precond=PRECOND_JACOBI,
                 E_bar=None, g=(0.0, 0.0, -9.81), stats=None, stream=None, alpha=0.0, beta=0.0):
        """Returns (d_bar, v_bar, stats); accumulates dL/dE into E_bar if given.
        alpha, beta: the Rayleigh damping of the step being differentiated."""
        for t, n in ((d_n, "d_n"), (v_np1, "v_np1"), (gx, "gx"), (gv, "gv")):
            self._vec(t, n)
        d_bar = torch.empty_like(d_n)
        v_bar = torch.empty_like(d_n)
        if stats is None:
            stats = torch.zeros(3, dtype=torch.int64, device=d_n.device)
        if E_bar is not None:
            _dev(E_bar, torch.float64, "E_bar")
        p = StepParams(float(dt), (C.c_double * 3)(*g), float(tol), int(maxit), int(precond), float(alpha),
                       float(beta))
        _check(lib().ebbx_implicit_step_vjp(self.h, _ptr(d_n), _ptr(v_np1), C.byref(p), _ptr(gx), _ptr(gv),
                                            _ptr(d_bar), _ptr(v_bar), _ptr(E_bar), _ptr(stats),
                                            _stream(stream)))
        return d_bar, v_bar, stats

    def implicit_step(self, d, v, dt, g=(0.0, 0.0, -9.81), tol=0.0, maxit=100,
                      precond=PRECOND_JACOBI, stats=None, stream=None, alpha=0.0, beta=0.0):
        """Advance (d, v) in place; returns the device stats tensor (24 bytes).
        alpha, beta: Rayleigh damping D = alpha M - beta K (K = df/dx)."""
        self._vec(d, "d")
        self._vec(v, "v")
        if stats is None:
            stats = torch.zeros(3, dtype=torch.int64, device=d.device)
        p = StepParams(float(dt), (C.c_double * 3)(*g), float(tol), int(maxit), int(precond), float(alpha),
                       float(beta))
        _check(lib().ebbx_implicit_step(self.h, _ptr(d), _ptr(v), C.byref(p), _ptr(stats),
                                        _stream(stream)))
        return stats


class Batch:
    """Many meshes in one set of relations (see ebbx_batch_create)."""

    def __init__(self, meshes: Relation, tets: Relation, verts: Relation, model: int, elem_prec: int,
                 tet_verts="v", tet_mesh="mesh", vert_mesh="mesh", pos="X", pinned: Optional[str] = "pinned",
                 E="E", nu="nu", rho=1000.0, strategy=STRAT_BLOCK, block=0):
        f = BatchFields(tet_verts.encode(), tet_mesh.encode(), vert_mesh.encode(), pos.encode(),
                        pinned.encode() if pinned else None, E.encode(), nu.encode())
        p = FemParams(model, elem_prec, rho, 0.0, 0.0, None, strategy, block)
        h = C.c_void_p()
        _check(lib().ebbx_batch_create(meshes.h, tets.h, verts.h, C.byref(f), C.byref(p), C.byref(h)))
        self.h = h
        self.meshes, self.tets, self.verts = meshes, tets, verts
        self.nm = meshes.size
        hf = C.c_void_p()
        _check(lib().ebbx_batch_fem(self.h, C.byref(hf)))
        self.fem = Fem._borrowed(hf, tets, verts, model, elem_prec)

    def implicit_step(self, d, v, dt, g=(0.0, 0.0, -9.81), tol=1e-8, maxit=1000, precond=PRECOND_JACOBI,
                      stats=None, stream=None, alpha=0.0, beta=0.0):
        """Advance every mesh in place; returns the (nm, 3) int64 device stats tensor."""
        self.fem._vec(d, "d")
        self.fem._vec(v, "v")
        if stats is None:
            stats = torch.zeros(self.nm, 3, dtype=torch.int64, device=d.device)
        p = StepParams(float(dt), (C.c_double * 3)(*g), float(tol), int(maxit), int(precond), float(alpha),
                       float(beta))
        _check(lib().ebbx_batch_implicit_step(self.h, _ptr(d), _ptr(v), C.byref(p), _ptr(stats), _stream(stream)))
        return stats

    def close(self):
        if self.h:
            self.fem.h = None
            _check(lib().ebbx_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchMesh:
    """Convenience: upload a meshgen.MeshUnion with per-mesh E and nu and build its Batch.

    morton=True reorders the union into a Morton order within each mesh (the runtime's
    ebbx_morton_order with the verts' mesh key-field as segments, then ebbx_relation_reorder),
    which keeps the meshes contiguous as a batch requires; to_dev and from_dev translate between
    the caller's vertex order and the library's."""

    def __init__(self, un, E, nu, model=NH, elem_prec=F32, rho=1000.0, strategy=STRAT_BLOCK, block=0,
                 morton=False):
        self.un = un
        nm = len(un.vptr) - 1
        self.meshes = Relation("meshes", nm)
        self.verts = Relation("verts", un.nv)
        self.tets = Relation("tets", un.nt)
        self.meshes.bind_field("E", torch.as_tensor(E, dtype=torch.float64).contiguous().cuda())
        self.meshes.bind_field("nu", torch.as_tensor(nu, dtype=torch.float64).contiguous().cuda())
        self.verts.bind_field("X", torch.as_tensor(un.X, dtype=torch.float64).t().contiguous().cuda())
        self.verts.bind_field("pinned", torch.as_tensor(un.pinned).to(torch.uint8).contiguous().cuda())
        self.verts.bind_keyfield("mesh", self.meshes, torch.as_tensor(un.vert_mesh).to(torch.int32).cuda())
        self.tets.bind_keyfield("v", self.verts, torch.as_tensor(un.tets).to(torch.int32).t().contiguous().cuda())
        self.tets.bind_keyfield("mesh", self.meshes, torch.as_tensor(un.tet_mesh).to(torch.int32).cuda())
        self.vperm = self.tperm = None
        if morton:
            _codes, self.vperm, self.tperm = morton_order(self.verts, "X", self.tets, "v", seg="mesh")
            self.verts.reorder(self.vperm)
            self.tets.reorder(self.tperm)
        self.batch = Batch(self.meshes, self.tets, self.verts, model, elem_prec, rho=rho, strategy=strategy,
                           block=block)
        self.fem = self.batch.fem
        self.nm, self.nv, self.nt = nm, un.nv, un.nt

    def to_dev(self, a):
        """(nv, 3) array in the union's vertex order -> (3, nv) device tensor in library order."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if self.vperm is not None:
            t = t[self.vperm.cpu().long()]
        return t.t().contiguous().cuda()

    def from_dev(self, t):
        """(3, nv) device tensor in library order -> (nv, 3) numpy in the union's vertex order."""
        a = t.t().cpu().numpy()
        if self.vperm is not None:
            out = a.copy()
            out[self.vperm.cpu().numpy()] = a
            a = out
        return a


def stats_parse(stats_dev: torch.Tensor):
    """(n, 3) int64 device stats records -> list of StepStats (one copy, syncs)."""
    raw = stats_dev.reshape(-1, 3).cpu().numpy()
    return [StepStats.from_buffer_copy(raw[i].tobytes()) for i in range(raw.shape[0])]


def stats_fetch(stats_dev: torch.Tensor, stream=None) -> StepStats:
    h = StepStats()
    _check(lib().ebbx_stats_fetch(_ptr(stats_dev), C.byref(h), _stream(stream)))
    return h


def cache_flush(nbytes: int = 1 << 30, stream=None):
    _check(lib().ebbx_cache_flush(C.c_size_t(int(nbytes)), _stream(stream)))


class FemMesh:
    """Convenience: relations + bound fields of one tet mesh, then its Fem.

    X: (nv, 3) float64; tets: (nt, 4) int32; pinned: (nv,) uint8 (numpy or
    torch).  Uploads to the GPU in column-store layout.
    """

    def __init__(self, X, tets, pinned=None, model=NH, elem_prec=F64, E=1e5, nu=0.3, rho=1000.0,
                 E_tet=None, strategy=STRAT_ATOMIC, block=0, morton=False):
        Xd = torch.as_tensor(X, dtype=torch.float64).t().contiguous().cuda()
        Td = torch.as_tensor(tets).to(torch.int32).t().contiguous().cuda()
        nv, nt = Xd.shape[1], Td.shape[1]
        self.verts = Relation("verts", nv)
        self.tets = Relation("tets", nt)
        self.verts.bind_field("X", Xd)
        self.tets.bind_keyfield("v", self.verts, Td)
        if pinned is not None:
            self.verts.bind_field("pinned", torch.as_tensor(pinned).to(torch.uint8).contiguous().cuda())
        if E_tet is not None:
            self.tets.bind_field("E", torch.as_tensor(E_tet, dtype=torch.float64).contiguous().cuda())
        self.vperm = self.tperm = None
        if morton:
            _codes, self.vperm, self.tperm = morton_order(self.verts, "X", self.tets, "v")
            self.verts.reorder(self.vperm)
            self.tets.reorder(self.tperm)
        self.X, self.T = Xd, Td
        self.fem = Fem(self.tets, "v", self.verts, "X", "pinned" if pinned is not None else None, model,
                       elem_prec, E, nu, rho, "E" if E_tet is not None else None, strategy, block)

    @property
    def nv(self):
        return self.verts.size

    @property
    def nt(self):
        return self.tets.size

    def to_dev(self, a):
        """(nv, 3) array in the caller's vertex order -> (3, nv) device tensor in library order."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if self.vperm is not None:
            t = t[self.vperm.cpu().long()]
        return t.t().contiguous().cuda()

    def from_dev(self, t):
        """(3, nv) device tensor in library order -> (nv, 3) numpy in the caller's vertex order."""
        a = t.t().cpu().numpy()
        if self.vperm is not None:
            out = a.copy()
            out[self.vperm.cpu().numpy()] = a
            a = out
        return a

    def tet_to_dev(self, a):
        """(nt,) per-tet array in the caller's tet order -> FP64 device tensor in library order."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if self.tperm is not None:
            t = t[self.tperm.cpu().long()]
        return t.contiguous().cuda()

    def tet_from_dev(self, t):
        """(nt,) device tensor in library order -> numpy in the caller's tet order."""
        a = t.detach().cpu().numpy()
        if self.tperm is not None:
            out = a.copy()
            out[self.tperm.cpu().numpy()] = a
            a = out
        return a


class Springs:
    """Spring-mass domain over an edges relation (key-fields tail, head -> verts); see ebbx_springs_create."""

    def __init__(self, edges: Relation, verts: Relation, K: float, tail="tail", head="head", pos="X"):
        h = C.c_void_p()
        _check(lib().ebbx_springs_create(edges.h, tail.encode(), head.encode(), verts.h, pos.encode(), float(K),
                                         C.byref(h)))
        self.h = h
        self.edges, self.verts = edges, verts
        self.nv, self.ne = verts.size, edges.size

    def _vec(self, t, what):
        _dev(t, torch.float64, what)
        if tuple(t.shape) != (3, self.nv):
            raise ValueError(f"{what}: expected shape (3, {self.nv}), got {tuple(t.shape)}")

    def rest(self, stream=None):
        out = torch.empty(max(self.ne, 1), dtype=torch.float64, device="cuda")
        _check(lib().ebbx_springs_rest(self.h, _ptr(out), _stream(stream)))
        return out[: self.ne]

    def forces(self, q, force=None, accumulate=False, stream=None):
        self._vec(q, "q")
        if force is None:
            force = torch.zeros_like(q)
        self._vec(force, "force")
        _check(lib().ebbx_springs_forces(self.h, _ptr(q), _ptr(force), int(bool(accumulate)), _stream(stream)))
        return force

    def apply(self, mass, dt, q, qd, force, stream=None):
        for t, n in ((q, "q"), (qd, "qd"), (force, "force")):
            self._vec(t, n)
        _dev(mass, torch.float64, "mass")
        _check(lib().ebbx_springs_apply(self.h, _ptr(mass), float(dt), _ptr(q), _ptr(qd), _ptr(force),
                                        _stream(stream)))

    def kinetic_energy(self, mass, qd, E=None, stream=None):
        self._vec(qd, "qd")
        _dev(mass, torch.float64, "mass")
        if E is None:
            E = torch.zeros(1, dtype=torch.float64, device="cuda")
        _check(lib().ebbx_springs_kinetic_energy(self.h, _ptr(mass), _ptr(qd), _ptr(E), _stream(stream)))
        return E

    def run(self, mass, dt, nsteps, q, qd, force, stream=None):
        for t, n in ((q, "q"), (qd, "qd"), (force, "force")):
            self._vec(t, n)
        _dev(mass, torch.float64, "mass")
        _check(lib().ebbx_springs_run(self.h, _ptr(mass), float(dt), int(nsteps), _ptr(q), _ptr(qd), _ptr(force),
                                      _stream(stream)))

    def close(self):
        if self.h:
            _check(lib().ebbx_springs_destroy(self.h))
            self.h = None


class SpringMesh:
    """Convenience: verts (rest positions X) and edges (tail, head key-fields) relations, then Springs.

    X: (nv, 3) float64; tail, head: (ne,) int32 (numpy or torch).  morton: reorder the vertices
    (and the edges by tail) in Morton order first; to_dev / from_dev / scalar_to_dev then map
    between the caller's vertex order and the library's."""

    def __init__(self, X, tail, head, K, morton=False):
        Xd = torch.as_tensor(X, dtype=torch.float64).t().contiguous().cuda()
        nv = Xd.shape[1]
        self.verts = Relation("verts", nv)
        self.edges = Relation("edges", len(tail))
        self.verts.bind_field("X", Xd)
        self.edges.bind_keyfield("tail", self.verts, torch.as_tensor(tail).to(torch.int32).contiguous().cuda())
        self.edges.bind_keyfield("head", self.verts, torch.as_tensor(head).to(torch.int32).contiguous().cuda())
        self.vperm = None
        if morton:
            _codes, self.vperm, eperm = morton_order(self.verts, "X", self.edges, "tail")
            self.verts.reorder(self.vperm)
            self.edges.reorder(eperm)
        self.springs = Springs(self.edges, self.verts, K)
        self.nv = nv

    def to_dev(self, a):
        """(nv, 3) array in the caller's vertex order -> (3, nv) device tensor in library order."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if self.vperm is not None:
            t = t[self.vperm.cpu().long()]
        return t.t().contiguous().cuda()

    def scalar_to_dev(self, a):
        """(nv,) array (e.g. the masses) in the caller's vertex order -> device tensor in library order."""
        t = torch.as_tensor(a, dtype=torch.float64)
        if self.vperm is not None:
            t = t[self.vperm.cpu().long()]
        return t.contiguous().cuda()

    def from_dev(self, t):
        """(3, nv) device tensor in library order -> (nv, 3) numpy in the caller's vertex order."""
        a = t.t().cpu().numpy()
        if self.vperm is not None:
            out = a.copy()
            out[self.vperm.cpu().numpy()] = a
            return out
        return a
