"""The allocation-free stiffness product (ebbx_fem_Kmul_noalloc) against ebbx_fem_Kmul.

The allocation-free call runs the same kernels as ebbx_fem_Kmul with the call's scratch (the
shared-vertex partials of the block strategies, the per-corner partials of SEG) in a
library-wide device array.  Each case makes two calls in a row on one GPU -- first on a
14^3 Kuhn cube (16,464 tets), then on a smaller 8^3 one (3,072 tets), so the array still
holds the first call's partials -- and compares each with ebbx_fem_Kmul on the same inputs:
bit for bit for the deterministic strategies, within the oracle tolerance (FP64 1e-10, FP32
1e-5, relative to the largest entry) for the atomic ones, whose summation order varies run
to run.  Both results are also checked against the FP64 oracle at that tolerance.

Meshes: jittered by U(+-1%) of the edge (seed 0), Morton order, pinned bottom face; d =
U(+-0.02 h) (seed 10), u = U(-1, 1) (seed 11).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1506_07577_amd import meshgen as mg

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1506_07577_amd import ebbx
else:  # collected on a CPU host only to be deselected
    ebbx = None


def nerr(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _case(n, model, prec, strategy, block):
    m = mg.jitter(mg.kuhn_cube(n), 0.01, seed=0)
    E, nu = (1e6, 0.45) if model == "nh" else (1e5, 0.3)
    mdl = ebbx.NH if model == "nh" else ebbx.STVK
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=mdl, elem_prec=ebbx.F32 if prec == "f32" else ebbx.F64,
                        E=E, nu=nu, strategy=strategy, block=block, morton=True)
    ref = oracle.FEM.create(mdl, m.X, m.tets, E, nu, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    u = mg.direction(m, 11)
    return mesh, d, u, ref.kmul(d, u)


# (strategy name, tets or blocks per workgroup, model, element precision, deterministic)
CASES = [
    ("BLOCK", 256, "nh", "f32", True),
    ("BLOCK", 128, "stvk", "f64", True),
    ("PIPE", 4, "nh", "f32", True),
    ("LANES", 128, "stvk", "f64", True),
    ("SEG", 0, "nh", "f64", True),
    ("OWNER", 0, "stvk", "f32", True),
    ("BLOCK_LDS", 256, "stvk", "f64", False),
    ("ATOMIC", 0, "nh", "f64", False),
]


@pytest.mark.parametrize("strat,block,model,prec,det", CASES)
def test_noalloc_matches_kmul_two_calls(strat, block, model, prec, det):
    tol = 1e-5 if prec == "f32" else 1e-10
    strategy = getattr(ebbx, "STRAT_" + strat)
    print(f"[noalloc] {strat}/{block} {model} {prec}: 14^3 then 8^3", flush=True)
    big = _case(14, model, prec, strategy, block)
    small = _case(8, model, prec, strategy, block)
    outs = []
    for mesh, d, u, yr in (big, small):   # two allocation-free calls in a row, the second smaller
        dd, ud = mesh.to_dev(d), mesh.to_dev(u)
        y = torch.full_like(dd, float("nan"))
        mesh.fem.kmul_noalloc(dd, ud, y)
        outs.append((mesh, dd, ud, yr, y))
    torch.cuda.synchronize()
    for mesh, dd, ud, yr, y in outs:
        y_ref = mesh.fem.kmul(dd, ud)
        torch.cuda.synchronize()
        if det:
            assert torch.equal(y, y_ref), (strat, mesh.nt)
        else:
            assert nerr(mesh.from_dev(y), mesh.from_dev(y_ref)) <= tol, (strat, mesh.nt)
        assert nerr(mesh.from_dev(y), yr) <= tol, (strat, mesh.nt)
        # accumulate adds to what the output holds
        y2 = mesh.fem.kmul_noalloc(dd, ud, y.clone(), accumulate=True)
        assert nerr(mesh.from_dev(y2), 2 * yr) <= tol
    for mesh, *_ in (big, small):
        mesh.fem.close()


def test_noalloc_full_size_bench_configuration():
    """The 64^3 neo-Hookean FP32 mesh in the block strategy and Morton order fits the array and
    gives ebbx_fem_Kmul's result bit for bit; its SEG partials (12 FP32 per tet, 75.5 MB) do
    not fit and are refused before any work, leaving the output untouched."""
    w = mg.workload_plain()
    m = w.mesh
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F32, E=w.E, nu=w.nu,
                        strategy=ebbx.STRAT_BLOCK, morton=True)
    d = mg.perturbed_state(m, 0.02, seed=10)
    u = mg.direction(m, 11)
    dd, ud = mesh.to_dev(d), mesh.to_dev(u)
    print("[noalloc] 64^3 NH FP32 BLOCK/256", flush=True)
    y = mesh.fem.kmul_noalloc(dd, ud, torch.empty_like(dd))
    assert torch.equal(y, mesh.fem.kmul(dd, ud))
    ref = oracle.FEM.create(w.model, m.X, m.tets, w.E, w.nu, pinned=m.pinned)
    assert nerr(mesh.from_dev(y), ref.kmul(d, u)) <= 1e-5
    mesh.fem.set_strategy(ebbx.STRAT_SEG, 0)
    keep = torch.full_like(dd, 7.0)
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.kmul_noalloc(dd, ud, keep)
    assert e.value.code == ebbx.E_ARG
    torch.cuda.synchronize()
    assert bool((keep == 7.0).all())
    mesh.fem.close()


def test_noalloc_argument_errors():
    mesh, d, u, _ = _case(4, "stvk", "f64", ebbx.STRAT_BLOCK, 0)
    dd, ud = mesh.to_dev(d), mesh.to_dev(u)
    L = ebbx.lib()
    assert L.ebbx_fem_Kmul_noalloc(mesh.fem.h, dd.data_ptr(), ud.data_ptr(), dd.data_ptr(), 0, None) == ebbx.E_PHASE
    assert L.ebbx_fem_Kmul_noalloc(mesh.fem.h, None, ud.data_ptr(), dd.data_ptr(), 0, None) == ebbx.E_ARG
    assert L.ebbx_fem_Kmul_noalloc(None, dd.data_ptr(), ud.data_ptr(), dd.data_ptr(), 0, None) == ebbx.E_ARG
    mesh.fem.close()
