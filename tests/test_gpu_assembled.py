"""Stiffness assembled on the edges relation (one 3x3 block per ordered vertex
pair sharing a tet) and its block-CSR product, through the C-ABI, against the
oracle.

Tolerances (normwise): edges bit-exact; FP64 blocks 1e-12 of the largest
block entry (per-tet sums in a different order); FP64 products 1e-10; FP32
element storage (B, the material and the blocks rounded to FP32) 1e-5.
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


def _mesh(m, model, prec, morton=False, E=2e5, nu=0.35):
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=model, elem_prec=ebbx.F64 if prec == "f64" else ebbx.F32,
                        E=E, nu=nu, strategy=ebbx.STRAT_BLOCK, morton=morton)
    ref = oracle.FEM.create(model, m.X, m.tets, E, nu, pinned=m.pinned)
    return mesh, ref


def _lib_tets(mesh, m):
    """The tets as the library stores them (Morton-permuted rows and vertex ids)."""
    if mesh.vperm is None:
        return m.tets
    vp = mesh.vperm.cpu().numpy()
    inv = np.empty_like(vp)
    inv[vp] = np.arange(len(vp), dtype=vp.dtype)
    return inv[m.tets[mesh.tperm.cpu().numpy()]]


def _lib_X(mesh, m):
    return m.X if mesh.vperm is None else m.X[mesh.vperm.cpu().numpy()]


@pytest.mark.parametrize("morton", [False, True])
def test_edges_match_oracle(morton):
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(5), 0.01, seed=2), seed=3)
    mesh, _ = _mesh(m, ebbx.NH, "f64", morton=morton)
    row, col, _ = mesh.fem.edges(blocks=False)
    rp_e, col_e = oracle.edges(m.nv, _lib_tets(mesh, m))
    assert np.array_equal(row.cpu().numpy().astype(np.int64), rp_e)
    assert np.array_equal(col.cpu().numpy(), col_e)
    mesh.fem.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("model", [0, 1])
def test_assembled_blocks_and_spmv_parity(model, prec):
    m = mg.jitter(mg.kuhn_cube(6), 0.01, seed=5)
    mesh, ref = _mesh(m, model, prec, morton=True)
    d0 = mg.perturbed_state(m, 0.02, seed=10)
    d = mesh.to_dev(d0)
    mesh.fem.assemble(d)
    row, col, blk = mesh.fem.edges()
    # the oracle assembles on the library's own vertex and tet order
    lt, lX = _lib_tets(mesh, m), _lib_X(mesh, m)
    lref = oracle.FEM.create(model, lX, lt, 2e5, 0.35)
    rp_e, col_e = oracle.edges(m.nv, lt)
    ld = d.t().cpu().numpy()
    want = lref.assemble(ld, rp_e, col_e).reshape(-1, 9).T
    bound = 1e-12 if prec == "f64" else 1e-5
    assert nerr(blk.cpu().numpy(), want) <= bound
    rng = np.random.default_rng(17)
    for _ in range(2):
        u0 = rng.standard_normal((m.nv, 3))
        y = mesh.fem.spmv(mesh.to_dev(u0))
        assert nerr(mesh.from_dev(y), ref.kmul(d0, u0)) <= (1e-10 if prec == "f64" else 1e-5)
    # accumulate, and the library's matrix-free product
    u = mesh.to_dev(rng.standard_normal((m.nv, 3)))
    y0 = torch.ones_like(u)
    mesh.fem.spmv(u, y0, accumulate=True)
    ymf = mesh.fem.kmul(d, u)
    assert nerr((y0 - 1.0).cpu().numpy(), ymf.cpu().numpy()) <= (1e-10 if prec == "f64" else 1e-5)
    mesh.fem.close()


def test_assembly_deterministic_and_reassembled():
    m = mg.jitter(mg.kuhn_cube(5), 0.01, seed=6)
    mesh, ref = _mesh(m, ebbx.NH, "f64", morton=True)
    da, db = mg.perturbed_state(m, 0.02, seed=1), mg.perturbed_state(m, 0.03, seed=2)
    u0 = mg.direction(m, 3)
    u = mesh.to_dev(u0)
    mesh.fem.assemble(mesh.to_dev(da))
    b1 = mesh.fem.edges()[2].clone()
    y1 = mesh.fem.spmv(u).clone()
    mesh.fem.assemble(mesh.to_dev(db))
    assert nerr(mesh.from_dev(mesh.fem.spmv(u)), ref.kmul(db, u0)) <= 1e-10
    mesh.fem.assemble(mesh.to_dev(da))
    assert torch.equal(mesh.fem.edges()[2], b1)
    assert torch.equal(mesh.fem.spmv(u), y1)
    mesh.fem.close()


def test_isolated_vertex_and_errors():
    m = mg.jitter(mg.kuhn_cube(2), 0.01, seed=7)
    X = np.vstack([m.X, [[2.0, 2.0, 2.0]]])
    pinned = np.concatenate([m.pinned, [0]]).astype(np.uint8)
    mesh = ebbx.FemMesh(X, m.tets, pinned, model=ebbx.STVK, elem_prec=ebbx.F64, E=1e5, nu=0.3)
    ref = oracle.FEM.create(ebbx.STVK, X, m.tets, 1e5, 0.3, pinned=pinned)
    z = np.zeros((m.nv + 1, 3))
    u0 = np.random.default_rng(1).standard_normal((m.nv + 1, 3))
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.spmv(mesh.to_dev(u0))
    assert e.value.code == ebbx.E_STATE
    mesh.fem.assemble(mesh.to_dev(z))
    row, _col, _ = mesh.fem.edges(blocks=False)
    assert int(row[-1] - row[-2]) == 0   # the isolated vertex has no edge
    y = mesh.from_dev(mesh.fem.spmv(mesh.to_dev(u0)))
    assert np.all(y[-1] == 0.0)
    assert nerr(y, ref.kmul(z, u0)) <= 1e-10
    u = mesh.to_dev(u0)
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx._check(ebbx.lib().ebbx_fem_spmv(mesh.fem.h, ebbx._ptr(u), ebbx._ptr(u), 0, None))
    assert e.value.code == ebbx.E_PHASE
    mesh.fem.close()


def test_assembled_full_size():
    """64^3 cube (1,572,864 tets), neo-Hookean, FP32 element storage, Morton order: the product
    with the assembled blocks against the oracle's matrix-free K u over the whole mesh."""
    w = mg.workload_plain()
    m = w.mesh
    mesh, ref = _mesh(m, w.model, w.prec, morton=True, E=w.E, nu=w.nu)
    d0 = mg.perturbed_state(m, 0.02, seed=10)
    u0 = mg.direction(m, 11)
    mesh.fem.assemble(mesh.to_dev(d0))
    assert mesh.fem.edge_count() == int(np.diff(oracle.edges(m.nv, m.tets)[0]).sum())
    y = mesh.from_dev(mesh.fem.spmv(mesh.to_dev(u0)))
    assert nerr(y, ref.kmul(d0, u0)) <= 1e-5
    mesh.fem.close()


def test_randomized_assembled():
    """Seeded sweep: 8 jittered cubes of side 1..6 (half scrambled, half Morton-reordered),
    random model, precision and material: edges bit-exact, products against the oracle's K u."""
    rng = np.random.default_rng(91)
    for case in range(8):
        n = int(rng.integers(1, 7))
        m = mg.jitter(mg.kuhn_cube(n), 0.01, seed=int(rng.integers(1 << 30)))
        if rng.random() < 0.5:
            m, _, _ = mg.scramble(m, seed=int(rng.integers(1 << 30)))
        model = int(rng.integers(0, 2))
        prec = "f64" if rng.random() < 0.5 else "f32"
        E, nu = float(10 ** rng.uniform(4, 6)), float(rng.uniform(0.25, 0.45))
        mesh, ref = _mesh(m, model, prec, morton=bool(rng.random() < 0.5), E=E, nu=nu)
        d0 = mg.perturbed_state(m, 0.01, seed=int(rng.integers(1 << 30)))
        u0 = rng.standard_normal((m.nv, 3))
        mesh.fem.assemble(mesh.to_dev(d0))
        row, col, _ = mesh.fem.edges(blocks=False)
        rp_e, col_e = oracle.edges(m.nv, _lib_tets(mesh, m))
        case_id = (case, n, model, prec)
        assert np.array_equal(row.cpu().numpy().astype(np.int64), rp_e), case_id
        assert np.array_equal(col.cpu().numpy(), col_e), case_id
        y = mesh.from_dev(mesh.fem.spmv(mesh.to_dev(u0)))
        assert nerr(y, ref.kmul(d0, u0)) <= (1e-10 if prec == "f64" else 1e-5), case_id
        mesh.fem.close()
