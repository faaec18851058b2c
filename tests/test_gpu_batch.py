"""Batched implicit step (many meshes, one set of relations, per-mesh CG)
through the C-ABI against the oracle run mesh by mesh.

Each mesh of a batch is an independent implicit step, so the oracle is the
plain step applied to each mesh on its own.  Tolerances (normwise per mesh):
FP64 elements with both solves run to 1e-12: 1e-9; FP32 elements: 1e-5.
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


def _small_batch(sides=(1, 3, 2, 4, 1, 5, 2), seed=4):
    rng = np.random.default_rng(seed)
    meshes = [mg.jitter(mg.kuhn_cube(n), 0.01, seed=100 + i) for i, n in enumerate(sides)]
    E = 10.0 ** rng.uniform(4.0, 6.0, len(sides))
    nu = rng.uniform(0.3, 0.45, len(sides))
    return meshes, E, nu


def _states(un, seed=10, amp=0.002):
    """Small seeded initial displacement and velocity over the union."""
    rng = np.random.default_rng(seed)
    d = amp * rng.uniform(-1, 1, (un.nv, 3))
    v = 0.05 * rng.uniform(-1, 1, (un.nv, 3))
    d[un.pinned == 1] = 0.0
    v[un.pinned == 1] = 0.0
    return d, v


def _oracle_steps(meshes, un, E, nu, d, v, dt, tol, maxit, model):
    out_d, out_v, stats = [], [], []
    for i, m in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        ref = oracle.FEM.create(model, m.X, m.tets, E[i], nu[i], pinned=m.pinned)
        d1, v1, _dv, st = ref.implicit_step(d[a:b], v[a:b], dt, tol=tol, maxit=maxit)
        out_d.append(d1)
        out_v.append(v1)
        stats.append(st)
    return out_d, out_v, stats


@pytest.mark.parametrize("morton", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("model", [ebbx.NH if ebbx else 1, ebbx.STVK if ebbx else 0])
def test_batch_step_parity(prec, model, morton):
    """Lattice order, and Morton order within each mesh (the union reordered by the runtime)."""
    meshes, E, nu = _small_batch()
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=model, elem_prec=ebbx.F64 if prec == "f64" else ebbx.F32, morton=morton)
    d, v = _states(un)
    dt, tol = 1e-3, (1e-12 if prec == "f64" else 1e-8)
    dd, vv = bm.to_dev(d), bm.to_dev(v)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, dt, tol=tol, maxit=1000))
    ed, ev, est = _oracle_steps(meshes, un, E, nu, d, v, dt, tol, 1000, model)
    gd, gv = bm.from_dev(dd), bm.from_dev(vv)
    bound = 1e-9 if prec == "f64" else 1e-5
    for i in range(len(meshes)):
        a, b = un.vptr[i], un.vptr[i + 1]
        assert st[i].status == ebbx.OK, (i, st[i].status)
        assert st[i].rel_res <= tol
        if prec == "f64":
            assert abs(st[i].iters - est[i].iters) <= 2
        assert nerr(gv[a:b], ev[i]) < bound, i
        assert nerr(gd[a:b] - d[a:b], ed[i] - d[a:b]) < bound, i


def test_batch_mesh_results_equal_single_mesh_solves_bitwise():
    # segmented strategy: the union's per-vertex sums and per-mesh dot products run in the
    # same order as each mesh's own solve, so every mesh matches its plain step bit for bit
    meshes, E, nu = _small_batch(sides=(2, 4, 3, 1))
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F32, strategy=ebbx.STRAT_SEG)
    d, v = _states(un)
    dd, vv = bm.to_dev(d), bm.to_dev(v)
    bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-8, maxit=200)
    gd, gv = bm.from_dev(dd), bm.from_dev(vv)
    for i, m in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        one = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F32, E=E[i], nu=nu[i],
                           strategy=ebbx.STRAT_SEG)
        d1, v1 = one.to_dev(d[a:b]), one.to_dev(v[a:b])
        one.fem.implicit_step(d1, v1, 1e-3, tol=1e-8, maxit=200)
        assert np.array_equal(one.from_dev(d1), gd[a:b]), i
        assert np.array_equal(one.from_dev(v1), gv[a:b]), i


def test_batch_per_mesh_outcomes():
    # mesh 0: fully pinned (b = 0: converged in 0 iterations); mesh 1: an inverted tet (NH);
    # mesh 2: stiff; mesh 3: soft.  Each mesh reports and applies its own outcome.
    meshes, E, nu = _small_batch(sides=(2, 2, 3, 3))
    meshes[0].pinned[:] = 1
    E = np.array([1e5, 1e5, 1e6, 1e4])
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    d, v = _states(un)
    d[: un.vptr[1]] = 0.0
    v[: un.vptr[1]] = 0.0
    # invert the first tet of mesh 1 by pushing its 4th corner through the opposite face
    t = un.tets[un.tptr[1]]
    x = un.X[t]
    c = x[:3].mean(axis=0)
    d[t[3]] = 2.0 * (c - x[3])
    dd, vv = bm.to_dev(d), bm.to_dev(v)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-10, maxit=500))
    gd, gv = bm.from_dev(dd), bm.from_dev(vv)
    assert st[0].status == ebbx.OK and st[0].iters == 0 and st[0].rel_res == 0.0
    assert st[1].status == ebbx.E_INVERTED and st[1].n_inverted >= 1
    a, b = un.vptr[1], un.vptr[2]
    assert np.array_equal(gd[a:b], d[a:b]) and np.array_equal(gv[a:b], v[a:b])   # left unchanged
    assert st[2].status == ebbx.OK and st[3].status == ebbx.OK
    assert st[2].iters != st[3].iters
    _ed, ev, est = _oracle_steps(meshes[2:], mg.union(meshes[2:]), E[2:], nu[2:], d[un.vptr[2]:], v[un.vptr[2]:],
                                 1e-3, 1e-10, 500, ebbx.NH)
    for j, i in enumerate((2, 3)):
        a, b = un.vptr[i], un.vptr[i + 1]
        assert abs(st[i].iters - est[j].iters) <= 2
        assert nerr(gv[a:b], ev[j]) < 1e-8


def test_batch_many_small_meshes():
    """300 meshes of 1 to 3 cells a side (6 to 162 tets; up to dozens of meshes share one 256-tet
    block), a few of them fully pinned (finished before the first iteration) and two with an
    inverted tet: the block lists of the batched solve span two tiles of meshes, keep every block
    that an unfinished mesh touches and list it once, whichever meshes around it have finished.
    Every mesh matches the oracle (FP64, 1e-9) or reports its own outcome."""
    rng = np.random.default_rng(21)
    sides = rng.integers(1, 4, 300)
    meshes, E, nu = _small_batch(sides=tuple(int(x) for x in sides), seed=22)
    pinned = set(int(i) for i in rng.choice(300, 25, replace=False))
    for i in pinned:
        meshes[i].pinned[:] = 1
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    d, v = _states(un, seed=23)
    for i in pinned:
        d[un.vptr[i]:un.vptr[i + 1]] = 0.0
        v[un.vptr[i]:un.vptr[i + 1]] = 0.0
    inverted = [i for i in (7, 151) if i not in pinned]
    for i in inverted:
        t = un.tets[un.tptr[i]]
        x = un.X[t]
        d[t[3]] = 2.0 * (x[:3].mean(axis=0) - x[3])
    dd, vv = bm.to_dev(d), bm.to_dev(v)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-12, maxit=400))
    gv = bm.from_dev(vv)
    iters = set()
    for i, m in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        if i in inverted:
            assert st[i].status == ebbx.E_INVERTED, i
            assert np.array_equal(gv[a:b], v[a:b]), i
            continue
        assert st[i].status == ebbx.OK, (i, st[i].status)
        if i in pinned:
            assert st[i].iters == 0 and np.all(gv[a:b] == 0.0), i
            continue
        iters.add(st[i].iters)
        ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, E[i], nu[i], pinned=m.pinned)
        _d1, v1, _dv, _s = ref.implicit_step(d[a:b], v[a:b], 1e-3, tol=1e-12, maxit=400)
        assert nerr(gv[a:b], v1) < 1e-9, i
    assert len(iters) > 3   # meshes finish at different iterations
    bm.batch.close()


def test_batch_element_maps_cover_every_block():
    """The union's force and stiffness maps (block strategy) over a batch of 815 tet blocks:
    batches deal runs of 64 blocks to the XCDs in turn and map the blocks past the last whole
    round of 8 runs contiguously, so this size runs both paths.  Every mesh's result matches the
    oracle (FP64 elements, 1e-10 normwise per mesh), so each block is evaluated exactly once."""
    sides = (12, 16, 20, 14, 18, 10, 22, 9)
    meshes, E, nu = _small_batch(sides=sides, seed=9)
    un = mg.union(meshes)
    assert 512 < un.nt // 256 < 1024
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    rng = np.random.default_rng(12)
    d = 0.002 * rng.uniform(-1, 1, (un.nv, 3))
    u = rng.uniform(-1, 1, (un.nv, 3))
    dd, ud = bm.to_dev(d), bm.to_dev(u)
    f = bm.from_dev(bm.fem.forces(dd))
    k = bm.from_dev(bm.fem.kmul(dd, ud))
    for i, m in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, E[i], nu[i], pinned=m.pinned)
        assert nerr(f[a:b], ref.forces(d[a:b])) <= 1e-10, i
        assert nerr(k[a:b], ref.kmul(d[a:b], u[a:b])) <= 1e-10, i
    bm.batch.close()


def test_batch_errors():
    meshes, E, nu = _small_batch(sides=(1, 2))
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx._check(ebbx.lib().ebbx_fem_destroy(bm.fem.h))
    assert e.value.code == ebbx.E_STATE
    z = torch.zeros(3, un.nv, dtype=torch.float64, device="cuda")
    with pytest.raises(ebbx.EbbxError) as e:
        bm.fem.implicit_step(z, z.clone(), 1e-3)
    assert e.value.code == ebbx.E_STATE
    # the union's element maps work on every mesh at once
    f = bm.fem.forces(z)
    assert float(f.abs().max()) == 0.0
    # layout violations
    bad = mg.union(meshes)
    bad.vert_mesh = bad.vert_mesh[::-1].copy()
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx.BatchMesh(bad, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    assert e.value.code == ebbx.E_LAYOUT
    cross = mg.union(meshes)
    cross.tets[0, 0] = cross.vptr[1]   # a corner in the next mesh
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx.BatchMesh(cross, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    assert e.value.code in (ebbx.E_LAYOUT, ebbx.E_DEGENERATE)
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx.BatchMesh(un, np.array([1e5, -1.0]), nu, model=ebbx.NH, elem_prec=ebbx.F64)
    assert e.value.code == ebbx.E_ARG


def test_batch_full_size_sampled():
    """256 cubes with sides 8..40 (about 31M tets), neo-Hookean, FP32 elements, per-mesh E and nu,
    CG to 1e-8: every mesh converges; every 8th mesh of the batch (32 meshes), the smallest, a
    median and the largest mesh match the oracle."""
    meshes, E, nu = mg.workload_batch()
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F32)
    dd = torch.zeros(3, un.nv, dtype=torch.float64, device="cuda")
    vv = torch.zeros_like(dd)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-8, maxit=1000))
    assert all(s.status == ebbx.OK for s in st)
    assert max(s.rel_res for s in st) <= 1e-8
    sizes = np.array([m.nt for m in meshes])
    order = np.argsort(sizes, kind="stable")
    pick = sorted(set(range(0, len(meshes), 8)) | {int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    assert len(pick) >= 32
    gv = bm.from_dev(vv)
    for i in pick:
        m = meshes[i]
        a, b = un.vptr[i], un.vptr[i + 1]
        ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, E[i], nu[i], pinned=m.pinned)
        z = np.zeros((m.nv, 3))
        _d1, v1, _dv, _so = ref.implicit_step(z, z, 1e-3, tol=1e-8, maxit=1000)
        assert nerr(gv[a:b], v1) < 1e-5, i
