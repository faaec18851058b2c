"""OWNER strategy (vertex-owned blocks that re-evaluate boundary tets):
bitwise equality with the segmented strategy, whose per-vertex sums run in
the same (tet, corner) order, plus its limits."""
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _two(m, model, prec, vb, morton=True, E_tet=None):
    kw = dict(model=model, elem_prec=ebbx.F64 if prec == "f64" else ebbx.F32, E=1e5, nu=0.3, E_tet=E_tet,
              morton=morton)
    own = ebbx.FemMesh(m.X, m.tets, m.pinned, strategy=ebbx.STRAT_OWNER, block=vb, **kw)
    seg = ebbx.FemMesh(m.X, m.tets, m.pinned, strategy=ebbx.STRAT_SEG, **kw)
    return own, seg


@pytest.mark.parametrize("prec,vb", [("f32", 64), ("f32", 128), ("f64", 64)])
@pytest.mark.parametrize("model", [0, 1])
def test_owner_equals_seg_bitwise(model, prec, vb):
    m = mg.jitter(mg.kuhn_cube(13), 0.01, seed=0)   # 2197 verts: several blocks and a ragged last one
    E = 1e5 * np.exp(0.5 * np.random.default_rng(2).standard_normal(m.nt))
    own, seg = _two(m, model, prec, vb, E_tet=E)
    d = own.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    u = own.to_dev(mg.direction(m, 11))
    w = own.to_dev(mg.direction(m, 12))
    assert torch.equal(own.fem.forces(d), seg.fem.forces(d))
    assert torch.equal(own.fem.jacobi_diag(d, 1e-3), seg.fem.jacobi_diag(d, 1e-3))
    assert torch.equal(own.fem.kmul(d, u), seg.fem.kmul(d, u))
    if vb == 64:
        assert torch.equal(own.fem.tmul(d, u, w), seg.fem.tmul(d, u, w))
    # accumulate
    y = own.fem.kmul(d, u).clone()
    own.fem.kmul(d, u, y=y, accumulate=True)
    assert torch.equal(y, 2 * seg.fem.kmul(d, u))


def test_owner_matches_oracle_and_steps():
    m = mg.jitter(mg.kuhn_cube(10), 0.01, seed=0)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F32, E=1e6, nu=0.45,
                        strategy=ebbx.STRAT_OWNER, morton=True)
    ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, 1e6, 0.45, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    u = mg.direction(m, 11)
    y = mesh.from_dev(mesh.fem.kmul(mesh.to_dev(d), mesh.to_dev(u)))
    e = ref.kmul(d, u)
    assert np.abs(y - e).max() / np.abs(e).max() < 1e-5
    z = np.zeros((m.nv, 3))
    dd, vv = mesh.to_dev(z), mesh.to_dev(z)
    st = ebbx.stats_fetch(mesh.fem.implicit_step(dd, vv, 1e-3, tol=1e-8, maxit=300))
    _d1, v1, _dv, so = ref.implicit_step(z, z, 1e-3, tol=1e-8, maxit=300)
    assert st.status == ebbx.OK
    got = mesh.from_dev(vv)
    assert np.abs(got - v1).max() / np.abs(v1).max() < 1e-5


def test_owner_scrambled_and_limits():
    # without Morton order a block's tets reach far: 64 owned vertices still fit, 256 do not
    m, _, _ = mg.scramble(mg.kuhn_cube(20), seed=1)
    own, seg = _two(m, 1, "f32", 64, morton=False)
    d = own.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    assert torch.equal(own.fem.forces(d), seg.fem.forces(d))
    with pytest.raises(ebbx.EbbxError) as e:
        own.fem.set_strategy(ebbx.STRAT_OWNER, 256)
    assert e.value.code == ebbx.E_ARG
    with pytest.raises(ebbx.EbbxError) as e:
        own.fem.set_strategy(ebbx.STRAT_OWNER, 100)
    assert e.value.code == ebbx.E_ARG
    # single tet and isolated vertices
    X = np.vstack([mg.single_tet().X, [[5.0, 5.0, 5.0]]])
    one = ebbx.FemMesh(X, np.array([[0, 1, 2, 3]]), None, model=1, elem_prec=ebbx.F64, strategy=ebbx.STRAT_OWNER)
    ref = oracle.FEM.create(1, X, np.array([[0, 1, 2, 3]], dtype=np.int32), 1e5, 0.3)
    dd = 0.01 * mg.direction(mg.Mesh(X=X, tets=np.array([[0, 1, 2, 3]]), pinned=np.zeros(5, np.uint8)), 3)
    got = one.from_dev(one.fem.forces(one.to_dev(dd)))
    assert np.abs(got - ref.forces(dd)).max() <= 1e-10 * np.abs(ref.forces(dd)).max()
    assert np.all(got[4] == 0.0)
