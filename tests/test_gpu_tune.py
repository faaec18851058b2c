"""Autotuner: timing every strategy and block size, choosing the fastest,
and the JSON cache of choices."""
import json

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


def _mesh(n, morton=True):
    m = mg.jitter(mg.kuhn_cube(n), 0.01, seed=0)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F32, E=1e6, nu=0.45,
                        strategy=ebbx.STRAT_AUTO, morton=morton)
    return m, mesh


def test_autotune_picks_fastest_and_results_stay_correct(tmp_path):
    m, mesh = _mesh(24)
    assert mesh.fem.get_strategy() == (ebbx.STRAT_BLOCK, 256)   # AUTO before tuning
    d = mesh.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    u = mesh.to_dev(mg.direction(m, 11))
    res = mesh.fem.autotune(d, u)
    strategies = {r[0] for r in res}
    assert {ebbx.STRAT_BLOCK, ebbx.STRAT_BLOCK_LDS, ebbx.STRAT_SEG, ebbx.STRAT_ATOMIC} <= strategies
    assert all(r[2] > 0 for r in res)
    best = min(res, key=lambda r: r[2])
    assert mesh.fem.get_strategy() == (best[0], best[1])
    ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, 1e6, 0.45, pinned=m.pinned)
    exp = ref.kmul(mg.perturbed_state(m, 0.02, seed=10), mg.direction(m, 11))
    got = mesh.from_dev(mesh.fem.kmul(d, u))
    assert np.abs(got - exp).max() / np.abs(exp).max() < 1e-5
    # the step after tuning rebuilds its graphs with the chosen strategy
    st = mesh.fem.implicit_step(d.clone(), torch.zeros_like(d), 1e-3, tol=1e-8, maxit=200)
    assert ebbx.stats_fetch(st).status == ebbx.OK


def test_autotune_cache(tmp_path):
    path = str(tmp_path / "tune.json")
    m, mesh = _mesh(12)
    first = mesh.fem.autotune(cache=path)
    assert len(first) >= 8
    choice = mesh.fem.get_strategy()
    with open(path) as fh:
        data = json.load(fh)
    assert len(data) == 1
    (entry,) = data.values()
    assert (entry["strategy"], entry["block"]) == choice
    # a hit: no timing, same choice, even from another strategy
    mesh.fem.set_strategy(ebbx.STRAT_ATOMIC, 64)
    again = mesh.fem.autotune(cache=path)
    assert again == [] and mesh.fem.get_strategy() == choice
    # another mesh (other keys) adds an entry
    _m2, mesh2 = _mesh(12, morton=False)
    assert len(mesh2.fem.autotune(cache=path)) >= 8
    with open(path) as fh:
        assert len(json.load(fh)) == 2
    with pytest.raises(ebbx.EbbxError) as e:
        mesh2.fem.autotune(cache=str(tmp_path / "no_such_dir" / "t.json"))
    assert e.value.code == ebbx.E_ARG


def test_autotune_two_tets_per_thread_candidates():
    """The tuner times blocks with two tets per thread too; such a choice is a valid strategy
    whose products match the oracle."""
    m, mesh = _mesh(16)
    res = mesh.fem.autotune()
    two = [(s, b) for s, b, _us in res if s == ebbx.STRAT_BLOCK and b & ebbx.BLOCK_TPT2]
    assert len(two) == 3
    ref = oracle.FEM.create(ebbx.NH, m.X, m.tets, 1e6, 0.45, pinned=m.pinned)
    d0, u0 = mg.perturbed_state(m, 0.02, seed=10), mg.direction(m, 11)
    exp = ref.kmul(d0, u0)
    for s, b in two:
        mesh.fem.set_strategy(s, b)
        assert mesh.fem.get_strategy() == (s, b)
        got = mesh.from_dev(mesh.fem.kmul(mesh.to_dev(d0), mesh.to_dev(u0)))
        assert np.abs(got - exp).max() / np.abs(exp).max() < 1e-5, b
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.set_strategy(ebbx.STRAT_BLOCK, 64 | ebbx.BLOCK_TPT2)
    assert e.value.code == ebbx.E_ARG
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.set_strategy(ebbx.STRAT_LANES, 128 | ebbx.BLOCK_TPT2)
    assert e.value.code == ebbx.E_ARG


def test_autotune_batch_union_picks_fastest():
    """On a batch's union domain (six meshes of uneven size) the tuner keeps the fastest
    candidate, and the batched step under that choice matches the oracle mesh by mesh."""
    sides = (3, 7, 4, 9, 5, 6)
    meshes = [mg.jitter(mg.kuhn_cube(n), 0.01, seed=100 + i) for i, n in enumerate(sides)]
    E = np.array([1e5, 3e5, 2e4, 8e5, 1e5, 5e4])
    nu = np.array([0.3, 0.4, 0.35, 0.45, 0.3, 0.42])
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    res = bm.batch.fem.autotune()
    assert len(res) >= 8 and all(r[2] > 0 for r in res)
    best = min(res, key=lambda r: r[2])
    assert bm.batch.fem.get_strategy() == (best[0], best[1])
    dd = torch.zeros(3, un.nv, dtype=torch.float64, device="cuda")
    vv = torch.zeros_like(dd)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-12, maxit=500))
    assert all(s.status == ebbx.OK for s in st)
    gv = bm.from_dev(vv)
    for i, mi in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        ref = oracle.FEM.create(ebbx.NH, mi.X, mi.tets, E[i], nu[i], pinned=mi.pinned)
        z = np.zeros((mi.nv, 3))
        _d1, v1, _dv, _s = ref.implicit_step(z, z, 1e-3, tol=1e-12, maxit=500)
        assert np.abs(gv[a:b] - v1).max() / np.abs(v1).max() < 1e-9, i
    bm.batch.close()
