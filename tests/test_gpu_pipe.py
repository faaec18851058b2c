"""The pipelined super-block strategy (PIPE) at full size and across its super-block sizes.

Workload: the 64^3 Kuhn cube (1,572,864 tets), neo-Hookean, E = 1e6, nu = 0.45, FP32 element
math with FP64 vectors, Morton order; d = U(+-0.02 h) (seed 10), u = U(-1, 1) (seed 11).
Tolerance 1e-5 normwise against the oracle (FP64); equal strategies bit for bit run to run.
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


@pytest.fixture(scope="module")
def full():
    w = mg.workload_plain()
    m = w.mesh
    ref = oracle.FEM.create(w.model, m.X, m.tets, w.E, w.nu, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    u = mg.direction(m, 11)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F32, E=w.E, nu=w.nu,
                        strategy=ebbx.STRAT_PIPE, morton=True)
    yield w, ref, d, u, ref.forces(d), ref.kmul(d, u), mesh
    mesh.fem.close()


@pytest.mark.parametrize("g", [1, 2, 3, 4, 6, 8, 12])
def test_pipe_full_size(full, g):
    w, ref, d, u, fr, yr, mesh = full
    mesh.fem.set_strategy(ebbx.STRAT_PIPE, g)
    assert mesh.fem.get_strategy() == (ebbx.STRAT_PIPE, g)
    print(f"[pipe] 64^3 NH FP32 Morton, {g} blocks per workgroup", flush=True)
    dd, ud = mesh.to_dev(d), mesh.to_dev(u)
    f = mesh.fem.forces(dd).clone()
    y = mesh.fem.kmul(dd, ud).clone()
    assert nerr(mesh.from_dev(f), fr) <= 1e-5
    assert nerr(mesh.from_dev(y), yr) <= 1e-5
    assert torch.equal(mesh.fem.kmul(dd, ud), y) and torch.equal(mesh.fem.forces(dd), f)
    # accumulate adds to what the output holds
    y2 = mesh.fem.kmul(dd, ud, y=y.clone(), accumulate=True)
    assert nerr(mesh.from_dev(y2), 2 * yr) <= 1e-5


def test_pipe_super_block_vertex_limit(full):
    """16 blocks of this mesh per workgroup touch more than 1023 vertices: refused, and the
    domain keeps its strategy."""
    w, ref, d, u, fr, yr, mesh = full
    mesh.fem.set_strategy(ebbx.STRAT_PIPE, 6)
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.set_strategy(ebbx.STRAT_PIPE, 16)
    assert e.value.code == ebbx.E_ARG
    assert mesh.fem.get_strategy() == (ebbx.STRAT_PIPE, 6)
    assert nerr(mesh.from_dev(mesh.fem.kmul(mesh.to_dev(d), mesh.to_dev(u))), yr) <= 1e-5


def test_pipe_and_block_switch(full):
    """PIPE replaces the block strategy's halo tables with super-block ones; switching back and
    forth rebuilds them, and each strategy keeps matching the oracle."""
    w, ref, d, u, fr, yr, mesh = full
    dd, ud = mesh.to_dev(d), mesh.to_dev(u)
    for strat, blk in [(ebbx.STRAT_BLOCK, 256), (ebbx.STRAT_PIPE, 4), (ebbx.STRAT_BLOCK, 128),
                       (ebbx.STRAT_PIPE, 3)]:
        mesh.fem.set_strategy(strat, blk)
        assert nerr(mesh.from_dev(mesh.fem.kmul(dd, ud)), yr) <= 1e-5, (strat, blk)


def test_pipe_refuses_scrambled_blocks():
    m, _, _ = mg.scramble(mg.kuhn_cube(12), seed=1)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.STVK, elem_prec=ebbx.F64, strategy=ebbx.STRAT_BLOCK)
    with pytest.raises(ebbx.EbbxError) as e:
        mesh.fem.set_strategy(ebbx.STRAT_PIPE, 4)
    assert e.value.code == ebbx.E_STATE
    # the domain keeps its previous strategy and still computes
    ref = oracle.FEM.create(ebbx.STVK, m.X, m.tets, 1e5, 0.3, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    assert nerr(mesh.from_dev(mesh.fem.forces(mesh.to_dev(d))), ref.forces(d)) <= 1e-10
    mesh.fem.close()
