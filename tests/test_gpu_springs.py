"""Spring-mass workload (the paper's introductory example) on the relational
runtime, through the C-ABI, against the oracle.

Tolerances (normwise): rest lengths 1e-15 (one square root of the same sum);
forces 1e-12 (sums over a vertex's edges in another order); trajectories of
explicit steps 1e-10 after 100 steps and 1e-9 after 200 steps at full size
(rounding differences carried through the steps); kinetic energy 1e-13.
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


def _case(n=5, seed=3, K=1.0, shuffle=True):
    """Jittered, scrambled n^3 cube; its directed edges in a shuffled row order."""
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(n), 0.02, seed=seed), seed=seed + 1)
    tail, head = mg.directed_edges(m.tets, m.nv)
    if shuffle:
        p = np.random.default_rng(seed).permutation(len(tail))
        tail, head = tail[p], head[p]
    rng = np.random.default_rng(seed + 2)
    mass = (1.0 + 0.5 * rng.uniform(-1, 1, m.nv)) / m.nv
    q0 = m.X + (0.1 / n) * rng.uniform(-1, 1, (m.nv, 3))
    qd0 = 0.05 * rng.uniform(-1, 1, (m.nv, 3))
    sm = ebbx.SpringMesh(m.X, tail, head, K)
    ref = oracle.Springs(m.X, tail, head, mass, K)
    return m, tail, head, mass, q0, qd0, sm, ref


def test_rest_lengths_and_forces():
    m, tail, head, mass, q0, _qd0, sm, ref = _case()
    order = np.lexsort((np.arange(len(tail)), tail))   # edges grouped by tail, rows ascending
    rest = sm.springs.rest().cpu().numpy()
    assert nerr(rest, ref.rest[: len(tail)][order]) <= 1e-15
    f = sm.springs.forces(sm.to_dev(q0))
    assert nerr(sm.from_dev(f), ref.forces(q0)) <= 1e-12
    # at rest the springs are relaxed
    assert np.abs(sm.from_dev(sm.springs.forces(sm.to_dev(m.X)))).max() <= 1e-14
    # accumulate (+=) into an existing force field
    f2 = torch.ones_like(f)
    sm.springs.forces(sm.to_dev(q0), f2, accumulate=True)
    assert nerr(sm.from_dev(f2) - 1.0, ref.forces(q0)) <= 1e-12
    sm.springs.close()


def test_steps_and_graph_run():
    _m, _t, _h, mass, q0, qd0, sm, ref = _case(n=6, seed=7)
    dt = 1e-4
    qs, qds = q0.copy(), qd0.copy()
    for _ in range(100):
        qs, qds = ref.step(qs, qds, dt)
    md = torch.as_tensor(mass).cuda()
    # kernel by kernel
    q, qd = sm.to_dev(q0), sm.to_dev(qd0)
    f = torch.zeros_like(q)
    for _ in range(100):
        sm.springs.forces(q, f, accumulate=True)
        sm.springs.apply(md, dt, q, qd, f)
    assert float(f.abs().max()) == 0.0
    assert nerr(sm.from_dev(q), qs) <= 1e-10 and nerr(sm.from_dev(qd), qds) <= 1e-10
    qa, qda = q.clone(), qd.clone()
    # the captured graph: 100 = 3 x 32 + 4, bitwise equal to the kernel-by-kernel run
    q, qd = sm.to_dev(q0), sm.to_dev(qd0)
    f = torch.zeros_like(q)
    sm.springs.run(md, dt, 100, q, qd, f)
    assert torch.equal(q, qa) and torch.equal(qd, qda)
    # nsteps = 0 is a no-op; a new dt recaptures
    sm.springs.run(md, dt, 0, q, qd, f)
    assert torch.equal(q, qa)
    sm.springs.run(md, 2 * dt, 33, q, qd, f)
    for _ in range(33):
        qs, qds = ref.step(qs, qds, 2 * dt)
    assert nerr(sm.from_dev(qd), qds) <= 1e-10
    sm.springs.close()


def test_fused_run_matches_separate_passes():
    """run() advances through fused steps and a second position buffer; for odd and even step
    counts, below and above one captured chunk, and with a nonzero force field on entry, its
    positions, velocities and cleared force equal the separate passes bit for bit."""
    _m, _t, _h, mass, q0, qd0, sm, _ref = _case(n=5, seed=13)
    md = torch.as_tensor(mass).cuda()
    dt = 3e-4
    fext = np.random.default_rng(14).uniform(-1, 1, q0.shape)
    for steps in (1, 2, 7, 8, 33, 64, 65):
        for with_f in (False, True):
            q, qd = sm.to_dev(q0), sm.to_dev(qd0)
            f = sm.to_dev(fext) if with_f else torch.zeros_like(q)
            for _ in range(steps):
                sm.springs.forces(q, f, accumulate=True)
                sm.springs.apply(md, dt, q, qd, f)
            qr, qdr, fr = sm.to_dev(q0), sm.to_dev(qd0), (sm.to_dev(fext) if with_f else torch.zeros_like(q))
            sm.springs.run(md, dt, steps, qr, qdr, fr)
            case_id = (steps, with_f)
            assert torch.equal(qr, q) and torch.equal(qdr, qd), case_id
            assert float(fr.abs().max()) == 0.0, case_id
    sm.springs.close()


def test_kinetic_energy_global_sum():
    _m, _t, _h, mass, _q0, qd0, sm, ref = _case(n=4, seed=11)
    md = torch.as_tensor(mass).cuda()
    qd = sm.to_dev(qd0)
    E = sm.springs.kinetic_energy(md, qd)
    want = ref.kinetic_energy(qd0)
    assert abs(float(E) - want) <= 1e-13 * want
    sm.springs.kinetic_energy(md, qd, E)    # += into the global
    assert abs(float(E) - 2 * want) <= 1e-13 * want
    E2 = sm.springs.kinetic_energy(md, qd)
    assert float(E2) * 2 == float(E)       # fixed-order sums: bitwise reproducible
    sm.springs.close()


def test_spring_errors():
    m, tail, head, mass, q0, qd0, sm, _ref = _case(n=2, seed=1)
    q = sm.to_dev(q0)
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx._check(ebbx.lib().ebbx_springs_forces(sm.springs.h, ebbx._ptr(q), ebbx._ptr(q), 0, None))
    assert e.value.code == ebbx.E_PHASE
    md = torch.as_tensor(mass).cuda()
    with pytest.raises(ebbx.EbbxError) as e:
        sm.springs.apply(md, 1e-4, q, q, torch.zeros_like(q))
    assert e.value.code == ebbx.E_PHASE
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx.Springs(sm.edges, sm.verts, float("nan"))
    assert e.value.code == ebbx.E_ARG
    pairs = ebbx.Relation("pairs", len(tail))
    pairs.bind_keyfield("tail", sm.verts, torch.as_tensor(np.stack([tail, head])).to(torch.int32).cuda())
    pairs.bind_keyfield("head", sm.verts, torch.as_tensor(head).to(torch.int32).cuda())
    with pytest.raises(ebbx.EbbxError) as e:
        ebbx.Springs(pairs, sm.verts, 1.0)
    assert e.value.code == ebbx.E_SHAPE
    sm.springs.close()


def test_springs_full_size():
    """Spring-mass on the 64^3 Kuhn cube (274,625 vertices, 3,744,128 directed edges), K = 1,
    dt = 1e-4: 200 steps from the captured graph against 200 oracle steps."""
    w = mg.workload_springs(64)
    m = w.mesh
    sm = ebbx.SpringMesh(m.X, w.tail, w.head, w.K)
    ref = oracle.Springs(m.X, w.tail, w.head, w.mass, w.K)
    md = torch.as_tensor(w.mass).cuda()
    q, qd = sm.to_dev(w.q0), sm.to_dev(w.qd0)
    f = torch.zeros_like(q)
    sm.springs.run(md, w.dt, 200, q, qd, f)
    qs, qds = w.q0, w.qd0
    for _ in range(200):
        qs, qds = ref.step(qs, qds, w.dt)
    assert nerr(sm.from_dev(q) - w.q0, qs - w.q0) <= 1e-9
    assert nerr(sm.from_dev(qd), qds) <= 1e-9
    E = float(sm.springs.kinetic_energy(md, qd))
    assert abs(E - ref.kinetic_energy(qds)) <= 1e-9 * E
    sm.springs.close()


def test_springs_wide_index_span():
    """A scrambled 40^3 mesh (68,921 vertices, heads up to the whole index range away from their
    tails): forces, then 34 steps (one captured chunk of fused steps and two direct ones) against
    the oracle."""
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(40), 0.02, seed=21), seed=22)
    tail, head = mg.directed_edges(m.tets, m.nv)
    assert np.abs(head.astype(np.int64) - tail).max() > 32767
    rng = np.random.default_rng(23)
    mass = (1.0 + 0.5 * rng.uniform(-1, 1, m.nv)) / m.nv
    q0 = m.X + (0.1 / 40) * rng.uniform(-1, 1, (m.nv, 3))
    qd0 = 0.05 * rng.uniform(-1, 1, (m.nv, 3))
    sm = ebbx.SpringMesh(m.X, tail, head, 1.3)
    ref = oracle.Springs(m.X, tail, head, mass, 1.3)
    assert nerr(sm.from_dev(sm.springs.forces(sm.to_dev(q0))), ref.forces(q0)) <= 1e-12
    md = torch.as_tensor(mass).cuda()
    q, qd = sm.to_dev(q0), sm.to_dev(qd0)
    sm.springs.run(md, 1e-4, 34, q, qd, torch.zeros_like(q))
    qs, qds = q0, qd0
    for _ in range(34):
        qs, qds = ref.step(qs, qds, 1e-4)
    assert nerr(sm.from_dev(qd), qds) <= 1e-10
    assert nerr(sm.from_dev(q) - q0, qs - q0) <= 1e-10
    sm.springs.close()


def test_springs_morton_order():
    """The domain over Morton-ordered vertices and edges (the runtime's reorder of both
    relations): forces and 40 steps against the oracle in the caller's order."""
    m, tail, head, mass, q0, qd0, _sm, ref = _case(n=9, seed=31)
    sm = ebbx.SpringMesh(m.X, tail, head, 1.0, morton=True)
    assert sm.vperm is not None
    assert nerr(sm.from_dev(sm.springs.forces(sm.to_dev(q0))), ref.forces(q0)) <= 1e-12
    md = sm.scalar_to_dev(mass)
    q, qd = sm.to_dev(q0), sm.to_dev(qd0)
    sm.springs.run(md, 1e-4, 40, q, qd, torch.zeros_like(q))
    qs, qds = q0, qd0
    for _ in range(40):
        qs, qds = ref.step(qs, qds, 1e-4)
    assert nerr(sm.from_dev(qd), qds) <= 1e-10
    assert nerr(sm.from_dev(q) - q0, qs - q0) <= 1e-10
    sm.springs.close()
    _sm.springs.close()


def test_randomized_springs():
    """Seeded sweep: 8 cubes of side 1..6 with shuffled (or sorted) edge rows, random K and dt:
    forces, then 20 steps (launched directly) or 40 (one captured chunk of 32 plus 8) against the
    oracle."""
    rng = np.random.default_rng(123)
    for case in range(8):
        n = int(rng.integers(1, 7))
        K = float(10 ** rng.uniform(-1, 1))
        m, tail, head, mass, q0, qd0, sm, ref = _case(n=n, seed=int(rng.integers(1 << 20)), K=K,
                                                    shuffle=bool(rng.random() < 0.5))
        dt = float(10 ** rng.uniform(-5, -4))
        md = torch.as_tensor(mass).cuda()
        f = sm.springs.forces(sm.to_dev(q0))
        case_id = (case, n, K, dt)
        assert nerr(sm.from_dev(f), ref.forces(q0)) <= 1e-12, case_id
        steps = 20 if case % 2 else 40
        q, qd = sm.to_dev(q0), sm.to_dev(qd0)
        f = torch.zeros_like(q)
        sm.springs.run(md, dt, steps, q, qd, f)
        qs, qds = q0, qd0
        for _ in range(steps):
            qs, qds = ref.step(qs, qds, dt)
        assert nerr(sm.from_dev(qd), qds) <= 1e-10, case_id
        sm.springs.close()
