"""Rayleigh damping in the implicit step (D = alpha M - beta K, K = df/dx) and
in its vector-Jacobian product, through the C-ABI, against the oracle.

Tolerances (normwise, ||a - b||_inf / ||b||_inf): fixed-count FP64 solves:
1e-10 (summation order only); solves run to tol 1e-13 on both sides: 1e-9;
FP32 elements against the FP64 oracle: 1e-5; the 64^3 residual check allows
10x the GPU's reported residual or 1e-5 (FP32 element error).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1506_07577_amd import meshgen as mg

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1506_07577_amd import adjoint, ebbx
else:  # collected on a CPU host only to be deselected
    ebbx = adjoint = None

ALPHA, BETA = 2.5, 4e-3


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


def _strat(name):
    return {"atomic": ebbx.STRAT_ATOMIC, "seg": ebbx.STRAT_SEG, "block": ebbx.STRAT_BLOCK,
            "block_lds": ebbx.STRAT_BLOCK_LDS, "owner": ebbx.STRAT_OWNER, "pipe": ebbx.STRAT_PIPE,
            "lanes": ebbx.STRAT_LANES}[name]


def _pair(m, model, prec, strat, E=1e5, nu=0.3, E_tet=None, morton=False):
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=model, elem_prec=ebbx.F64 if prec == "f64" else ebbx.F32,
                        E=E, nu=nu, E_tet=E_tet, strategy=_strat(strat), morton=morton,
                        block=64 if strat == "owner" else 0)
    ref = oracle.FEM.create(model, m.X, m.tets, E if E_tet is None else E_tet, nu, pinned=m.pinned)
    return mesh, ref


@pytest.mark.parametrize("strat", ["atomic", "seg", "block", "owner", "pipe", "lanes"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("model", [0, 1])
def test_damped_step_parity(model, prec, strat):
    """7^3 cube, jittered, from a perturbed state with a velocity: two fixed-count damped steps."""
    m = mg.jitter(mg.kuhn_cube(7), 0.01, seed=3)
    mesh, ref = _pair(m, model, prec, strat, E=2e5, nu=0.35, morton=(strat in ("block", "pipe")))
    d0 = mg.perturbed_state(m, 0.01, seed=10)
    v0 = 0.1 * mg.direction(m, 11)
    d, v = mesh.to_dev(d0), mesh.to_dev(v0)
    dt, it = 1e-3, 60
    s = ebbx.stats_fetch(mesh.fem.implicit_step(d, v, dt, tol=0.0, maxit=it, alpha=ALPHA, beta=BETA))
    d1, v1, _dv, so = ref.implicit_step(d0, v0, dt, tol=0.0, maxit=it, alpha=ALPHA, beta=BETA)
    bound = 1e-10 if prec == "f64" else 1e-5
    assert s.status == ebbx.OK and s.iters == it == so.iters
    assert nerr(mesh.from_dev(v), v1) <= bound
    assert nerr(mesh.from_dev(d) - d0, d1 - d0) <= bound
    mesh.fem.implicit_step(d, v, dt, tol=0.0, maxit=it, alpha=ALPHA, beta=BETA)
    _d2, v2, _dv, _ = ref.implicit_step(d1, v1, dt, tol=0.0, maxit=it, alpha=ALPHA, beta=BETA)
    assert nerr(mesh.from_dev(v), v2) <= bound
    mesh.fem.close()


def test_damped_rigid_translation_closed_form():
    # nothing pinned, at rest, uniform velocity: v' = (v0 + dt g) / (1 + dt alpha) at every vertex
    m = mg.jitter(mg.kuhn_cube(5), 0.01, seed=1)
    mesh = ebbx.FemMesh(m.X, m.tets, np.zeros(m.nv, np.uint8), model=ebbx.NH, elem_prec=ebbx.F64, E=1e5, nu=0.3,
                        strategy=ebbx.STRAT_BLOCK)
    dt = 1e-2
    g = (0.5, -1.0, -9.81)
    v0 = np.array([0.3, -0.2, 0.7])
    d, v = mesh.to_dev(np.zeros((m.nv, 3))), mesh.to_dev(np.tile(v0, (m.nv, 1)))
    s = ebbx.stats_fetch(mesh.fem.implicit_step(d, v, dt, g=g, tol=1e-14, maxit=500, alpha=4.0, beta=3e-3))
    want = (v0 + dt * np.array(g)) / (1.0 + dt * 4.0)
    assert s.status == ebbx.OK
    assert nerr(mesh.from_dev(v), np.tile(want, (m.nv, 1))) <= 1e-12
    mesh.fem.close()


def test_damping_change_rebuilds_graphs():
    """The captured step graphs bake the coefficients: alternating damped and undamped steps on
    one domain each match the oracle, and repeating a configuration is bitwise reproducible."""
    m = mg.jitter(mg.kuhn_cube(5), 0.01, seed=4)
    mesh, ref = _pair(m, 1, "f64", "block")
    d0 = mg.perturbed_state(m, 0.01, seed=12)
    v0 = 0.1 * mg.direction(m, 13)
    outs = []
    for a, b in ((0.0, 0.0), (ALPHA, 0.0), (0.0, BETA), (ALPHA, BETA), (0.0, 0.0)):
        d, v = mesh.to_dev(d0), mesh.to_dev(v0)
        mesh.fem.implicit_step(d, v, 1e-3, tol=0.0, maxit=40, alpha=a, beta=b)
        _d1, v1, _dv, _ = ref.implicit_step(d0, v0, 1e-3, tol=0.0, maxit=40, alpha=a, beta=b)
        got = mesh.from_dev(v)
        assert nerr(got, v1) <= 1e-10, (a, b)
        outs.append(got)
    assert np.array_equal(outs[0], outs[-1])
    assert not np.array_equal(outs[0], outs[3])
    mesh.fem.close()


def test_damping_argument_errors():
    m = mg.kuhn_cube(2)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F64, E=1e5, nu=0.3)
    z = np.zeros((m.nv, 3))
    for a, b in ((-1.0, 0.0), (0.0, -1e-3), (float("nan"), 0.0), (0.0, float("inf"))):
        d, v = mesh.to_dev(z), mesh.to_dev(z)
        with pytest.raises(ebbx.EbbxError) as e:
            mesh.fem.implicit_step(d, v, 1e-3, maxit=5, alpha=a, beta=b)
        assert e.value.code == ebbx.E_ARG
        assert torch.count_nonzero(v).item() == 0
    mesh.fem.close()


@pytest.mark.parametrize("strategy", ["atomic", "block"])
@pytest.mark.parametrize("model", [0, 1])
def test_damped_step_vjp_parity(model, strategy):
    m = mg.jitter(mg.kuhn_cube(6), 0.01, seed=0)
    E_tet, _, _ = mg.adjoint_recipe(m, seed=2)
    mesh, ref = _pair(m, model, "f64", strategy, E=float(np.median(E_tet)), E_tet=E_tet)
    d_n = mg.perturbed_state(m, 0.002, seed=10)
    v_np1 = 0.05 * mg.direction(m, 11)
    rng = np.random.default_rng(7)
    gx = rng.standard_normal((m.nv, 3))
    gv = rng.standard_normal((m.nv, 3))
    dt = 1e-3
    db_e, vb_e, Eb_e, st_e = ref.step_vjp(d_n, v_np1, gx, gv, dt, tol=1e-13, maxit=2000, alpha=ALPHA, beta=BETA)
    E_bar = torch.zeros(m.nt, dtype=torch.float64, device="cuda")
    db, vb, st = mesh.fem.step_vjp(mesh.to_dev(d_n), mesh.to_dev(v_np1), mesh.to_dev(gx), mesh.to_dev(gv), dt,
                                   tol=1e-13, maxit=2000, E_bar=E_bar, alpha=ALPHA, beta=BETA)
    s = ebbx.stats_fetch(st)
    assert s.status == ebbx.OK and s.rel_res <= 1e-13
    assert abs(s.iters - st_e.iters) <= 2
    assert nerr(mesh.from_dev(db), db_e) < 1e-9
    assert nerr(mesh.from_dev(vb), vb_e) < 1e-9
    assert nerr(mesh.tet_from_dev(E_bar), Eb_e) < 1e-9
    mesh.fem.close()


def test_damped_trajectory_gradient_vs_oracle():
    m = mg.jitter(mg.kuhn_cube(5), 0.01, seed=0)
    E_tet, target, _ = mg.adjoint_recipe(m, seed=2)
    mesh, ref = _pair(m, ebbx.NH, "f64", "block", E=float(np.median(E_tet)), E_tet=E_tet)
    steps, dt, tol = 5, 1e-3, 1e-13
    sim = adjoint.Simulation(fem=mesh.fem, steps=steps, dt=dt, tol=tol, maxit=2000, checkpoint_every=2,
                             alpha=ALPHA, beta=BETA)
    Et = mesh.tet_to_dev(E_tet).requires_grad_(True)
    d0 = torch.zeros(3, mesh.nv, dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = torch.zeros(3, mesh.nv, dtype=torch.float64, device="cuda")
    dT, _vT = adjoint.trajectory(sim, d0, v0, Et)
    L = adjoint.position_loss(mesh.to_dev(m.X), dT, mesh.to_dev(target))
    L.backward()
    z = np.zeros((m.nv, 3))
    L_e, gd0_e, gE_e = oracle.trajectory_grad(ref, z, z, steps, dt, tol, 2000, target, m.X, alpha=ALPHA, beta=BETA)
    assert abs(float(L.detach()) - L_e) <= 1e-10 * abs(L_e)
    assert nerr(mesh.from_dev(d0.grad), gd0_e) < 1e-8
    assert nerr(mesh.tet_from_dev(Et.grad), gE_e) < 1e-8
    mesh.fem.close()


def test_damped_batch_parity():
    rng = np.random.default_rng(5)
    sides = (1, 3, 2, 4, 2)
    meshes = [mg.jitter(mg.kuhn_cube(n), 0.01, seed=200 + i) for i, n in enumerate(sides)]
    E = 10.0 ** rng.uniform(4.0, 6.0, len(sides))
    nu = rng.uniform(0.3, 0.45, len(sides))
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F64)
    d = 0.002 * rng.uniform(-1, 1, (un.nv, 3))
    v = 0.05 * rng.uniform(-1, 1, (un.nv, 3))
    d[un.pinned == 1] = 0.0
    v[un.pinned == 1] = 0.0
    dd, vv = bm.to_dev(d), bm.to_dev(v)
    st = ebbx.stats_parse(bm.batch.implicit_step(dd, vv, 1e-3, tol=1e-12, maxit=1000, alpha=ALPHA, beta=BETA))
    gv = bm.from_dev(vv)
    for i, mi in enumerate(meshes):
        a, b = un.vptr[i], un.vptr[i + 1]
        ref = oracle.FEM.create(ebbx.NH, mi.X, mi.tets, E[i], nu[i], pinned=mi.pinned)
        _d1, v1, _dv, so = ref.implicit_step(d[a:b], v[a:b], 1e-3, tol=1e-12, maxit=1000, alpha=ALPHA, beta=BETA)
        assert st[i].status == ebbx.OK and abs(st[i].iters - so.iters) <= 2
        assert nerr(gv[a:b], v1) < 1e-9, i


def test_damped_plain_workload_residual():
    """One damped step of the 64^3 NH FP32 workload to tol 1e-8: the oracle recomputes the FP64
    residual ||Pi(b - A dv)|| / ||Pi b|| of the GPU iterate."""
    w = mg.workload_plain()
    m = w.mesh
    mesh, ref = _pair(m, w.model, w.prec, "block", E=w.E, nu=w.nu, morton=True)
    d0 = mg.perturbed_state(m, 0.02, seed=10)
    v0 = 0.05 * mg.direction(m, 11)
    d, v = mesh.to_dev(d0), mesh.to_dev(v0)
    dt = w.dt
    s = ebbx.stats_fetch(mesh.fem.implicit_step(d, v, dt, tol=1e-8, maxit=1000, alpha=ALPHA, beta=BETA))
    assert s.status == ebbx.OK and s.rel_res <= 1e-8
    dv = mesh.from_dev(v) - v0
    g = np.array([0.0, 0.0, -9.81])
    M = ref.mass[:, None]
    Kv = ref.kmul(d0, v0)
    b = dt * (ref.forces(d0) + M * g - ALPHA * M * v0 + (dt + BETA) * Kv)
    Ad = (1.0 + dt * ALPHA) * M * dv - (dt * dt + dt * BETA) * ref.kmul(d0, dv)
    free = (m.pinned == 0)[:, None]
    r = np.linalg.norm(((b - Ad) * free).ravel()) / np.linalg.norm((b * free).ravel())
    assert r <= max(10 * s.rel_res, 1e-5)
    mesh.fem.close()


def test_randomized_damped_steps():
    """Seeded sweep: 8 jittered (half of them scrambled) cubes of side 1..5, random model,
    precision, strategy, material, damping and step; two fixed-count steps against the oracle."""
    rng = np.random.default_rng(77)
    for case in range(8):
        n = int(rng.integers(1, 6))
        m = mg.jitter(mg.kuhn_cube(n), 0.01, seed=int(rng.integers(1 << 30)))
        if rng.random() < 0.5:
            m, _, _ = mg.scramble(m, seed=int(rng.integers(1 << 30)))
        model = int(rng.integers(0, 2))
        prec = "f64" if rng.random() < 0.5 else "f32"
        strat = ["atomic", "seg", "block", "owner"][int(rng.integers(0, 4))]
        E, nu = float(10 ** rng.uniform(4, 6)), float(rng.uniform(0.25, 0.45))
        alpha, beta = float(rng.uniform(0, 10)), float(10 ** rng.uniform(-4, -2))
        dt = float(10 ** rng.uniform(-4, -2.5))
        mesh, ref = _pair(m, model, prec, strat, E=E, nu=nu)
        d0 = mg.perturbed_state(m, 0.005, seed=int(rng.integers(1 << 30)))
        v0 = 0.05 * mg.direction(m, int(rng.integers(1 << 30)))
        d, v = mesh.to_dev(d0), mesh.to_dev(v0)
        for _ in range(2):
            mesh.fem.implicit_step(d, v, dt, tol=0.0, maxit=30, alpha=alpha, beta=beta)
            d0, v0, _dv, _ = ref.implicit_step(d0, v0, dt, tol=0.0, maxit=30, alpha=alpha, beta=beta)
        bound = 1e-9 if prec == "f64" else 1e-5
        case_id = (case, n, model, prec, strat, alpha, beta, dt)
        assert nerr(mesh.from_dev(v), v0) <= bound, case_id
        mesh.fem.close()
