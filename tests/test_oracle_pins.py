"""Pins of the CPU oracle against what the mathematics fixes.

None of these re-types the oracle's formulas: they check closed forms,
finite differences, invariants, an independent textbook assembly (Voigt
strain-displacement matrices for linear elasticity), dense linear solves and
brute force.  The paper prints no worked numeric example for its FEM
workloads (Performance Evaluation, Vega and FreeFem++), so no golden value
of the paper's own exists for these functions.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1506_07577_amd import meshgen as mg

MODELS = [oracle.STVK, oracle.NH]


def _rng(s):
    return np.random.default_rng(1000 + s)


# --------------------------------------------------------------------------
# material
# --------------------------------------------------------------------------

def test_lame_values():
    mu, lam = oracle.lame(1e5, 0.3)
    # E = 1e5, nu = 0.3: mu = 1e5/2.6, lam = 3e4/0.52 (hand-computed)
    assert mu == pytest.approx(38461.538461538461, rel=1e-15)
    assert lam == pytest.approx(57692.307692307692, rel=1e-15)
    for E, nu in [(1e6, 0.45), (3.3e4, 0.31), (1.0, 0.0)]:
        mu, lam = oracle.lame(E, nu)
        assert mu * (3 * lam + 2 * mu) / (lam + mu) == pytest.approx(E, rel=1e-14)
        assert lam / (2 * (lam + mu)) == pytest.approx(nu, rel=1e-14, abs=1e-15)


# --------------------------------------------------------------------------
# fixtures (the seeded input generator)
# --------------------------------------------------------------------------

def test_kuhn_cube_structure():
    n = 3
    m = mg.kuhn_cube(n)
    assert m.nv == (n + 1) ** 3 and m.nt == 6 * n ** 3
    P = m.X[m.tets]                           # (nt, 4, 3)
    Dm = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    vol = np.linalg.det(Dm) / 6
    assert np.allclose(vol, m.h ** 3 / 6, rtol=1e-12)
    assert vol.sum() == pytest.approx(1.0, rel=1e-12)
    # conforming: every interior face is shared by exactly two tets
    faces = {}
    for t in range(m.nt):
        for f in itertools.combinations(sorted(m.tets[t]), 3):
            faces[f] = faces.get(f, 0) + 1
    assert set(faces.values()) <= {1, 2}
    boundary = sum(1 for c in faces.values() if c == 1)
    assert boundary == 6 * 2 * n * n
    assert m.pinned.sum() == (n + 1) ** 2
    assert np.all(m.X[m.pinned == 1, 2] == 0.0)


def test_generator_reproducible():
    a = mg.jitter(mg.kuhn_cube(4), 0.01, seed=0)
    b = mg.jitter(mg.kuhn_cube(4), 0.01, seed=0)
    assert np.array_equal(a.X, b.X)
    assert np.max(np.abs(a.X - mg.kuhn_cube(4).X)) <= 0.01 * 0.25
    s1, pv, pt = mg.scramble(mg.kuhn_cube(3), seed=1)
    base = mg.kuhn_cube(3)
    # same geometry per tet after undoing the permutations
    assert np.array_equal(s1.X[s1.tets], base.X[base.tets][pt])


# --------------------------------------------------------------------------
# precompute
# --------------------------------------------------------------------------

def test_precompute_against_numpy():
    m = mg.jitter(mg.kuhn_cube(3), 0.05, seed=5)
    fem = oracle.FEM.create(oracle.STVK, m.X, m.tets, 1e5, 0.3, rho=1000.0)
    P = m.X[m.tets]
    Dm = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    assert np.allclose(fem.V0, np.linalg.det(Dm) / 6, rtol=1e-13)
    eye = np.einsum("tij,tjk->tik", fem.B, Dm)
    assert np.allclose(eye, np.eye(3), atol=1e-12)
    assert fem.mass.sum() == pytest.approx(1000.0 * fem.V0.sum(), rel=1e-13)


def test_precompute_degenerate():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=float)  # flat
    with pytest.raises(oracle.OracleError) as e:
        oracle.FEM.create(oracle.STVK, X, np.array([[0, 1, 2, 3]]), 1e5, 0.3)
    assert e.value.code == oracle.E_DEGENERATE
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 1], [0, 1, 0]], dtype=float)  # inverted
    with pytest.raises(oracle.OracleError):
        oracle.FEM.create(oracle.STVK, X, np.array([[0, 1, 2, 3]]), 1e5, 0.3)


# --------------------------------------------------------------------------
# constitutive closed forms and derivatives
# --------------------------------------------------------------------------

@pytest.mark.parametrize("s", [0.8, 0.97, 1.0, 1.001, 1.3])
def test_uniaxial_closed_forms(s):
    mu, lam = oracle.lame(1e5, 0.3)
    G = np.diag([s - 1.0, 0.0, 0.0])
    # StVK with F = diag(s,1,1): E = diag((s^2-1)/2, 0, 0)
    e = (s * s - 1) / 2
    P = oracle.stress(oracle.STVK, mu, lam, G)
    assert P[0, 0] == pytest.approx(s * (2 * mu + lam) * e, rel=1e-12, abs=1e-9)
    assert P[1, 1] == pytest.approx(lam * e, rel=1e-12, abs=1e-9)
    assert P[2, 2] == pytest.approx(lam * e, rel=1e-12, abs=1e-9)
    assert np.allclose(P - np.diag(np.diag(P)), 0)
    psi = oracle.energy_density(oracle.STVK, mu, lam, G)
    assert psi == pytest.approx((2 * mu + lam) * (s * s - 1) ** 2 / 8, rel=1e-12, abs=1e-12)
    # NH: P11 = mu (s - 1/s) + lam ln(s)/s, P22 = P33 = lam ln s
    P = oracle.stress(oracle.NH, mu, lam, G)
    assert P[0, 0] == pytest.approx(mu * (s - 1 / s) + lam * np.log(s) / s, rel=1e-12, abs=1e-9)
    assert P[1, 1] == pytest.approx(lam * np.log(s), rel=1e-12, abs=1e-9)
    psi = oracle.energy_density(oracle.NH, mu, lam, G)
    ref = 0.5 * mu * (s * s - 1) - mu * np.log(s) + 0.5 * lam * np.log(s) ** 2
    # tr(F^T F) - 3 cancels near s = 1: allow a few ulps of the O(mu) terms
    assert psi == pytest.approx(ref, rel=1e-12, abs=1e-14 * (mu + lam))


@pytest.mark.parametrize("model", MODELS)
def test_stress_is_energy_gradient(model):
    mu, lam = oracle.lame(1e5, 0.3)
    rng = _rng(1)
    for _ in range(4):
        G = 0.1 * rng.standard_normal((3, 3))
        P = oracle.stress(model, mu, lam, G)
        eps = 1e-6
        fd = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                E = np.zeros((3, 3))
                E[i, j] = eps
                fd[i, j] = (oracle.energy_density(model, mu, lam, G + E)
                            - oracle.energy_density(model, mu, lam, G - E)) / (2 * eps)
        assert np.max(np.abs(fd - P)) <= 1e-6 * np.max(np.abs(P))


@pytest.mark.parametrize("model", MODELS)
def test_dstress_d2stress_fd_and_symmetry(model):
    mu, lam = oracle.lame(1e5, 0.3)
    rng = _rng(2)
    for _ in range(4):
        G = 0.1 * rng.standard_normal((3, 3))
        A = rng.standard_normal((3, 3))
        W = rng.standard_normal((3, 3))
        eps = 1e-6
        dP = oracle.dstress(model, mu, lam, G, A)
        fd = (oracle.stress(model, mu, lam, G + eps * A)
              - oracle.stress(model, mu, lam, G - eps * A)) / (2 * eps)
        assert np.max(np.abs(fd - dP)) <= 1e-6 * np.max(np.abs(dP))
        # major symmetry of the elasticity tensor
        assert np.sum(W * dP) == pytest.approx(
            np.sum(A * oracle.dstress(model, mu, lam, G, W)), rel=1e-12)
        Q = oracle.d2stress(model, mu, lam, G, A, W)
        fd = (oracle.dstress(model, mu, lam, G + eps * W, A)
              - oracle.dstress(model, mu, lam, G - eps * W, A)) / (2 * eps)
        assert np.max(np.abs(fd - Q)) <= 1e-6 * np.max(np.abs(Q))
        assert np.allclose(Q, oracle.d2stress(model, mu, lam, G, W, A), rtol=1e-12,
                           atol=1e-12 * np.max(np.abs(Q)))


@pytest.mark.parametrize("model", MODELS)
def test_rest_tangent_is_hooke(model):
    """At F = I both models reduce to isotropic linear elasticity."""
    mu, lam = oracle.lame(2.5e5, 0.35)
    rng = _rng(3)
    for _ in range(3):
        A = rng.standard_normal((3, 3))
        hooke = mu * (A + A.T) + lam * np.trace(A) * np.eye(3)
        assert np.allclose(oracle.dstress(model, mu, lam, np.zeros((3, 3)), A), hooke,
                           rtol=1e-13, atol=1e-9)


def test_nh_inverted_element():
    mu, lam = oracle.lame(1e5, 0.3)
    with pytest.raises(oracle.OracleError) as e:
        oracle.stress(oracle.NH, mu, lam, np.diag([-1.5, 0, 0]))
    assert e.value.code == oracle.E_INVERTED


# --------------------------------------------------------------------------
# assembled forces and stiffness
# --------------------------------------------------------------------------

def _meshes():
    yield "tet", mg.single_tet(np.array([[0.1, 0.0, 0.2], [1.1, 0.1, 0.0],
                                         [0.0, 0.9, 0.1], [0.2, 0.1, 1.2]]))
    yield "cube1", mg.jitter(mg.kuhn_cube(1), 0.05, seed=7)
    yield "cube2", mg.jitter(mg.kuhn_cube(2), 0.05, seed=8)


def _fem(model, m, E=1e5, nu=0.3):
    return oracle.FEM.create(model, m.X, m.tets, E, nu, pinned=m.pinned)


@pytest.mark.parametrize("model", MODELS)
def test_force_zero_at_rest(model):
    m = mg.jitter(mg.kuhn_cube(3), 0.01, seed=0)
    f = _fem(model, m).forces(np.zeros((m.nv, 3)))
    assert np.all(f == 0.0)


@pytest.mark.parametrize("model", MODELS)
def test_rigid_motion_invariance(model):
    m = mg.jitter(mg.kuhn_cube(3), 0.01, seed=0)
    fem = _fem(model, m)
    R = mg.rotation(20)
    d = m.X @ R.T - m.X + np.array([0.3, -0.2, 0.5])
    f = fem.forces(d)
    mu = fem.mu[0]
    assert np.max(np.abs(f)) <= 1e-10 * mu * m.h ** 2
    # translation is in the kernel of K; so is an infinitesimal rotation at rest
    u = np.tile([0.7, -1.1, 0.4], (m.nv, 1))
    dr = mg.perturbed_state(m, 0.02, seed=10)
    assert np.max(np.abs(fem.kmul(dr, u))) <= 1e-12 * np.max(np.abs(fem.kmul(dr, dr / m.h)))
    w = np.array([0.3, -0.5, 0.8])
    assert np.max(np.abs(fem.kmul(np.zeros_like(u), np.cross(w, m.X)))) <= 1e-9 * mu * m.h


@pytest.mark.parametrize("model", MODELS)
def test_force_sum_zero(model):
    m = mg.jitter(mg.kuhn_cube(3), 0.01, seed=0)
    fem = _fem(model, m)
    d = mg.perturbed_state(m, 0.05, seed=10)
    f = fem.forces(d)
    assert np.max(np.abs(f.sum(axis=0))) <= 1e-12 * np.abs(f).sum()
    y = fem.kmul(d, mg.direction(m, 11))
    assert np.max(np.abs(y.sum(axis=0))) <= 1e-12 * np.abs(y).sum()


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("name,m", list(_meshes()))
def test_force_is_minus_energy_gradient(model, name, m):
    fem = _fem(model, m)
    rng = _rng(4)
    d = 0.03 * rng.standard_normal((m.nv, 3)) * max(m.h, 0.5)
    f = fem.forces(d)
    eps = 1e-6 * max(m.h, 0.5)
    fd = np.zeros_like(d)
    for i in range(m.nv):
        for k in range(3):
            e = np.zeros_like(d)
            e[i, k] = eps
            fd[i, k] = -(fem.energy(d + e) - fem.energy(d - e)) / (2 * eps)
    assert np.max(np.abs(fd - f)) <= 1e-7 * np.max(np.abs(f))


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("name,m", list(_meshes()))
def test_kmul_is_force_derivative_and_symmetric(model, name, m):
    fem = _fem(model, m)
    rng = _rng(5)
    d = 0.03 * rng.standard_normal((m.nv, 3)) * max(m.h, 0.5)
    u = rng.standard_normal((m.nv, 3))
    w = rng.standard_normal((m.nv, 3))
    eps = 1e-6
    Ku = fem.kmul(d, u)
    fd = (fem.forces(d + eps * u) - fem.forces(d - eps * u)) / (2 * eps)
    assert np.max(np.abs(fd - Ku)) <= 1e-7 * np.max(np.abs(Ku))
    Kw = fem.kmul(d, w)
    assert np.sum(w * Ku) == pytest.approx(np.sum(u * Kw), rel=1e-12)


def _voigt_stiffness(m, E, nu):
    """Textbook linear-elastic stiffness V0 Bv^T D Bv, assembled densely."""
    mu = E / (2 * (1 + nu))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[:3, :3] += 2 * mu * np.eye(3)
    D[3:, 3:] = mu * np.eye(3)
    K = np.zeros((3 * m.nv, 3 * m.nv))
    for t in range(m.nt):
        P = m.X[m.tets[t]]
        # shape-function gradients from the linear system X(xi) = X0 + Dm xi
        M = np.hstack([np.ones((4, 1)), P])       # N_a(X) = c_a + g_a . X
        coef = np.linalg.inv(M)                   # column a: (c_a, g_a)
        grads = coef[1:, :].T                     # (4, 3)
        vol = abs(np.linalg.det(M)) / 6
        Bv = np.zeros((6, 12))
        for a in range(4):
            bx, by, bz = grads[a]
            Bv[:, 3 * a:3 * a + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz],
                                      [0, bz, by], [bz, 0, bx], [by, bx, 0]]
        Ke = vol * Bv.T @ D @ Bv
        idx = np.concatenate([[3 * v, 3 * v + 1, 3 * v + 2] for v in m.tets[t]])
        K[np.ix_(idx, idx)] += Ke
    return K


def _dense_K(fem, d):
    n = 3 * fem.nv
    K = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = fem.kmul(d, e.reshape(-1, 3)).ravel()
    return K


@pytest.mark.parametrize("model", MODELS)
def test_rest_stiffness_is_linear_elasticity(model):
    m = mg.jitter(mg.kuhn_cube(2), 0.05, seed=9)
    fem = _fem(model, m, E=3e5, nu=0.33)
    K = _dense_K(fem, np.zeros((m.nv, 3)))
    Kv = _voigt_stiffness(m, 3e5, 0.33)
    assert np.max(np.abs(K + Kv)) <= 1e-12 * np.max(np.abs(Kv))
    ev = np.linalg.eigvalsh(-0.5 * (K + K.T))
    zero = np.sum(np.abs(ev) <= 1e-9 * np.max(np.abs(ev)))
    assert zero == 6 and np.min(ev) > -1e-9 * np.max(ev)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("s", [0.95, 1.02])
def test_uniaxial_patch(model, s):
    n = 3
    m = mg.kuhn_cube(n)
    fem = _fem(model, m)
    d = np.zeros((m.nv, 3))
    d[:, 0] = (s - 1.0) * m.X[:, 0]
    f = fem.forces(d)
    mu, lam = fem.mu[0], fem.lam[0]
    interior = np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1)
    scale = mu + lam
    assert np.max(np.abs(f[interior])) <= 1e-10 * scale
    face = np.abs(m.X[:, 0] - 1.0) < 1e-12
    if model == oracle.STVK:
        P11 = s * (2 * mu + lam) * (s * s - 1) / 2
        psi = (2 * mu + lam) * (s * s - 1) ** 2 / 8
    else:
        P11 = mu * (s - 1 / s) + lam * np.log(s) / s
        psi = 0.5 * mu * (s * s - 1) - mu * np.log(s) + 0.5 * lam * np.log(s) ** 2
    assert f[face, 0].sum() == pytest.approx(-P11, rel=1e-10)
    assert fem.energy(d) == pytest.approx(psi, rel=1e-10)


@pytest.mark.parametrize("model", MODELS)
def test_unit_tet_forces_closed_form(model):
    """Unit right tet (Dm = I, V0 = 1/6) under F = diag(s,1,1):
    f_a = -P e_a / 6 for a = 1..3 and f_0 = -(f_1 + f_2 + f_3)."""
    s = 1.1
    m = mg.single_tet()
    fem = _fem(model, m)
    d = np.zeros((4, 3))
    d[:, 0] = (s - 1.0) * m.X[:, 0]
    mu, lam = fem.mu[0], fem.lam[0]
    if model == oracle.STVK:
        e = (s * s - 1) / 2
        P = np.diag([s * (2 * mu + lam) * e, lam * e, lam * e])
    else:
        P = np.diag([mu * (s - 1 / s) + lam * np.log(s) / s, lam * np.log(s), lam * np.log(s)])
    ref = np.zeros((4, 3))
    ref[1:] = -P.T / 6
    ref[0] = -ref[1:].sum(axis=0)
    assert np.allclose(fem.forces(d), ref, rtol=1e-13, atol=1e-13 * np.abs(P).max())


@pytest.mark.parametrize("model", MODELS)
def test_tmul_is_derivative_of_wKa(model):
    m = mg.jitter(mg.kuhn_cube(1), 0.05, seed=3)
    fem = _fem(model, m)
    rng = _rng(6)
    d = 0.02 * rng.standard_normal((m.nv, 3))
    a = rng.standard_normal((m.nv, 3))
    w = rng.standard_normal((m.nv, 3))
    T = fem.tmul(d, a, w)
    eps = 1e-6
    fd = np.zeros_like(d)
    for i in range(m.nv):
        for k in range(3):
            e = np.zeros_like(d)
            e[i, k] = eps
            fd[i, k] = (np.sum(w * fem.kmul(d + e, a)) - np.sum(w * fem.kmul(d - e, a))) / (2 * eps)
    assert np.max(np.abs(fd - T)) <= 1e-6 * np.max(np.abs(T))


# --------------------------------------------------------------------------
# Jacobi diagonal, PCG and the implicit step
# --------------------------------------------------------------------------

@pytest.mark.parametrize("model", MODELS)
def test_jacobi_diag_is_dense_diagonal(model):
    m = mg.jitter(mg.kuhn_cube(2), 0.05, seed=4)
    fem = _fem(model, m)
    d = mg.perturbed_state(m, 0.05, seed=10)
    dt = 1e-3
    # diagonal of the dense stiffness from central differences of the force
    eps = 1e-6
    kd = np.zeros(3 * m.nv)
    for j in range(3 * m.nv):
        e = np.zeros(3 * m.nv)
        e[j] = eps
        e = e.reshape(-1, 3)
        kd[j] = ((fem.forces(d + e) - fem.forces(d - e)).ravel()[j]) / (2 * eps)
    ref = np.repeat(fem.mass, 3) - dt * dt * kd
    got = fem.jacobi_diag(d, dt).ravel()
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))


def _dense_solve(fem, d, v, dt, g):
    n = 3 * fem.nv
    K = _dense_K(fem, d)
    A = np.diag(np.repeat(fem.mass, 3)) - dt * dt * K
    b = dt * (fem.forces(d).ravel() + np.repeat(fem.mass, 3) * np.tile(g, fem.nv)
              + dt * K @ v.ravel())
    free = np.repeat(fem.pinned == 0, 3)
    x = np.zeros(n)
    Aff = A[np.ix_(free, free)]
    np.linalg.cholesky(0.5 * (Aff + Aff.T))   # SPD
    x[free] = np.linalg.solve(Aff, b[free])
    return x.reshape(-1, 3)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("precond", [oracle.PRECOND_NONE, oracle.PRECOND_JACOBI])
def test_step_matches_dense_solve(model, precond):
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=5)
    fem = _fem(model, m, E=1e6, nu=0.45)
    d = mg.perturbed_state(m, 0.02, seed=10)
    v = 0.1 * mg.direction(m, 11)
    dt = 1e-3
    g = (0.0, 0.0, -9.81)
    d1, v1, dv, st = fem.implicit_step(d, v, dt, g=g, tol=1e-14, maxit=1000, precond=precond)
    assert st.status == oracle.OK
    ref = _dense_solve(fem, d, v, dt, np.array(g))
    assert np.max(np.abs(dv - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.allclose(v1, v + dv, rtol=0, atol=0)
    assert np.allclose(d1, d + dt * v1, rtol=0, atol=1e-18)
    assert np.all(dv[m.pinned == 1] == 0.0)


@pytest.mark.parametrize("model", MODELS)
def test_free_fall_and_momentum(model):
    m = mg.jitter(mg.kuhn_cube(3), 0.01, seed=0)
    fem = oracle.FEM.create(model, m.X, m.tets, 1e5, 0.3)   # nothing pinned
    dt = 1e-3
    g = np.array([0.0, 0.0, -9.81])
    z = np.zeros((m.nv, 3))
    _d, _v, dv, st = fem.implicit_step(z, z, dt, g=g, tol=1e-15, maxit=500)
    assert np.max(np.abs(dv - dt * g)) <= 1e-12 * dt * 9.81
    # momentum: sum m dv = dt M g from any state, once converged
    d = mg.perturbed_state(m, 0.05, seed=10)
    v = mg.direction(m, 11)
    _d, _v, dv, st = fem.implicit_step(d, v, dt, g=g, tol=1e-14, maxit=2000)
    mom = (fem.mass[:, None] * dv).sum(axis=0)
    assert np.max(np.abs(mom - dt * fem.mass.sum() * g)) <= 1e-10 * dt * fem.mass.sum() * 9.81


def test_pcg_breakdown_and_maxit():
    m = mg.kuhn_cube(2)
    fem = oracle.FEM.create(oracle.STVK, m.X, m.tets, -1e9, 0.3, pinned=m.pinned)  # E < 0
    z = np.zeros((m.nv, 3))
    with pytest.raises(oracle.OracleError) as e:
        fem.implicit_step(z, z, 1e-2, tol=0.0, maxit=50, precond=oracle.PRECOND_NONE)
    assert e.value.code == oracle.E_NOT_SPD
    fem = oracle.FEM.create(oracle.STVK, m.X, m.tets, 1e7, 0.3, pinned=m.pinned)
    _d, _v, _dv, st = fem.implicit_step(z, z, 1e-2, tol=1e-30, maxit=2)
    assert st.status == oracle.E_NOT_CONVERGED and st.iters == 2


# --------------------------------------------------------------------------
# assembled stiffness on edges (Vega keeps K on the mesh edges)
# --------------------------------------------------------------------------

def test_edges_brute_force():
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(3), 0.02, seed=2), seed=5)
    row_ptr, col = oracle.edges(m.nv, m.tets)
    want = sorted({(int(i), int(j)) for t in m.tets for i in t for j in t})
    got = [(i, int(col[e])) for i in range(m.nv) for e in range(row_ptr[i], row_ptr[i + 1])]
    assert got == want
    # Kuhn lattice: an interior vertex has 14 neighbours plus itself
    k = mg.kuhn_cube(3)
    rp, _ = oracle.edges(k.nv, k.tets)
    deg = np.diff(rp)
    interior = np.all((k.X > 0.01) & (k.X < 0.99), axis=1)
    assert np.all(deg[interior] == 15)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("name,m", list(_meshes()))
def test_assembled_spmv_is_matrix_free_kmul(model, name, m):
    fem = _fem(model, m)
    rp, col = oracle.edges(m.nv, m.tets)
    rng = _rng(31)
    for d in (np.zeros((m.nv, 3)), mg.perturbed_state(m, 0.05, seed=10)):
        blocks = fem.assemble(d, rp, col)
        for _ in range(3):
            u = rng.standard_normal((m.nv, 3))
            y = oracle.spmv(rp, col, blocks, u)
            ref = fem.kmul(d, u)
            assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("model", MODELS)
def test_assembled_blocks_symmetric_and_translation_free(model):
    m = mg.jitter(mg.kuhn_cube(2), 0.05, seed=8)
    fem = _fem(model, m)
    rp, col = oracle.edges(m.nv, m.tets)
    blocks = fem.assemble(mg.perturbed_state(m, 0.05, seed=10), rp, col)
    scale = np.abs(blocks).max()
    for i in range(m.nv):
        row = blocks[rp[i]:rp[i + 1]]
        assert np.abs(row.sum(axis=0)).max() <= 1e-12 * scale   # K annihilates translations
        for e in range(rp[i], rp[i + 1]):
            j = col[e]
            et = rp[j] + int(np.searchsorted(col[rp[j]:rp[j + 1]], i))
            assert col[et] == i
            assert np.abs(blocks[e] - blocks[et].T).max() <= 1e-12 * scale


@pytest.mark.parametrize("model", MODELS)
def test_assembled_rest_blocks_are_linear_elasticity(model):
    # independent textbook route: Voigt assembly of linear elasticity, read block by block
    m = mg.jitter(mg.kuhn_cube(2), 0.05, seed=9)
    fem = _fem(model, m, E=3e5, nu=0.33)
    rp, col = oracle.edges(m.nv, m.tets)
    blocks = fem.assemble(np.zeros((m.nv, 3)), rp, col)
    Kv = _voigt_stiffness(m, 3e5, 0.33)
    for i in range(m.nv):
        for e in range(rp[i], rp[i + 1]):
            j = col[e]
            want = -Kv[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            assert np.abs(blocks[e] - want).max() <= 1e-12 * np.abs(Kv).max()


# --------------------------------------------------------------------------
# spring-mass workload (the paper's introductory example)
# --------------------------------------------------------------------------

def _two_masses(K=3.0, m=(2.0, 0.5)):
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    return oracle.Springs(X, [0, 1], [1, 0], np.array(m), K)


def test_spring_two_masses_closed_form():
    sp = _two_masses()
    assert np.allclose(sp.rest[:2], [1.0, 1.0], rtol=0, atol=0)
    q = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]])       # stretched by 0.5
    f = sp.forces(q)
    assert np.allclose(f, [[1.5, 0, 0], [-1.5, 0, 0]], rtol=0, atol=1e-15)   # K * 0.5, restoring
    q = np.array([[0.0, 0.0, 0.0], [0.0, 0.8, 0.0]])       # compressed along y
    f = sp.forces(q)
    assert np.allclose(f, [[0, -0.6, 0], [0, 0.6, 0]], rtol=0, atol=1e-15)
    qd = np.array([[0.1, 0.0, 0.0], [0.0, 0.0, -0.2]])
    dt = 0.01
    q1, qd1 = sp.step(q, qd, dt)
    a = f / sp.mass[:, None]
    assert np.allclose(q1, q + qd * dt + 0.5 * a * dt * dt, rtol=0, atol=1e-16)
    assert np.allclose(qd1, qd + a * dt, rtol=0, atol=1e-16)


def test_spring_harmonic_oscillation():
    # two masses on one spring: the separation oscillates about the rest length with
    # omega^2 = K (1/m0 + 1/m1); the explicit update follows it to O(dt) over a period
    K, m = 3.0, (2.0, 0.5)
    sp = _two_masses(K, m)
    w = np.sqrt(K * (1 / m[0] + 1 / m[1]))
    A, dt = 0.01, 1e-4
    q = np.array([[0.0, 0.0, 0.0], [1.0 + A, 0.0, 0.0]])
    qd = np.zeros((2, 3))
    steps = int(round(2 * np.pi / w / dt))
    sep = []
    for _ in range(steps):
        q, qd = sp.step(q, qd, dt)
        sep.append(q[1, 0] - q[0, 0] - 1.0)
    t = dt * np.arange(1, steps + 1)
    assert np.max(np.abs(np.array(sep) - A * np.cos(w * t))) <= 0.02 * A
    # momentum is conserved exactly up to rounding (equal and opposite forces)
    p = (sp.mass[:, None] * qd).sum(axis=0)
    assert np.max(np.abs(p)) <= 1e-15


def test_spring_forces_sum_zero_gradient_and_rest():
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(3), 0.05, seed=4), seed=6)
    tail, head = mg.directed_edges(m.tets, m.nv)
    # the edge set is symmetric and free of self-pairs
    pairs = set(zip(tail.tolist(), head.tolist()))
    assert all((b, a) in pairs and a != b for a, b in pairs)
    sp = oracle.Springs(m.X, tail, head, np.ones(m.nv), 2.5)
    f0 = sp.forces(m.X)
    assert np.abs(f0).max() <= 1e-14
    rng = _rng(41)
    q = m.X + 0.05 * rng.standard_normal((m.nv, 3))
    f = sp.forces(q)
    assert np.abs(f.sum(axis=0)).max() <= 1e-13 * np.abs(f).max()

    def V(qq):   # each undirected spring twice, so a quarter K per directed edge
        dq = qq[head] - qq[tail]
        return 0.25 * 2.5 * np.sum((np.linalg.norm(dq, axis=1) - sp.rest[: len(tail)]) ** 2)

    eps = 1e-6
    for _ in range(3):
        a = rng.standard_normal((m.nv, 3))
        fd = (V(q + eps * a) - V(q - eps * a)) / (2 * eps)
        assert np.sum(f * a) == pytest.approx(-fd, rel=1e-7)


def test_spring_free_flight_and_energy():
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=2)
    tail, head = mg.directed_edges(m.tets, m.nv)
    rng = _rng(42)
    mass = rng.uniform(0.5, 1.5, m.nv)
    sp = oracle.Springs(m.X, tail, head, mass, 0.0)      # K = 0: free flight
    q = m.X + 0.1 * rng.standard_normal((m.nv, 3))
    qd = rng.standard_normal((m.nv, 3))
    q1, qd1 = sp.step(q, qd, 0.01)
    assert np.array_equal(qd1, qd)
    assert np.max(np.abs(q1 - (q + 0.01 * qd))) <= 1e-16
    assert sp.kinetic_energy(qd) == pytest.approx(0.5 * np.sum(mass[:, None] * qd * qd), rel=1e-14)


def test_kinetic_energy_worked_values():
    # hand-computed: 1/2 * 2 * (1 + 4 + 4) + 1/2 * 0.5 * 16 = 9 + 4; a vertex at rest adds nothing
    sp = oracle.Springs(np.zeros((3, 3)), [0], [1], np.array([2.0, 0.5, 7.0]), 1.0)
    assert sp.kinetic_energy(np.array([[1.0, 2.0, -2.0], [0.0, 0.0, 4.0], [0.0, 0.0, 0.0]])) == 13.0
    assert sp.kinetic_energy(np.zeros((3, 3))) == 0.0


def test_kinetic_energy_conserved_by_the_two_mass_oscillator():
    # Unequal masses on one spring along a direction with three nonzero components, plus a
    # common drift.  The exact motion conserves KE + K (|q1 - q0| - L)^2 / 2 = K A^2 / 2 plus
    # the drift energy M |V|^2 / 2; the relative part of KE vanishes at the turning points and
    # equals K A^2 / 2 where the separation crosses L.  The explicit update follows this to
    # O(dt) over a period, which a dropped factor, component or mass in the energy sum fails.
    K, m, A, dt = 3.0, (2.0, 0.5), 0.01, 1e-4
    n = np.array([1.0, 2.0, 2.0]) / 3.0
    X = np.array([[0.0, 0.0, 0.0], n])
    sp = oracle.Springs(X, [0, 1], [1, 0], np.array(m), K)
    V = np.array([0.004, -0.006, 0.003])
    q = np.array([[0.0, 0.0, 0.0], (1.0 + A) * n])
    qd = np.tile(V, (2, 1))
    drift = 0.5 * (m[0] + m[1]) * V.dot(V)
    E0 = 0.5 * K * A * A + drift
    w = np.sqrt(K * (1 / m[0] + 1 / m[1]))
    steps = int(round(2 * np.pi / w / dt))
    rel_ke = []
    for _ in range(steps):
        q, qd = sp.step(q, qd, dt)
        ext = np.linalg.norm(q[1] - q[0]) - 1.0
        E = sp.kinetic_energy(qd) + 0.5 * K * ext * ext
        assert abs(E - E0) <= 2e-3 * E0
        rel_ke.append(sp.kinetic_energy(qd) - drift)
    rel_ke = np.array(rel_ke)
    assert rel_ke.max() == pytest.approx(0.5 * K * A * A, rel=2e-3)
    assert rel_ke.min() >= -1e-3 * 0.5 * K * A * A
    # quarter period: crossing the rest length (maximum); half period: turning point (zero)
    assert rel_ke[steps // 4] == pytest.approx(0.5 * K * A * A, rel=1e-2)
    assert abs(rel_ke[steps // 2]) <= 1e-2 * 0.5 * K * A * A


# --------------------------------------------------------------------------
# Rayleigh damping (Vega's step computes damping with forces and stiffness:
# Performance Evaluation); D = alpha M - beta K with K = df/dx
# --------------------------------------------------------------------------

@pytest.mark.parametrize("model", MODELS)
def test_damped_rigid_translation(model):
    # nothing pinned, at rest, uniform velocity: f = 0 and K annihilates translations,
    # so every vertex follows the backward-Euler update of dv/dt = g - alpha v exactly
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=1)
    fem = oracle.FEM.create(model, m.X, m.tets, 1e5, 0.3)
    dt, alpha, beta = 1e-2, 4.0, 3e-3
    g = np.array([0.5, -1.0, -9.81])
    v0 = np.array([0.3, -0.2, 0.7])
    v = np.tile(v0, (m.nv, 1))
    d1, v1, _dv, st = fem.implicit_step(np.zeros((m.nv, 3)), v, dt, g=g, tol=1e-15, maxit=500,
                                        alpha=alpha, beta=beta)
    want = (v0 + dt * g) / (1.0 + dt * alpha)
    assert st.status == oracle.OK
    assert np.max(np.abs(v1 - want)) <= 1e-12 * np.abs(want).max()
    assert np.max(np.abs(d1 - dt * v1)) <= 1e-18


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("at_rest", [True, False])
def test_damped_step_is_modal_damped_oscillator(model, at_rest):
    # In the M-orthonormal eigenbasis of the free block (-K phi = lam M phi) each mode is a
    # damped oscillator with Rayleigh coefficient alpha + beta lam; one linearised backward-Euler
    # step gives c' = (c + dt f_i) / (1 + dt (alpha + beta lam) + dt^2 lam), f_i = phi_i . (f + M g)
    import scipy.linalg
    m = mg.jitter(mg.kuhn_cube(2), 0.03, seed=12)
    fem = _fem(model, m, E=2e5, nu=0.35)
    rng = _rng(21)
    d = np.zeros((m.nv, 3)) if at_rest else mg.perturbed_state(m, 0.01, seed=13)
    v = 0.2 * rng.standard_normal((m.nv, 3))
    v[m.pinned == 1] = 0.0
    dt, alpha, beta = 1e-2, 2.5, 4e-3
    g = np.array([0.0, 0.3, -9.81])
    free = np.repeat(m.pinned == 0, 3)
    K = _dense_K(fem, d)
    Kff = K[np.ix_(free, free)]
    Mff = np.repeat(fem.mass, 3)[free]
    lam, Phi = scipy.linalg.eigh(-0.5 * (Kff + Kff.T), np.diag(Mff))
    assert lam.min() > 0.0
    f = (fem.forces(d) + fem.mass[:, None] * g).ravel()[free]
    c = Phi.T @ (Mff * v.ravel()[free])     # modal velocities
    fi = Phi.T @ f                           # modal forces
    c1 = (c + dt * fi) / (1.0 + dt * (alpha + beta * lam) + dt * dt * lam)
    want = (Phi @ c1).reshape(-1, 3)
    _d1, v1, _dv, st = fem.implicit_step(d, v, dt, g=g, tol=1e-15, maxit=2000, alpha=alpha, beta=beta)
    got = v1.ravel()[free].reshape(-1, 3)
    assert st.status == oracle.OK
    assert np.max(np.abs(got - want)) <= 1e-10 * np.abs(want).max()
    # the undamped step is the alpha = beta = 0 case of the same modal formula
    c0 = (c + dt * fi) / (1.0 + dt * dt * lam)
    _d1, v0, _dv, _ = fem.implicit_step(d, v, dt, g=g, tol=1e-15, maxit=2000)
    assert np.max(np.abs(v0.ravel()[free] - Phi @ c0)) <= 1e-10 * np.abs(Phi @ c0).max()


@pytest.mark.parametrize("model", MODELS)
def test_damped_step_vjp_fd(model):
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=6)
    rng = _rng(17)
    E = 1e5 * np.exp(0.3 * rng.standard_normal(m.nt))
    fem = oracle.FEM.create(model, m.X, m.tets, E, 0.3, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    v = 0.05 * mg.direction(m, 11)
    dt, tol, alpha, beta = 1e-3, 1e-14, 3.0, 2e-3
    gx = rng.standard_normal((m.nv, 3))
    gv = rng.standard_normal((m.nv, 3))

    def J(dd, vv, EE):
        f2 = oracle.FEM.create(model, m.X, m.tets, EE, 0.3, pinned=m.pinned)
        d1, v1, _dv, _ = f2.implicit_step(dd, vv, dt, tol=tol, maxit=5000, alpha=alpha, beta=beta)
        return np.sum(gx * d1) + np.sum(gv * v1), v1

    _L0, v1 = J(d, v, E)
    d_bar, v_bar, E_bar, _st = fem.step_vjp(d, v1, gx, gv, dt, tol=tol, maxit=5000, alpha=alpha, beta=beta)
    eps = 1e-6
    a = rng.standard_normal((m.nv, 3))
    fd = (J(d + eps * a, v, E)[0] - J(d - eps * a, v, E)[0]) / (2 * eps)
    assert np.sum(d_bar * a) == pytest.approx(fd, rel=1e-6)
    fd = (J(d, v + eps * a, E)[0] - J(d, v - eps * a, E)[0]) / (2 * eps)
    assert np.sum(v_bar * a) == pytest.approx(fd, rel=1e-6)
    for t in [0, 7, 31]:
        dE = np.zeros(m.nt)
        dE[t] = 1e-6 * E[t]
        fd = (J(d, v, E + dE)[0] - J(d, v, E - dE)[0]) / (2 * dE[t])
        assert E_bar[t] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(E_bar).max())


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def test_force_linear_in_E():
    m = mg.jitter(mg.kuhn_cube(1), 0.05, seed=3)
    d = mg.perturbed_state(m, 0.05, seed=10)
    E = np.linspace(1e5, 3e5, m.nt)
    for model in MODELS:
        f1 = oracle.FEM.create(model, m.X, m.tets, E, 0.3).forces(d)
        f2 = oracle.FEM.create(model, m.X, m.tets, 2 * E, 0.3).forces(d)
        assert np.max(np.abs(f2 - 2 * f1)) <= 1e-14 * np.max(np.abs(f2))


@pytest.mark.parametrize("model", MODELS)
def test_step_vjp_dot_product_and_fd(model):
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=6)
    rng = _rng(7)
    E = 1e5 * np.exp(0.3 * rng.standard_normal(m.nt))
    fem = oracle.FEM.create(model, m.X, m.tets, E, 0.3, pinned=m.pinned)
    d = mg.perturbed_state(m, 0.02, seed=10)
    v = 0.05 * mg.direction(m, 11)
    dt, tol = 1e-3, 1e-14
    gx = rng.standard_normal((m.nv, 3))
    gv = rng.standard_normal((m.nv, 3))

    def J(dd, vv, EE):
        f2 = oracle.FEM.create(model, m.X, m.tets, EE, 0.3, pinned=m.pinned)
        d1, v1, _dv, _ = f2.implicit_step(dd, vv, dt, tol=tol, maxit=5000)
        return np.sum(gx * d1) + np.sum(gv * v1), v1

    L0, v1 = J(d, v, E)
    d_bar, v_bar, E_bar, st = fem.step_vjp(d, v1, gx, gv, dt, tol=tol, maxit=5000)
    eps = 1e-6
    a = rng.standard_normal((m.nv, 3))
    fd = (J(d + eps * a, v, E)[0] - J(d - eps * a, v, E)[0]) / (2 * eps)
    assert np.sum(d_bar * a) == pytest.approx(fd, rel=1e-6)
    fd = (J(d, v + eps * a, E)[0] - J(d, v - eps * a, E)[0]) / (2 * eps)
    assert np.sum(v_bar * a) == pytest.approx(fd, rel=1e-6)
    for t in [0, 7, 31]:
        dE = np.zeros(m.nt)
        dE[t] = 1e-6 * E[t]
        fd = (J(d, v, E + dE)[0] - J(d, v, E - dE)[0]) / (2 * dE[t])
        assert E_bar[t] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(E_bar).max())


def test_trajectory_gradient_fd_and_checkpoints():
    m = mg.jitter(mg.kuhn_cube(2), 0.02, seed=6)
    rng = _rng(8)
    E = 1e5 * np.exp(0.5 * rng.standard_normal(m.nt))
    fem = oracle.FEM.create(oracle.NH, m.X, m.tets, E, 0.3, pinned=m.pinned)
    target = m.X + 1e-3 * rng.standard_normal((m.nv, 3))
    z = np.zeros((m.nv, 3))
    kw = dict(steps=3, dt=1e-2, tol=1e-14, maxit=5000, target=target, X=m.X)
    L, gd0, gE = oracle.trajectory_grad(fem, z, z, **kw)
    L2, gd0b, gEb = oracle.trajectory_grad(fem, z, z, checkpoint_every=2, **kw)
    assert L == L2
    assert np.max(np.abs(gd0 - gd0b)) <= 1e-12 * np.max(np.abs(gd0))
    assert np.max(np.abs(gE - gEb)) <= 1e-12 * np.max(np.abs(gE))

    def loss(d0, EE):
        f2 = oracle.FEM.create(oracle.NH, m.X, m.tets, EE, 0.3, pinned=m.pinned)
        st = oracle.trajectory(f2, d0, z, 3, 1e-2, 1e-14, 5000)
        return float(np.sum((m.X + st[-1][0] - target) ** 2))

    a = rng.standard_normal((m.nv, 3))
    eps = 1e-6
    fd = (loss(eps * a, E) - loss(-eps * a, E)) / (2 * eps)
    assert np.sum(gd0 * a) == pytest.approx(fd, rel=1e-6)
    for t in [3, 20]:
        dE = np.zeros(m.nt)
        dE[t] = 1e-4 * E[t]
        fd = (loss(z, E + dE) - loss(z, E - dE)) / (2 * dE[t])
        assert gE[t] == pytest.approx(fd, rel=1e-6)


# --------------------------------------------------------------------------
# grouping and Morton order
# --------------------------------------------------------------------------

def test_group_by_brute_force():
    s, _pv, _pt = mg.scramble(mg.kuhn_cube(3), seed=1)
    row_ptr, inc = oracle.group_by(s.nv, s.tets)
    assert row_ptr[0] == 0 and row_ptr[-1] == 4 * s.nt
    assert np.array_equal(np.sort(inc), np.arange(4 * s.nt))
    for v in range(s.nv):
        seg = inc[row_ptr[v]:row_ptr[v + 1]]
        assert np.all(np.diff(seg) > 0)
        assert np.all(s.tets.ravel()[seg] == v)
        assert len(seg) == np.sum(s.tets == v)


def _naive_morton(X):
    lo, hi = X.min(axis=0), X.max(axis=0)
    codes = []
    for x in X:
        q = []
        for a in range(3):
            if hi[a] > lo[a]:
                sc = 2.0 ** 21 / (hi[a] - lo[a])
                q.append(min(2 ** 21 - 1, int(np.floor((x[a] - lo[a]) * sc))))
            else:
                q.append(0)
        c = 0
        for b in range(21):
            for a in range(3):
                c |= ((q[a] >> b) & 1) << (3 * b + a)
        codes.append(c)
    return np.array(codes, dtype=np.uint64)


def test_morton_brute_force():
    s, _pv, _pt = mg.scramble(mg.jitter(mg.kuhn_cube(3), 0.01, seed=0), seed=1)
    codes, vperm, tperm = oracle.morton(s.X, s.tets)
    assert np.array_equal(codes, _naive_morton(s.X))
    assert np.array_equal(np.sort(vperm), np.arange(s.nv))
    assert np.array_equal(np.sort(tperm), np.arange(s.nt))
    order = sorted(range(s.nv), key=lambda v: (int(codes[v]), v))
    assert np.array_equal(vperm, order)
    inv = np.empty(s.nv, dtype=np.int64)
    inv[vperm] = np.arange(s.nv)
    key = inv[s.tets].min(axis=1)
    order = sorted(range(s.nt), key=lambda t: (key[t], t))
    assert np.array_equal(tperm, order)
    # degenerate extent (flat in z): all z bits are zero
    Xf = s.X.copy()
    Xf[:, 2] = 0.25
    c2, _, _ = oracle.morton(Xf, s.tets)
    mask = sum(1 << (3 * b + 2) for b in range(21))
    assert np.all((c2.astype(object) & mask) == 0)


def test_morton_segmented_brute_force():
    """Morton order within segments: three jittered unit cubes of different resolutions in one
    union, labelled by cube.  The vertices must come in order of (label, code, id), with
    the codes from the union's one bounding box; the tets follow by their smallest new vertex, so
    each cube's tets stay together; with one label the order is the plain one."""
    cubes = [mg.jitter(mg.kuhn_cube(n), 0.01, seed=20 + i) for i, n in enumerate((2, 3, 2))]
    un = mg.union(cubes)
    # the cubes overlap in space, so only the labels keep their vertices apart
    seg = np.asarray(un.vert_mesh, dtype=np.int32)
    codes, vperm, tperm = oracle.morton(un.X, un.tets, seg=seg)
    assert np.array_equal(codes, _naive_morton(un.X))
    order = sorted(range(un.nv), key=lambda v: (int(seg[v]), int(codes[v]), v))
    assert np.array_equal(vperm, order)
    inv = np.empty(un.nv, dtype=np.int64)
    inv[vperm] = np.arange(un.nv)
    key = inv[un.tets].min(axis=1)
    assert np.array_equal(tperm, sorted(range(un.nt), key=lambda t: (key[t], t)))
    # each cube's vertices and tets stay contiguous and in cube order
    assert np.all(np.diff(seg[vperm]) >= 0)
    tseg = np.asarray(un.tet_mesh)[tperm]
    assert np.all(np.diff(tseg) >= 0)
    # a single label gives the plain Morton order
    c1, v1, t1 = oracle.morton(un.X, un.tets, seg=np.zeros(un.nv, dtype=np.int32))
    c0, v0, t0 = oracle.morton(un.X, un.tets)
    assert np.array_equal(v1, v0) and np.array_equal(t1, t0) and np.array_equal(c1, c0)


# --------------------------------------------------------------------------
# multi-threaded timing entries of the oracle
# --------------------------------------------------------------------------

@pytest.mark.parametrize("model", MODELS)
def test_threaded_forces_and_kmul_equal_the_serial_loop(model):
    # per-corner partials summed over the grouping in (tet, corner) order give every vertex the
    # serial loop's terms in its order: equal bit for bit, for any thread count
    m, _, _ = mg.scramble(mg.jitter(mg.kuhn_cube(6), 0.02, seed=3), seed=5)
    fem = oracle.FEM.create(model, m.X, m.tets, 1e5, 0.3)
    rng = _rng(77)
    d = 0.01 * rng.standard_normal((m.nv, 3)) / 6
    u = rng.standard_normal((m.nv, 3))
    f, y = fem.forces(d), fem.kmul(d, u)
    for threads in (1, 3, 8):
        assert np.array_equal(fem.forces_mt(d, threads), f)
        assert np.array_equal(fem.kmul_mt(d, u, threads), y)
