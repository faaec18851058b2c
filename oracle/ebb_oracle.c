/* ebb_oracle.c -- plain FP64 CPU reference for the tet-FEM element map.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares
 * no code with the GPU library.
 *
 * What it follows.  The paper (Developing Domain Libraries, "Example: FEM
 * tetmesh"; Performance Evaluation, Vega and FreeFem++) names the pieces but
 * prints none of their formulas: a tet mesh with displacement, velocity and
 * force on vertices and material on tets; St. Venant-Kirchhoff (Vega) and
 * neo-Hookean (FreeFem++) hyperelasticity; implicit backward Euler; a
 * Jacobi-preconditioned conjugate-gradient solve.  The formulas below are
 * the textbook definitions of those named methods on linear tetrahedra,
 * written out plainly:
 *   F = I + G, G = dD * B, dD = [d1-d0 | d2-d0 | d3-d0], B = Dm^-1;
 *   StVK: E = (F^T F - I)/2, S = 2 mu E + lam tr(E) I, P = F S;
 *   NH:   P = mu (F - F^-T) + lam ln(J) F^-T, J = det F;
 *   element forces H = -V0 P B^T (columns -> corners 1..3, corner 0 gets
 *   minus their sum), reduced (+=) into the vertices;
 *   K = df/dx applied matrix-free through dP = dP/dF : dF.
 * Reductions into vertex fields are serial, in tet-row order, as in the
 * paper's CPU specialisation (Runtime Implementation).
 */
#include "ebb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- 3x3 helpers (row-major: M[3*i + j] = M_ij) ------------------------- */

static void m_zero(double A[9]) { for (int i = 0; i < 9; ++i) A[i] = 0.0; }
static void m_eye(double A[9]) { m_zero(A); A[0] = A[4] = A[8] = 1.0; }

static void m_mul(const double A[9], const double B[9], double C[9]) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void m_transpose(const double A[9], double T[9]) {
    double R[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[3 * j + i] = A[3 * i + j];
    memcpy(T, R, sizeof R);
}

static double m_trace(const double A[9]) { return A[0] + A[4] + A[8]; }

static double m_ddot(const double A[9], const double B[9]) {
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += A[i] * B[i];
    return s;
}

static double m_det(const double A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse by adjugate / determinant */
static void m_inverse(const double A[9], double det, double R[9]) {
    double C[9];
    C[0] = A[4] * A[8] - A[5] * A[7];
    C[1] = A[2] * A[7] - A[1] * A[8];
    C[2] = A[1] * A[5] - A[2] * A[4];
    C[3] = A[5] * A[6] - A[3] * A[8];
    C[4] = A[0] * A[8] - A[2] * A[6];
    C[5] = A[2] * A[3] - A[0] * A[5];
    C[6] = A[3] * A[7] - A[4] * A[6];
    C[7] = A[1] * A[6] - A[0] * A[7];
    C[8] = A[0] * A[4] - A[1] * A[3];
    for (int i = 0; i < 9; ++i) R[i] = C[i] / det;
}

static void m_axpby(double a, const double A[9], double b, const double B[9], double C[9]) {
    for (int i = 0; i < 9; ++i) C[i] = a * A[i] + b * B[i];
}

static void m_sym(const double A[9], double S[9]) {
    double T[9];
    m_transpose(A, T);
    m_axpby(0.5, A, 0.5, T, S);
}

/* ---- material ------------------------------------------------------------ */

void orc_lame(double E, double nu, double *mu, double *lam) {
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Shared NH pieces: F = I + G, N = F^-T, J, ln J. */
static int nh_parts(const double G[9], double F[9], double N[9], double *lnJ) {
    double Fi[9];
    m_eye(F);
    for (int i = 0; i < 9; ++i) F[i] += G[i];
    double J = m_det(F);
    if (!(J > 0.0)) return ORC_E_INVERTED;
    m_inverse(F, J, Fi);
    m_transpose(Fi, N);
    *lnJ = log(J);
    return ORC_OK;
}

/* StVK second Piola-Kirchhoff stress S(F). */
static void stvk_S(double mu, double lam, const double F[9], double S[9]) {
    double Ft[9], C[9], E[9], I[9];
    m_transpose(F, Ft);
    m_mul(Ft, F, C);
    m_eye(I);
    m_axpby(0.5, C, -0.5, I, E);
    m_axpby(2.0 * mu, E, lam * m_trace(E), I, S);
}

/* dS[X] = 2 mu sym(F^T X) + lam tr(F^T X) I */
static void stvk_dS(double mu, double lam, const double F[9], const double X[9], double dS[9]) {
    double Ft[9], FtX[9], sy[9], I[9];
    m_transpose(F, Ft);
    m_mul(Ft, X, FtX);
    m_sym(FtX, sy);
    m_eye(I);
    m_axpby(2.0 * mu, sy, lam * m_trace(FtX), I, dS);
}

int orc_stress(int model, double mu, double lam, const double G[9], double P[9]) {
    double F[9];
    if (model == ORC_STVK) {
        double S[9];
        m_eye(F);
        for (int i = 0; i < 9; ++i) F[i] += G[i];
        stvk_S(mu, lam, F, S);
        m_mul(F, S, P);
        return ORC_OK;
    }
    if (model == ORC_NH) {
        double N[9], lnJ;
        int st = nh_parts(G, F, N, &lnJ);
        if (st) return st;
        for (int i = 0; i < 9; ++i) P[i] = mu * (F[i] - N[i]) + lam * lnJ * N[i];
        return ORC_OK;
    }
    return ORC_E_ARG;
}

int orc_dstress(int model, double mu, double lam, const double G[9],
                const double dF[9], double dP[9]) {
    double F[9];
    if (model == ORC_STVK) {
        double S[9], dS[9], a[9], b[9];
        m_eye(F);
        for (int i = 0; i < 9; ++i) F[i] += G[i];
        stvk_S(mu, lam, F, S);
        stvk_dS(mu, lam, F, dF, dS);
        m_mul(dF, S, a);   /* dF S  */
        m_mul(F, dS, b);   /* F dS  */
        for (int i = 0; i < 9; ++i) dP[i] = a[i] + b[i];
        return ORC_OK;
    }
    if (model == ORC_NH) {
        /* d(F^-T) = -N dF^T N, d(ln J) = N : dF */
        double N[9], lnJ, dFt[9], t1[9], NdFtN[9];
        int st = nh_parts(G, F, N, &lnJ);
        if (st) return st;
        m_transpose(dF, dFt);
        m_mul(N, dFt, t1);
        m_mul(t1, N, NdFtN);
        double c = mu - lam * lnJ;
        double trc = m_ddot(N, dF);
        for (int i = 0; i < 9; ++i) dP[i] = mu * dF[i] + c * NdFtN[i] + lam * trc * N[i];
        return ORC_OK;
    }
    return ORC_E_ARG;
}

int orc_d2stress(int model, double mu, double lam, const double G[9],
                 const double A[9], const double W[9], double Q[9]) {
    double F[9];
    if (model == ORC_STVK) {
        /* P = F S: d2P[A,W] = A S'[W] + W S'[A] + F S''[A,W],
         * S''[A,W] = 2 mu sym(A^T W) + lam tr(A^T W) I */
        double dSA[9], dSW[9], At[9], AtW[9], sy[9], I[9], S2[9], t1[9], t2[9], t3[9];
        m_eye(F);
        for (int i = 0; i < 9; ++i) F[i] += G[i];
        stvk_dS(mu, lam, F, A, dSA);
        stvk_dS(mu, lam, F, W, dSW);
        m_transpose(A, At);
        m_mul(At, W, AtW);
        m_sym(AtW, sy);
        m_eye(I);
        m_axpby(2.0 * mu, sy, lam * m_trace(AtW), I, S2);
        m_mul(A, dSW, t1);
        m_mul(W, dSA, t2);
        m_mul(F, S2, t3);
        for (int i = 0; i < 9; ++i) Q[i] = t1[i] + t2[i] + t3[i];
        return ORC_OK;
    }
    if (model == ORC_NH) {
        /* differentiate dP[A] = mu A + c N A^T N + lam (N:A) N along W, with
         * dN[W] = -N W^T N, dc[W] = -lam (N:W) */
        double N[9], lnJ, At[9], Wt[9], NAt[9], NAtN[9], NWt[9], NWtN[9];
        double x1[9], x2[9];
        int st = nh_parts(G, F, N, &lnJ);
        if (st) return st;
        double c = mu - lam * lnJ;
        m_transpose(A, At);
        m_transpose(W, Wt);
        m_mul(N, At, NAt);
        m_mul(NAt, N, NAtN);
        m_mul(N, Wt, NWt);
        m_mul(NWt, N, NWtN);
        m_mul(NWtN, At, x1);
        m_mul(x1, N, x1);       /* N W^T N A^T N */
        m_mul(NAtN, Wt, x2);
        m_mul(x2, N, x2);       /* N A^T N W^T N */
        double NA = m_ddot(N, A), NW = m_ddot(N, W), NWtNA = m_ddot(NWtN, A);
        for (int i = 0; i < 9; ++i)
            Q[i] = -lam * NW * NAtN[i] - lam * NA * NWtN[i] - c * (x1[i] + x2[i])
                   - lam * NWtNA * N[i];
        return ORC_OK;
    }
    return ORC_E_ARG;
}

int orc_energy_density(int model, double mu, double lam, const double G[9], double *psi) {
    double F[9], Ft[9], C[9], I[9];
    m_eye(F);
    for (int i = 0; i < 9; ++i) F[i] += G[i];
    m_transpose(F, Ft);
    m_mul(Ft, F, C);
    if (model == ORC_STVK) {
        double E[9];
        m_eye(I);
        m_axpby(0.5, C, -0.5, I, E);
        double trE = m_trace(E);
        *psi = mu * m_ddot(E, E) + 0.5 * lam * trE * trE;
        return ORC_OK;
    }
    if (model == ORC_NH) {
        double J = m_det(F);
        if (!(J > 0.0)) return ORC_E_INVERTED;
        double lnJ = log(J);
        *psi = 0.5 * mu * (m_trace(C) - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
        return ORC_OK;
    }
    return ORC_E_ARG;
}

/* ---- per-tet gather / scatter ------------------------------------------- */

/* dD = [q1-q0 | q2-q0 | q3-q0] (columns), M = dD B */
static void tet_grad(const int32_t *tv, const double *q, const double *B, double M[9]) {
    double dD[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            dD[3 * r + c] = q[3 * (int64_t)tv[c + 1] + r] - q[3 * (int64_t)tv[0] + r];
    m_mul(dD, B, M);
}

/* out[v_c] += columns of -V0 P B^T, corner 0 gets minus their sum */
static void tet_scatter(const int32_t *tv, double V0, const double P[9], const double *B,
                        double *out) {
    double Bt[9], H[9];
    m_transpose(B, Bt);
    m_mul(P, Bt, H);
    for (int i = 0; i < 9; ++i) H[i] *= -V0;
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            out[3 * (int64_t)tv[c + 1] + r] += H[3 * r + c];
            s += H[3 * r + c];
        }
        out[3 * (int64_t)tv[0] + r] -= s;
    }
}

/* ---- public API ------------------------------------------------------------ */

int orc_precompute(int64_t nv, int64_t nt, const double *X, const int32_t *tets,
                   double rho, const double *E, double nu,
                   double *B, double *V0, double *mu, double *lam, double *mass,
                   int64_t *bad_tet) {
    if (mass) memset(mass, 0, sizeof(double) * (size_t)nv);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *tv = tets + 4 * t;
        double Dm[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                Dm[3 * r + c] = X[3 * (int64_t)tv[c + 1] + r] - X[3 * (int64_t)tv[0] + r];
        double det = m_det(Dm);
        if (!(det > 0.0)) {
            if (bad_tet) *bad_tet = t;
            return ORC_E_DEGENERATE;
        }
        m_inverse(Dm, det, B + 9 * t);
        V0[t] = det / 6.0;
        orc_lame(E[t], nu, mu + t, lam + t);
        if (mass)
            for (int c = 0; c < 4; ++c) mass[tv[c]] += rho * V0[t] / 4.0;
    }
    return ORC_OK;
}

int orc_forces(int model, int64_t nv, int64_t nt, const int32_t *tets,
               const double *B, const double *V0, const double *mu, const double *lam,
               const double *d, double *f) {
    memset(f, 0, sizeof(double) * (size_t)(3 * nv));
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], P[9];
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        int st = orc_stress(model, mu[t], lam[t], G, P);
        if (st) return st;
        tet_scatter(tets + 4 * t, V0[t], P, B + 9 * t, f);
    }
    return ORC_OK;
}

int orc_kmul(int model, int64_t nv, int64_t nt, const int32_t *tets,
             const double *B, const double *V0, const double *mu, const double *lam,
             const double *d, const double *u, double *y) {
    memset(y, 0, sizeof(double) * (size_t)(3 * nv));
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], dF[9], dP[9];
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        tet_grad(tets + 4 * t, u, B + 9 * t, dF);
        int st = orc_dstress(model, mu[t], lam[t], G, dF, dP);
        if (st) return st;
        tet_scatter(tets + 4 * t, V0[t], dP, B + 9 * t, y);
    }
    return ORC_OK;
}

/* ---- multi-threaded forms, for timing the CPU baseline ----------------------------------
 *
 * The same element quantities with the tets split over threads: each tet writes its twelve
 * corner values to its own row of part (nt x 12, corner-major), then each vertex sums its rows
 * over the grouping (row_ptr, inc from orc_group_by), whose rows list a vertex's incidences in
 * (tet, corner) order.  A vertex therefore receives the same terms in the same order as in the
 * serial loop above, starting from zero, so the results are equal bit for bit. */

/* the twelve corner values h[3c + r] that tet_scatter adds into out */
static void tet_corners(double V0, const double P[9], const double *B, double h[12]) {
    double Bt[9], H[9];
    m_transpose(B, Bt);
    m_mul(P, Bt, H);
    for (int i = 0; i < 9; ++i) H[i] *= -V0;
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            h[3 * (c + 1) + r] = H[3 * r + c];
            s += H[3 * r + c];
        }
        h[r] = -s;
    }
}

static void gather_corners(int64_t nv, const int64_t *row_ptr, const int32_t *inc, const double *part,
                           double *out, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const double *h = part + 12 * (int64_t)(inc[j] >> 2) + 3 * (inc[j] & 3);
            a0 += h[0];
            a1 += h[1];
            a2 += h[2];
        }
        out[3 * v] = a0;
        out[3 * v + 1] = a1;
        out[3 * v + 2] = a2;
    }
}

int orc_forces_mt(int model, int64_t nv, int64_t nt, const int32_t *tets,
                  const double *B, const double *V0, const double *mu, const double *lam,
                  const double *d, double *f, const int64_t *row_ptr, const int32_t *inc, double *part,
                  int nthreads) {
    int err = ORC_OK;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], P[9];
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        const int st = orc_stress(model, mu[t], lam[t], G, P);
        if (st) {
#pragma omp atomic write
            err = st;
            continue;
        }
        tet_corners(V0[t], P, B + 9 * t, part + 12 * t);
    }
    if (err) return err;
    gather_corners(nv, row_ptr, inc, part, f, nthreads);
    return ORC_OK;
}

int orc_kmul_mt(int model, int64_t nv, int64_t nt, const int32_t *tets,
                const double *B, const double *V0, const double *mu, const double *lam,
                const double *d, const double *u, double *y, const int64_t *row_ptr, const int32_t *inc,
                double *part, int nthreads) {
    int err = ORC_OK;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], dF[9], dP[9];
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        tet_grad(tets + 4 * t, u, B + 9 * t, dF);
        const int st = orc_dstress(model, mu[t], lam[t], G, dF, dP);
        if (st) {
#pragma omp atomic write
            err = st;
            continue;
        }
        tet_corners(V0[t], dP, B + 9 * t, part + 12 * t);
    }
    if (err) return err;
    gather_corners(nv, row_ptr, inc, part, y, nthreads);
    return ORC_OK;
}

int orc_tmul(int model, int64_t nv, int64_t nt, const int32_t *tets,
             const double *B, const double *V0, const double *mu, const double *lam,
             const double *d, const double *a, const double *w, double *out) {
    memset(out, 0, sizeof(double) * (size_t)(3 * nv));
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], FA[9], FW[9], Q[9];
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        tet_grad(tets + 4 * t, a, B + 9 * t, FA);
        tet_grad(tets + 4 * t, w, B + 9 * t, FW);
        int st = orc_d2stress(model, mu[t], lam[t], G, FA, FW, Q);
        if (st) return st;
        /* grad_x (w^T K a) = scatter of -V0 Q B^T; the sign matches f's */
        tet_scatter(tets + 4 * t, V0[t], Q, B + 9 * t, out);
    }
    return ORC_OK;
}

int orc_energy(int model, int64_t nv, int64_t nt, const int32_t *tets,
               const double *B, const double *V0, const double *mu, const double *lam,
               const double *d, double *W) {
    (void)nv;
    double s = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
        double G[9], psi;
        tet_grad(tets + 4 * t, d, B + 9 * t, G);
        int st = orc_energy_density(model, mu[t], lam[t], G, &psi);
        if (st) return st;
        s += V0[t] * psi;
    }
    *W = s;
    return ORC_OK;
}

int orc_jacobi_diag(int model, int64_t nv, int64_t nt, const int32_t *tets,
                    const double *B, const double *V0, const double *mu, const double *lam,
                    const double *mass, double dt, const double *d, double *diag) {
    /* K[(v,c),(v,c)] = sum over incident (t, a) of -V0 dP(e_c b_a^T) : (e_c b_a^T),
     * b_a = row a-1 of B for a = 1..3 and b_0 = -(b_1 + b_2 + b_3). */
    double *kd = calloc((size_t)(3 * nv), sizeof(double));
    if (!kd) return ORC_E_ARG;
    for (int64_t t = 0; t < nt; ++t) {
        const double *Bt = B + 9 * t;
        double G[9];
        tet_grad(tets + 4 * t, d, Bt, G);
        for (int a = 0; a < 4; ++a) {
            double b[3];
            for (int j = 0; j < 3; ++j)
                b[j] = a ? Bt[3 * (a - 1) + j] : -(Bt[j] + Bt[3 + j] + Bt[6 + j]);
            for (int c = 0; c < 3; ++c) {
                double dF[9], dP[9];
                m_zero(dF);
                for (int j = 0; j < 3; ++j) dF[3 * c + j] = b[j];
                int st = orc_dstress(model, mu[t], lam[t], G, dF, dP);
                if (st) { free(kd); return st; }
                kd[3 * (int64_t)tets[4 * t + a] + c] += -V0[t] * m_ddot(dP, dF);
            }
        }
    }
    for (int64_t i = 0; i < 3 * nv; ++i) diag[i] = mass[i / 3] - dt * dt * kd[i];
    free(kd);
    return ORC_OK;
}

/* ---- implicit step ---------------------------------------------------------- */

static double vdot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

typedef struct {
    int model;
    int64_t nv, nt;
    const int32_t *tets;
    const double *B, *V0, *mu, *lam, *mass, *d;
    const uint8_t *pinned;
    double dt;
    double cm, ck;   /* A = cm M - ck K(d) */
} sys_t;

/* q = Pi (cm M p - ck K(d) p) */
static int apply_A(const sys_t *s, const double *p, double *q) {
    int st = orc_kmul(s->model, s->nv, s->nt, s->tets, s->B, s->V0, s->mu, s->lam, s->d, p, q);
    if (st) return st;
    for (int64_t i = 0; i < 3 * s->nv; ++i) {
        q[i] = s->cm * s->mass[i / 3] * p[i] - s->ck * q[i];
        if (s->pinned && s->pinned[i / 3]) q[i] = 0.0;
    }
    return ORC_OK;
}

/* Masked PCG (Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.1)
 * for A x = Pi rhs from x = 0.  diag == NULL means no preconditioner. */
static int pcg(const sys_t *s, const double *rhs, const double *diag, double tol,
               int32_t maxit, double *x, orc_stats *stats) {
    int64_t n = 3 * s->nv;
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    int status = ORC_OK;
    int32_t it = 0;
    double bnorm, rr, rel = 0.0;
    if (!r || !z || !p || !q) { status = ORC_E_ARG; goto done; }
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = (s->pinned && s->pinned[i / 3]) ? 0.0 : rhs[i];
    }
    bnorm = sqrt(vdot(n, r, r));
    if (bnorm == 0.0) goto done;
    for (int64_t i = 0; i < n; ++i) z[i] = diag ? r[i] / diag[i] : r[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rz = vdot(n, r, z);
    rr = bnorm * bnorm;
    int converged = 0;
    while (it < maxit) {
        int st = apply_A(s, p, q);
        if (st) { status = st; break; }
        double pq = vdot(n, p, q);
        if (!(pq > 0.0)) { status = ORC_E_NOT_SPD; break; }
        double alpha = rz / pq;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++it;
        rr = vdot(n, r, r);
        if (sqrt(rr) <= tol * bnorm) { converged = 1; break; }
        for (int64_t i = 0; i < n; ++i) z[i] = diag ? r[i] / diag[i] : r[i];
        double rz_new = vdot(n, r, z);
        if (rz_new == 0.0) { converged = 1; break; }
        double beta = rz_new / rz;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    rel = sqrt(rr) / bnorm;
    if (status == ORC_OK && !converged && tol > 0.0) status = ORC_E_NOT_CONVERGED;
done:
    if (stats) {
        stats->iters = it;
        stats->status = status;
        stats->rel_res = rel;
    }
    free(r); free(z); free(p); free(q);
    return status;
}

static int build_diag(const sys_t *s, int32_t precond, double **diag) {
    *diag = NULL;
    if (precond != ORC_PRECOND_JACOBI) return ORC_OK;
    *diag = malloc(sizeof(double) * (size_t)(3 * s->nv));
    if (!*diag) return ORC_E_ARG;
    /* diag(A) = cm M - ck diag(K): the undamped diagonal M - dt^2 diag(K) at dt = 1
     * and zero mass gives -diag(K) */
    double *zero_m = calloc((size_t)(s->nv > 0 ? s->nv : 1), sizeof(double));
    if (!zero_m) return ORC_E_ARG;
    int st = orc_jacobi_diag(s->model, s->nv, s->nt, s->tets, s->B, s->V0, s->mu, s->lam,
                             zero_m, 1.0, s->d, *diag);
    free(zero_m);
    if (st) return st;
    for (int64_t i = 0; i < 3 * s->nv; ++i) {
        (*diag)[i] = s->cm * s->mass[i / 3] + s->ck * (*diag)[i];
        if (s->pinned && s->pinned[i / 3]) (*diag)[i] = 1.0;
    }
    return ORC_OK;
}

int orc_implicit_step(int model, int64_t nv, int64_t nt, const int32_t *tets,
                      const double *B, const double *V0, const double *mu, const double *lam,
                      const double *mass, const uint8_t *pinned,
                      double dt, const double g[3], double alpha, double beta,
                      double tol, int32_t maxit, int32_t precond,
                      double *d, double *v, double *dv_out, orc_stats *stats) {
    /* Backward Euler with Rayleigh damping D = alpha M - beta K(d) (K = df/dx,
     * so -K is the stiffness of the textbook form alpha M + beta K_s), linearised
     * about (d, v):
     *   M dv = dt (f(d + dt (v + dv)) + M g - D (v + dv)),  f(d + e) ~ f(d) + K e
     *   => (M + dt D - dt^2 K) dv = dt (f + M g - D v + dt K v)
     *   => A = (1 + dt alpha) M - (dt^2 + dt beta) K,
     *      b = dt (f + M g - alpha M v + (dt + beta) K v). */
    int64_t n = 3 * nv;
    sys_t s = {model, nv, nt, tets, B, V0, mu, lam, mass, d, pinned, dt,
               1.0 + dt * alpha, dt * dt + dt * beta};
    double *f = malloc(sizeof(double) * (size_t)n), *kv = malloc(sizeof(double) * (size_t)n);
    double *b = malloc(sizeof(double) * (size_t)n), *dv = malloc(sizeof(double) * (size_t)n);
    double *diag = NULL;
    int st = ORC_E_ARG;
    if (!f || !kv || !b || !dv) goto done;
    /* b = dt (f(d) + M g - alpha M v + (dt + beta) K(d) v) */
    st = orc_forces(model, nv, nt, tets, B, V0, mu, lam, d, f);
    if (st) goto done;
    st = orc_kmul(model, nv, nt, tets, B, V0, mu, lam, d, v, kv);
    if (st) goto done;
    for (int64_t i = 0; i < n; ++i)
        b[i] = dt * (f[i] + mass[i / 3] * g[i % 3] - alpha * mass[i / 3] * v[i] + (dt + beta) * kv[i]);
    st = build_diag(&s, precond, &diag);
    if (st) goto done;
    st = pcg(&s, b, diag, tol, maxit, dv, stats);
    if (st != ORC_OK && st != ORC_E_NOT_CONVERGED) goto done;
    /* v += dv; d += dt v */
    for (int64_t i = 0; i < n; ++i) {
        v[i] += dv[i];
        d[i] += dt * v[i];
    }
    if (dv_out) memcpy(dv_out, dv, sizeof(double) * (size_t)n);
done:
    free(f); free(kv); free(b); free(dv); free(diag);
    return st;
}

int orc_step_vjp(int model, int64_t nv, int64_t nt, const int32_t *tets,
                 const double *B, const double *V0, const double *mu, const double *lam,
                 const double *E, const double *mass, const uint8_t *pinned,
                 double dt, double alpha, double beta, double tol, int32_t maxit, int32_t precond,
                 const double *d_n, const double *v_np1,
                 const double *gx, const double *gv,
                 double *d_bar, double *v_bar, double *E_bar, orc_stats *stats) {
    /* Forward (see orc_implicit_step): v' = v + dv, A dv = Pi b,
     *   A = cm M - ck K(d), b = dt f(d) + dt M g - dt alpha M v + ck K(d) v,
     *   cm = 1 + dt alpha, ck = dt^2 + dt beta, d' = d + dt v'.
     * Reverse, with g^ = gv + dt gx and A w = Pi g^ (A symmetric):
     *   d_bar = gx + dt K w + ck T[v, w] + ck T[dv, w] = gx + dt K w + ck T[v', w]
     *   v_bar = g^ + ck K w - dt alpha M w
     *   E_bar_t += (w_t . (dt f_t + ck K_t v')) / E_t   (f, K linear in E_t; M is not) */
    int64_t n = 3 * nv;
    const double cm = 1.0 + dt * alpha, ck = dt * dt + dt * beta;
    sys_t s = {model, nv, nt, tets, B, V0, mu, lam, mass, d_n, pinned, dt, cm, ck};
    double *gh = malloc(sizeof(double) * (size_t)n), *w = malloc(sizeof(double) * (size_t)n);
    double *kw = malloc(sizeof(double) * (size_t)n), *tw = malloc(sizeof(double) * (size_t)n);
    double *diag = NULL;
    int st = ORC_E_ARG;
    if (!gh || !w || !kw || !tw) goto done;
    for (int64_t i = 0; i < n; ++i) gh[i] = gv[i] + dt * gx[i];
    st = build_diag(&s, precond, &diag);
    if (st) goto done;
    st = pcg(&s, gh, diag, tol, maxit, w, stats);
    if (st != ORC_OK && st != ORC_E_NOT_CONVERGED) goto done;
    st = orc_kmul(model, nv, nt, tets, B, V0, mu, lam, d_n, w, kw);
    if (st) goto done;
    st = orc_tmul(model, nv, nt, tets, B, V0, mu, lam, d_n, v_np1, w, tw);
    if (st) goto done;
    for (int64_t i = 0; i < n; ++i) {
        d_bar[i] = gx[i] + dt * kw[i] + ck * tw[i];
        v_bar[i] = gh[i] + ck * kw[i] - dt * alpha * mass[i / 3] * w[i];
    }
    if (E_bar) {
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t *tv = tets + 4 * t;
            double G[9], dF[9], P[9], dP[9], lin[9];
            tet_grad(tv, d_n, B + 9 * t, G);
            tet_grad(tv, v_np1, B + 9 * t, dF);
            st = orc_stress(model, mu[t], lam[t], G, P);
            if (st) goto done;
            st = orc_dstress(model, mu[t], lam[t], G, dF, dP);
            if (st) goto done;
            for (int i = 0; i < 9; ++i) lin[i] = dt * P[i] + ck * dP[i];
            /* w_t . (scatter of -V0 lin B^T) */
            double loc[12] = {0};
            int32_t id[4] = {0, 1, 2, 3};
            tet_scatter(id, V0[t], lin, B + 9 * t, loc);
            double s2 = 0.0;
            for (int c = 0; c < 4; ++c)
                for (int r = 0; r < 3; ++r) s2 += w[3 * (int64_t)tv[c] + r] * loc[3 * c + r];
            E_bar[t] += s2 / E[t];
        }
    }
    st = ORC_OK;
    if (stats && stats->status == ORC_E_NOT_CONVERGED) st = ORC_E_NOT_CONVERGED;
done:
    free(gh); free(w); free(kw); free(tw); free(diag);
    return st;
}

/* ---- assembled stiffness on edges --------------------------------------------
 * The Vega workload keeps its stiffness matrix on the mesh edges (Developing
 * Domain Libraries, "Example: FEM tetmesh"; Performance Evaluation): one 3x3
 * block per ordered vertex pair that shares a tet, self-pairs included,
 * grouped by the first (tail) vertex.  Block (i, j) is df_i/dd_j, the sum over
 * the tets holding both vertices of that tet's corner block. */

static int i64_cmp(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : x > y;
}

int orc_edges(int64_t nv, int64_t nt, const int32_t *tets, int64_t *row_ptr, int32_t *col,
              int64_t cap, int64_t *n_edges) {
    int64_t *key = malloc(sizeof(int64_t) * (size_t)(16 * nt + 1));
    if (!key) return ORC_E_ARG;
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int32_t i = tets[4 * t + a], j = tets[4 * t + b];
                if (i < 0 || i >= nv || j < 0 || j >= nv) { free(key); return ORC_E_ARG; }
                key[16 * t + 4 * a + b] = (int64_t)i * nv + j;
            }
    qsort(key, (size_t)(16 * nt), sizeof(int64_t), i64_cmp);
    int64_t n = 0;
    for (int64_t v = 0; v <= nv; ++v) row_ptr[v] = 0;
    for (int64_t k = 0; k < 16 * nt; ++k) {
        if (k > 0 && key[k] == key[k - 1]) continue;
        if (n < cap) col[n] = (int32_t)(key[k] % nv);
        ++row_ptr[key[k] / nv + 1];
        ++n;
    }
    for (int64_t v = 0; v < nv; ++v) row_ptr[v + 1] += row_ptr[v];
    free(key);
    *n_edges = n;
    return n <= cap ? ORC_OK : ORC_E_ARG;
}

static int64_t edge_find(const int64_t *row_ptr, const int32_t *col, int32_t i, int32_t j) {
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < row_ptr[i + 1] && col[lo] == j) ? lo : -1;
}

int orc_assemble(int model, int64_t nv, int64_t nt, const int32_t *tets,
                 const double *B, const double *V0, const double *mu, const double *lam,
                 const double *d, const int64_t *row_ptr, const int32_t *col, double *blocks) {
    memset(blocks, 0, sizeof(double) * (size_t)(9 * row_ptr[nv]));
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *tv = tets + 4 * t;
        const double *Bt = B + 9 * t;
        double G[9];
        tet_grad(tv, d, Bt, G);
        for (int b = 0; b < 4; ++b)
            for (int k = 0; k < 3; ++k) {
                /* unit displacement of corner b along axis k: dF = e_k (x) grad(N_b) */
                double gb[3], dF[9], dP[9], loc[12] = {0};
                const int32_t id[4] = {0, 1, 2, 3};
                for (int j = 0; j < 3; ++j)
                    gb[j] = b ? Bt[3 * (b - 1) + j] : -(Bt[j] + Bt[3 + j] + Bt[6 + j]);
                m_zero(dF);
                for (int j = 0; j < 3; ++j) dF[3 * k + j] = gb[j];
                int st = orc_dstress(model, mu[t], lam[t], G, dF, dP);
                if (st) return st;
                tet_scatter(id, V0[t], dP, Bt, loc);   /* loc[3a + r] = df_{a,r} / dd_{b,k} */
                for (int a = 0; a < 4; ++a) {
                    const int64_t e = edge_find(row_ptr, col, tv[a], tv[b]);
                    if (e < 0) return ORC_E_ARG;
                    for (int r = 0; r < 3; ++r) blocks[9 * e + 3 * r + k] += loc[3 * a + r];
                }
            }
    }
    return ORC_OK;
}

int orc_spmv(int64_t nv, const int64_t *row_ptr, const int32_t *col, const double *blocks,
             const double *u, double *y) {
    for (int64_t i = 0; i < nv; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) acc[r] += blocks[9 * e + 3 * r + c] * u[3 * (int64_t)col[e] + c];
        for (int r = 0; r < 3; ++r) y[3 * i + r] = acc[r];
    }
    return ORC_OK;
}

/* ---- spring-mass workload ---------------------------------------------------
 * The introductory example of the paper (Ebb by example: a spring-mass
 * simulation on the edges of a tet mesh): a spring on every directed edge,
 * its rest length from the rest positions; each vertex sums the springs of
 * the edges leaving it (a query loop over the edges grouped by tail, a +=
 * reduction into the vertex force), then an exclusive per-vertex update
 * integrates and clears the force; the kinetic energy is a global +=.
 * Springs restore: an edge (v -> h) adds K (dq - L dq/|dq|), dq = q_h - q_v, to
 * the force on v (minus the gradient of K (|dq| - L)^2 / 2); |dq| = 0 adds 0. */

int orc_spring_rest(int64_t ne, const int32_t *tail, const int32_t *head, const double *X, double *rest) {
    for (int64_t e = 0; e < ne; ++e) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double t = X[3 * (int64_t)head[e] + k] - X[3 * (int64_t)tail[e] + k];
            s += t * t;
        }
        rest[e] = sqrt(s);
    }
    return ORC_OK;
}

int orc_spring_forces(int64_t nv, int64_t ne, const int32_t *tail, const int32_t *head, const double *rest,
                      double K, const double *q, double *force) {
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t v = tail[e], h = head[e];
        if (v < 0 || v >= nv || h < 0 || h >= nv) return ORC_E_ARG;
        double dq[3], n2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            dq[k] = q[3 * h + k] - q[3 * v + k];
            n2 += dq[k] * dq[k];
        }
        const double n = sqrt(n2);
        for (int k = 0; k < 3; ++k) {
            const double dir = n > 0.0 ? dq[k] / n : 0.0;
            force[3 * v + k] += K * (dq[k] - rest[e] * dir);
        }
    }
    return ORC_OK;
}

int orc_spring_apply(int64_t nv, const double *mass, double dt, double *q, double *qd, double *force) {
    for (int64_t v = 0; v < nv; ++v)
        for (int k = 0; k < 3; ++k) {
            const int64_t i = 3 * v + k;
            const double a = force[i] / mass[v];
            q[i] += qd[i] * dt + 0.5 * a * dt * dt;
            qd[i] += a * dt;
            force[i] = 0.0;
        }
    return ORC_OK;
}

double orc_kinetic_energy(int64_t nv, const double *mass, const double *qd) {
    double E = 0.0;
    for (int64_t v = 0; v < nv; ++v)
        E += 0.5 * mass[v] * (qd[3 * v] * qd[3 * v] + qd[3 * v + 1] * qd[3 * v + 1] + qd[3 * v + 2] * qd[3 * v + 2]);
    return E;
}

/* ---- grouping and reordering ------------------------------------------------ */

typedef struct { int64_t key; int64_t val; } kv_t;

static int kv_cmp(const void *a, const void *b) {
    const kv_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->val != y->val) return x->val < y->val ? -1 : 1;
    return 0;
}

int orc_group_by(int64_t nv, int64_t nt, const int32_t *tets, int64_t *row_ptr, int32_t *inc) {
    /* Sort the (vertex, tet, corner) incidence table by its vertex key
     * (ties by tet, then corner) and record each vertex's [begin, end)
     * range: the grouping of Runtime Implementation, "Relational
     * Primitives Implementations". */
    kv_t *e = malloc(sizeof(kv_t) * (size_t)(4 * nt + 1));
    if (!e) return ORC_E_ARG;
    for (int64_t t = 0; t < nt; ++t)
        for (int c = 0; c < 4; ++c) {
            int32_t v = tets[4 * t + c];
            if (v < 0 || v >= nv) { free(e); return ORC_E_ARG; }
            e[4 * t + c].key = v;
            e[4 * t + c].val = 4 * t + c;
        }
    qsort(e, (size_t)(4 * nt), sizeof(kv_t), kv_cmp);
    int64_t k = 0;
    for (int64_t v = 0; v <= nv; ++v) {
        while (k < 4 * nt && e[k].key < v) ++k;
        row_ptr[v] = k;
    }
    for (int64_t i = 0; i < 4 * nt; ++i) inc[i] = (int32_t)e[i].val;
    free(e);
    return ORC_OK;
}

typedef struct { int64_t seg; uint64_t code; int64_t id; } skv_t;

static int skv_cmp(const void *a, const void *b) {
    const skv_t *x = a, *y = b;
    if (x->seg != y->seg) return x->seg < y->seg ? -1 : 1;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

int orc_morton(int64_t nv, int64_t nt, const double *X, const int32_t *tets,
               uint64_t *codes, int32_t *vperm, int32_t *tperm) {
    return orc_morton_seg(nv, nt, X, tets, NULL, codes, vperm, tperm);
}

int orc_morton_seg(int64_t nv, int64_t nt, const double *X, const int32_t *tets, const int32_t *seg,
                   uint64_t *codes, int32_t *vperm, int32_t *tperm) {
    double lo[3], hi[3], sc[3];
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t v = 0; v < nv; ++v)
        for (int a = 0; a < 3; ++a) {
            if (X[3 * v + a] < lo[a]) lo[a] = X[3 * v + a];
            if (X[3 * v + a] > hi[a]) hi[a] = X[3 * v + a];
        }
    const double two21 = 2097152.0;
    for (int a = 0; a < 3; ++a) sc[a] = (hi[a] > lo[a]) ? two21 / (hi[a] - lo[a]) : 0.0;
    kv_t *e = malloc(sizeof(kv_t) * (size_t)(nt ? nt : 1));
    skv_t *sv = malloc(sizeof(skv_t) * (size_t)(nv ? nv : 1));
    if (!e || !sv) { free(e); free(sv); return ORC_E_ARG; }
    for (int64_t v = 0; v < nv; ++v) {
        uint64_t q[3], code = 0;
        for (int a = 0; a < 3; ++a) {
            volatile double diff = X[3 * v + a] - lo[a]; /* one subtract, one multiply */
            volatile double s = diff * sc[a];
            double fl = floor(s);
            q[a] = fl >= two21 - 1.0 ? (uint64_t)2097151 : (uint64_t)fl;
        }
        for (int b = 0; b < 21; ++b)
            for (int a = 0; a < 3; ++a)
                code |= ((q[a] >> b) & 1ull) << (3 * b + a);
        codes[v] = code;
        /* vertices in order of (segment, code, id); one segment when seg is NULL */
        sv[v].seg = seg ? seg[v] : 0;
        sv[v].code = code;
        sv[v].id = v;
    }
    qsort(sv, (size_t)nv, sizeof(skv_t), skv_cmp);
    int32_t *inv = malloc(sizeof(int32_t) * (size_t)(nv ? nv : 1));
    if (!inv) { free(e); free(sv); return ORC_E_ARG; }
    for (int64_t i = 0; i < nv; ++i) {
        vperm[i] = (int32_t)sv[i].id;
        inv[sv[i].id] = (int32_t)i;
    }
    free(sv);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t m = inv[tets[4 * t]];
        for (int c = 1; c < 4; ++c)
            if (inv[tets[4 * t + c]] < m) m = inv[tets[4 * t + c]];
        e[t].key = m;
        e[t].val = t;
    }
    qsort(e, (size_t)nt, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < nt; ++i) tperm[i] = (int32_t)e[i].val;
    free(inv);
    free(e);
    return ORC_OK;
}
