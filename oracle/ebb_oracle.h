/* ebb_oracle.h -- CPU reference for the tet-FEM element map.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the GPU library.
 *
 * Everything is plain FP64 and serial: one tet at a time in row order, the
 * semantics of the paper's CPU specialisation (Runtime Implementation,
 * "CPU/GPU Specialization": the kernel body wrapped in a loop over rows).
 *
 * Layout: row-major AoS.  X, d, u, v, f, y: [nv][3]; tets: [nt][4] int32;
 * B: [nt][3][3] (B = Dm^-1); V0, mu, lam, E: [nt]; mass: [nv].
 */
#ifndef EBB_ORACLE_H
#define EBB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_STVK = 0, ORC_NH = 1 };
enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_DEGENERATE = -8, ORC_E_INVERTED = -9,
       ORC_E_NOT_SPD = -10, ORC_E_NOT_CONVERGED = -11 };
enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_JACOBI = 1 };

/* Lame parameters from Young's modulus and Poisson's ratio. */
void orc_lame(double E, double nu, double *mu, double *lam);

/* Rest-shape precompute: B = Dm^-1, V0 = det(Dm)/6, per-tet mu/lam from
 * E[t] (nt values) and nu, lumped mass m_v = sum rho V0 / 4.
 * Returns ORC_E_DEGENERATE (and *bad_tet) if some V0 <= 0. */
int orc_precompute(int64_t nv, int64_t nt, const double *X, const int32_t *tets,
                   double rho, const double *E, double nu,
                   double *B, double *V0, double *mu, double *lam, double *mass,
                   int64_t *bad_tet);

/* First Piola-Kirchhoff stress of one element for displacement gradient G. */
int orc_stress(int model, double mu, double lam, const double G[9], double P[9]);
/* Directional derivative dP = dP/dF : dF at G. */
int orc_dstress(int model, double mu, double lam, const double G[9],
                const double dF[9], double dP[9]);
/* Second directional derivative d2P[A, W] at G (symmetric in A, W). */
int orc_d2stress(int model, double mu, double lam, const double G[9],
                 const double A[9], const double W[9], double Q[9]);
/* Strain energy density. */
int orc_energy_density(int model, double mu, double lam, const double G[9], double *psi);

/* Internal force f = -dW/dx, overwriting f.  ORC_E_INVERTED if NH J <= 0. */
int orc_forces(int model, int64_t nv, int64_t nt, const int32_t *tets,
               const double *B, const double *V0, const double *mu, const double *lam,
               const double *d, double *f);
/* y = K u with K = df/dx at displacement d, overwriting y. */
int orc_kmul(int model, int64_t nv, int64_t nt, const int32_t *tets,
             const double *B, const double *V0, const double *mu, const double *lam,
             const double *d, const double *u, double *y);
/* Total strain energy W = sum_t V0 psi. */
int orc_energy(int model, int64_t nv, int64_t nt, const int32_t *tets,
               const double *B, const double *V0, const double *mu, const double *lam,
               const double *d, double *W);
/* diag[v][c] = mass[v] - dt^2 K[(v,c),(v,c)]. */
int orc_jacobi_diag(int model, int64_t nv, int64_t nt, const int32_t *tets,
                    const double *B, const double *V0, const double *mu, const double *lam,
                    const double *mass, double dt, const double *d, double *diag);

typedef struct { int32_t iters, status; double rel_res; } orc_stats;

/* One linearised backward-Euler step with masked (Jacobi-)PCG and Rayleigh
 * damping D = alpha M - beta K (alpha = beta = 0: undamped).  d and v are
 * updated in place.  dv_out (nullable) receives the velocity increment. */
int orc_implicit_step(int model, int64_t nv, int64_t nt, const int32_t *tets,
                      const double *B, const double *V0, const double *mu, const double *lam,
                      const double *mass, const uint8_t *pinned,
                      double dt, const double g[3], double alpha, double beta,
                      double tol, int32_t maxit, int32_t precond,
                      double *d, double *v, double *dv_out, orc_stats *stats);

/* T[a, w] = grad_x (w^T K(x) a), overwriting out. */
int orc_tmul(int model, int64_t nv, int64_t nt, const int32_t *tets,
             const double *B, const double *V0, const double *mu, const double *lam,
             const double *d, const double *a, const double *w, double *out);

/* Vector-Jacobian product of one implicit step.  Given gx = dL/dx_{n+1} and
 * gv = dL/dv_{n+1}, returns dL/dd_n (d_bar), dL/dv_n (v_bar) and accumulates
 * dL/dE_t into E_bar (E is the per-tet Young's modulus used in precompute). */
int orc_step_vjp(int model, int64_t nv, int64_t nt, const int32_t *tets,
                 const double *B, const double *V0, const double *mu, const double *lam,
                 const double *E, const double *mass, const uint8_t *pinned,
                 double dt, double alpha, double beta, double tol, int32_t maxit, int32_t precond,
                 const double *d_n, const double *v_np1,
                 const double *gx, const double *gv,
                 double *d_bar, double *v_bar, double *E_bar, orc_stats *stats);

/* Directed edges (i, j) of the tets, self-pairs included, sorted by (i, j):
 * row_ptr (nv+1) over tails, col (heads, capacity cap); *n_edges = count
 * (ORC_E_ARG if it exceeds cap). */
int orc_edges(int64_t nv, int64_t nt, const int32_t *tets, int64_t *row_ptr, int32_t *col,
              int64_t cap, int64_t *n_edges);
/* Assembled stiffness at displacement d: blocks[9e + 3r + c] = df_{i,r}/dd_{j,c}
 * for edge e = (i, j), summed over the tets holding both vertices. */
int orc_assemble(int model, int64_t nv, int64_t nt, const int32_t *tets,
                 const double *B, const double *V0, const double *mu, const double *lam,
                 const double *d, const int64_t *row_ptr, const int32_t *col, double *blocks);
/* y_i = sum over edges (i, j) of K_ij u_j. */
int orc_spmv(int64_t nv, const int64_t *row_ptr, const int32_t *col, const double *blocks,
             const double *u, double *y);

/* Spring-mass workload: rest[e] = |X_head - X_tail|; force[tail] += K (dq - rest dq/|dq|)
 * over the edges in row order (dq = q_head - q_tail; 0 if |dq| = 0); the exclusive
 * update a = force/mass, q += qd dt + a dt^2/2, qd += a dt, force = 0; the kinetic
 * energy sum of mass |qd|^2 / 2.  Vectors (nv, 3). */
int orc_spring_rest(int64_t ne, const int32_t *tail, const int32_t *head, const double *X, double *rest);
int orc_spring_forces(int64_t nv, int64_t ne, const int32_t *tail, const int32_t *head, const double *rest,
                      double K, const double *q, double *force);
int orc_spring_apply(int64_t nv, const double *mass, double dt, double *q, double *qd, double *force);
double orc_kinetic_energy(int64_t nv, const double *mass, const double *qd);

/* Grouping of the tets.v[4] key-field by vertex: CSR of incidence 4t+c,
 * rows in (t, c) order.  row_ptr: nv+1, inc: 4 nt. */
int orc_group_by(int64_t nv, int64_t nt, const int32_t *tets, int64_t *row_ptr, int32_t *inc);
/* Multi-threaded orc_forces / orc_kmul for timing (OpenMP, nthreads threads): per-corner
 * partials in part (nt x 12, caller-owned), then per-vertex sums over the grouping of
 * orc_group_by in (tet, corner) order; equal bit for bit to the serial functions. */
int orc_forces_mt(int model, int64_t nv, int64_t nt, const int32_t *tets,
                  const double *B, const double *V0, const double *mu, const double *lam,
                  const double *d, double *f, const int64_t *row_ptr, const int32_t *inc, double *part,
                  int nthreads);
int orc_kmul_mt(int model, int64_t nv, int64_t nt, const int32_t *tets,
                const double *B, const double *V0, const double *mu, const double *lam,
                const double *d, const double *u, double *y, const int64_t *row_ptr, const int32_t *inc,
                double *part, int nthreads);


/* Morton order of the rest positions.  codes[nv]; vperm[new] = old vertex;
 * tperm[new] = old tet (tets sorted by the min new vertex id of their
 * corners, ties by old row). */
int orc_morton(int64_t nv, int64_t nt, const double *X, const int32_t *tets,
               uint64_t *codes, int32_t *vperm, int32_t *tperm);
/* The same with the vertices ordered by (seg[v], code, v): a Morton order within each segment
 * (seg: one int32 label per vertex, e.g. the mesh of a batch).  The tets are then ordered as
 * above, by their smallest new vertex id, so tets of one segment stay together when no tet
 * spans two. */
int orc_morton_seg(int64_t nv, int64_t nt, const double *X, const int32_t *tets, const int32_t *seg,
                   uint64_t *codes, int32_t *vperm, int32_t *tperm);

#ifdef __cplusplus
}
#endif
#endif
