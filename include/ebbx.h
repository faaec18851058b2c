/* ebbx.h -- C-ABI of the MI355X (gfx950) tet-FEM element map.
 *
 * The calls follow the relational model of Ebb (Bernstein et al., "Ebb: A
 * DSL for Physical Simulation on CPUs and GPUs"): relations are tables,
 * fields are column-stored arrays over a relation, key-fields map rows of one
 * relation to rows of another, and grouping a relation by a key-field builds
 * the inverted index that query-loops read (Developing Domain Libraries,
 * "Relational Modeling Primitives"; Runtime Implementation).  Calls execute
 * immediately, like the paper's OpenGL-style runtime API.
 *
 * On top of the relations sits the tet-FEM domain of the paper's Vega and
 * FreeFem++ workloads (Developing Domain Libraries, "Example: FEM tetmesh";
 * Performance Evaluation): displacement, velocity and force on vertices,
 * material on tets, hyperelastic internal forces, the stiffness product and
 * an implicit backward-Euler step solved with (Jacobi-)preconditioned CG.
 *
 * Conventions shared by every call:
 *  - Return value: EBBX_OK (0) or a negative ebbx_status.  A failed call has
 *    no side effect and sets any output handle to NULL; ebbx_last_error()
 *    returns a thread-local message for the last failure.  No C++ exception
 *    crosses this boundary.
 *  - Memory: every pointer argument named *_dev (and every vector argument of
 *    the compute calls) is device memory on the GPU the library runs on.
 *    Bound fields are borrowed: the caller owns them and keeps them alive
 *    while a relation or FEM object that uses them exists.  Hidden fields
 *    (B = Dm^-1, V0, mass, incidence, scratch, solver vectors) are owned by
 *    the library, allocated through the allocator hook (default hipMalloc)
 *    and released by the matching *_destroy call.
 *  - Layout: column store ("struct of arrays").  A field of ncomp components
 *    over a relation of size n is ncomp contiguous columns of n elements
 *    (a C-contiguous array of shape (ncomp, n)).  Vertex vectors d, u, v, f,
 *    y are FP64 (3, nv).
 *  - Streams: ebbx_stream is a hipStream_t (NULL = the null stream).  Setup
 *    calls (create, bind, group, reorder, fem_create) are synchronous.  Compute
 *    calls enqueue on the given stream and return without synchronising;
 *    conditions found on the device (inverted element, CG breakdown, no
 *    convergence) are reported in device-side stats read by ebbx_stats_fetch.
 *  - Threads: calls on different objects may come from different threads;
 *    calls on one object must not overlap.
 *  - Streams of one FEM domain: its element calls share library scratch (the
 *    block strategies' halo, the segmented strategy's partials) and its steps
 *    share the solver's vectors, so work on one domain must be ordered: one
 *    stream, or events between streams.  Different domains are independent.
 *  - Rounding: the SEG, BLOCK and OWNER strategies and every CG reduction sum
 *    in a fixed order, so their results are bitwise reproducible run to run;
 *    ATOMIC and BLOCK_LDS are not.
 */
#ifndef EBBX_H
#define EBBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ebbx_status;
enum {
    EBBX_OK = 0,
    EBBX_E_ARG = -1,          /* null handle, bad enum, bad size */
    EBBX_E_DTYPE = -2,        /* field has the wrong element type */
    EBBX_E_SHAPE = -3,        /* field has the wrong component count */
    EBBX_E_LAYOUT = -4,       /* pointer misaligned for its type */
    EBBX_E_KEY_RANGE = -5,    /* a key is outside [0, size of target) */
    EBBX_E_PHASE = -6,        /* an output aliases an input of the same call */
    EBBX_E_NOT_GROUPED = -7,  /* the call needs a grouping that was not built */
    EBBX_E_DEGENERATE = -8,   /* a rest tet has V0 <= 0 */
    EBBX_E_INVERTED = -9,     /* a deformed neo-Hookean tet has J <= 0 */
    EBBX_E_NOT_SPD = -10,     /* CG met p^T A p <= 0 */
    EBBX_E_NOT_CONVERGED = -11, /* CG reached maxit before tol (iterate kept) */
    EBBX_E_HIP = -12,         /* a HIP runtime call failed */
    EBBX_E_OOM = -13,         /* allocation failed */
    EBBX_E_STATE = -14,       /* object used in a state that forbids the call */
    EBBX_E_NOT_FOUND = -15    /* no field or key-field of that name */
};

typedef enum { EBBX_F32 = 0, EBBX_F64 = 1, EBBX_I32 = 2, EBBX_U8 = 3, EBBX_I64 = 4 } ebbx_dtype;
typedef struct ebbx_relation_s *ebbx_relation;
typedef struct ebbx_fem_s *ebbx_fem;
typedef struct ebbx_batch_s *ebbx_batch;
typedef struct ebbx_springs_s *ebbx_springs;
typedef void *ebbx_stream;   /* hipStream_t */

/* Message of the last failed call on this thread ("" if none). */
const char *ebbx_last_error(void);

/* Library version, e.g. 100 for 0.1.0. */
int32_t ebbx_version(void);

/* Allocator hook for hidden fields.  alloc(bytes, ctx, stream) returns device
 * memory or NULL; free(ptr, ctx) releases it.  Passing alloc = NULL restores
 * hipMalloc/hipFree.  Objects keep the hook that was current when they were
 * created and release their memory through it. */
ebbx_status ebbx_set_allocator(void *(*alloc)(size_t bytes, void *ctx, ebbx_stream stream),
                               void (*free_fn)(void *ptr, void *ctx), void *ctx);

/* ---- relations, fields, key-fields (Developing Domain Libraries) -------- */

/* A relation (table) of `size` rows; `name` is copied. */
ebbx_status ebbx_relation_create(const char *name, int64_t size, ebbx_relation *out);
ebbx_status ebbx_relation_destroy(ebbx_relation rel);
ebbx_status ebbx_relation_size(ebbx_relation rel, int64_t *out);

/* Bind caller-owned column-store memory (ncomp, size) of type dtype as field
 * `name` (a zero-copy view, as the paper's interoperation with external
 * libraries allows).  Rebinding a name replaces the view.  EBBX_E_LAYOUT if
 * dev_ptr is not aligned to its element size. */
ebbx_status ebbx_field_bind(ebbx_relation rel, const char *name, ebbx_dtype dtype,
                            int32_t ncomp, void *dev_ptr);

/* Bind a key-field: `arity` int32 keys per row of rel, column store
 * (arity, size), each referring to a row of `target` (e.g. tets.v[4] ->
 * verts).  Validates on the device that every key is in [0, size(target)),
 * returning EBBX_E_KEY_RANGE otherwise (the paper's guarantee that key
 * accesses stay in bounds by construction).  Synchronous. */
ebbx_status ebbx_keyfield_bind(ebbx_relation rel, const char *name, ebbx_relation target,
                               int32_t arity, int32_t *dev_ptr);

/* Group rel by key-field `keyfield` (Runtime Implementation, "Relational
 * Primitives Implementations"): builds on the target relation the hidden
 * index of the (row, slot) incidences of rel whose key equals each target
 * row -- CSR with row_ptr (size(target)+1, int64) and entries 4*row+slot
 * (for arity 4; in general arity*row+slot, int32), each target row's entries
 * in increasing order.  Deterministic and bit-exact.  Synchronous. */
ebbx_status ebbx_relation_group_by(ebbx_relation rel, const char *keyfield);

/* Copy the grouping built by ebbx_relation_group_by into caller buffers:
 * row_ptr_dev (size(target)+1 int64), inc_dev (arity*size(rel) int32).
 * EBBX_E_NOT_GROUPED if the grouping does not exist.  Synchronous. */
ebbx_status ebbx_group_export(ebbx_relation rel, const char *keyfield, int64_t *row_ptr_dev,
                              int32_t *inc_dev);

/* Morton (Z-order) locality order, which the opaque-key model lets the
 * runtime choose (Developing Domain Libraries: keys are opaque, so the
 * runtime may reorder relations).  From the FP64 (3, nv) field `pos_field`
 * of verts: per-axis bounding box [lo, hi], q = min(2^21-1, floor((x-lo) *
 * (2^21/(hi-lo)))) (q = 0 on a flat axis), bit b of q_x, q_y, q_z at bits
 * 3b, 3b+1, 3b+2 of a uint64 code; vertices sorted by (code, old id).  With
 * seg_keyfield (nullable), an arity-1 key-field of verts (e.g. the mesh of
 * each vertex of a batch), the vertices are sorted by (segment, code, old id)
 * instead: a Morton order within each segment, the segments in key order, so
 * a batch's meshes stay contiguous (codes still use the one bounding box of
 * all vertices).  Rows of rel are then sorted by (min over slots of the new
 * vertex id of key-field `keyfield`, old row).  Outputs (device, nullable):
 * codes_dev[nv] (uint64), vperm_dev[nv] and tperm_dev[size(rel)], each
 * mapping new -> old.  Nothing is permuted.  Synchronous. */
ebbx_status ebbx_morton_order(ebbx_relation verts, const char *pos_field, const char *seg_keyfield,
                              ebbx_relation rel, const char *keyfield, uint64_t *codes_dev,
                              int32_t *vperm_dev, int32_t *tperm_dev);

/* Permute rel in place by new_to_old_dev (a permutation of [0, size)): every
 * bound field and key-field of rel is gathered row-wise, and every key-field
 * of any live relation that targets rel is remapped through the inverse.
 * Groupings involving rel are dropped.  EBBX_E_STATE (nothing permuted) if a
 * live domain holds per-row data of rel: a FEM domain or batch union over rel
 * as its tets or verts, a batch over rel as its meshes, a springs domain over
 * rel as its edges or verts.  Synchronous. */
ebbx_status ebbx_relation_reorder(ebbx_relation rel, const int32_t *new_to_old_dev);

/* ---- the tet-FEM domain -------------------------------------------------- */

enum { EBBX_STVK = 0, EBBX_NH = 1 };
/* Scatter-reduce of per-tet results into vertex fields:
 *   ATOMIC:    FP64 hardware atomics, one per (tet, corner, component);
 *   SEG:       per-corner partials, then a vertex-owned sum over the grouping's
 *              incidence in fixed order (bitwise deterministic);
 *   BLOCK:     consecutive tets form blocks (best after Morton reordering);
 *              a block stages its vertices' fields in LDS, writes each tet
 *              corner's result to its row of the block's precomputed incidence
 *              order, sums each vertex's contiguous rows in fixed order,
 *              stores the vertices whose incident tets all lie in the block,
 *              and writes partial sums of the others to a halo buffer that a
 *              vertex pass sums in block order: no global atomics, bitwise
 *              deterministic;
 *   BLOCK_LDS: as BLOCK, but the in-block sums use FP64 LDS atomics (not
 *              bitwise reproducible);
 *   OWNER:     each block owns a contiguous range of vertices (best after
 *              Morton reordering) and evaluates every tet incident to them,
 *              so a tet on a block boundary is evaluated once per block it
 *              touches; each owned vertex sums its incidences in the
 *              grouping's (tet, corner) order and is stored once: no halo,
 *              no atomics, one kernel, results bitwise equal to SEG;
 *   PIPE:      as BLOCK with blocks of 256 tets, but one workgroup walks a
 *              super-block of `block` consecutive blocks: while it evaluates
 *              one block, the next block's vertex fields stream into LDS
 *              (global-to-LDS loads), and each block vertex's sum is added
 *              to an FP64 accumulator of the super-block, so only vertices
 *              shared between super-blocks go through the halo pass (summed
 *              in super-block order): no global atomics, bitwise
 *              deterministic.  Needs at most 256 vertices per 256-tet block
 *              (a Morton-ordered mesh) and at most 1023 per super-block
 *              (EBBX_E_STATE / EBBX_E_ARG otherwise);
 *   LANES:     as BLOCK (blocks of 64, 128 or 256 tets), but the stiffness
 *              product spends four lanes on each tet: lane r of a quad owns
 *              row (spatial component) r of every 3x3 quantity and the sums
 *              over rows are reduced across the quad (DPP), trading issue
 *              for registers per lane; the other element maps run as
 *              BLOCK.  Bitwise deterministic;
 *   AUTO:      BLOCK with 256 tets per block (ebbx_fem_autotune times the
 *              alternatives on the domain itself).
 * The `block` argument of the calls below is the workgroup size (threads) for
 * ATOMIC and SEG, the number of tets per block (a multiple of 64 from 64 to
 * 1024) for BLOCK and BLOCK_LDS (64..256 for LANES), the owned vertices per block
 * (64, 128 or 256) for OWNER and the 256-tet blocks per workgroup (1..16) for
 * PIPE; 0 picks the
 * default (PIPE: 6, which on a Morton-ordered Kuhn mesh is 256 cells).
 * Tets per thread, BLOCK and BLOCK_LDS: one, or two when the block size is
 * or-ed with EBBX_BLOCK_TPT2 (a block of bt tets on bt/2 threads; bt of 128
 * to 1024); blocks of 1024 tets always take two.  ebbx_fem_get_strategy
 * returns the block argument as set, flag included. */
enum { EBBX_STRAT_AUTO = 0, EBBX_STRAT_ATOMIC = 1, EBBX_STRAT_SEG = 2, EBBX_STRAT_BLOCK = 3,
       EBBX_STRAT_BLOCK_LDS = 4, EBBX_STRAT_OWNER = 5, EBBX_STRAT_PIPE = 6, EBBX_STRAT_LANES = 7 };
#define EBBX_BLOCK_TPT2 0x10000

typedef struct {
    int32_t model;       /* EBBX_STVK or EBBX_NH */
    int32_t elem_prec;   /* EBBX_F32 or EBBX_F64: per-tet arithmetic and storage */
    double rho;          /* density, > 0 */
    double E;            /* Young's modulus (ignored if E_field is set) */
    double nu;           /* Poisson's ratio, in (-1, 0.5) */
    const char *E_field; /* nullable: FP64 (1, nt) per-tet Young's modulus on tets */
    int32_t strategy;    /* EBBX_STRAT_* */
    int32_t block;       /* see the strategies above; 0 = default */
} ebbx_fem_params;

/* Build the FEM domain over `tets` (key-field `keyfield`, arity 4, target
 * `verts`) with rest positions `pos_field` (FP64 (3, nv) on verts) and an
 * optional U8 (1, nv) `pinned_field` (nonzero = Dirichlet vertex).  Computes
 * per tet Dm = [X1-X0 | X2-X0 | X3-X0], V0 = det(Dm)/6 and B = Dm^-1, the Lame
 * parameters mu = E/(2(1+nu)), lam = E nu/((1+nu)(1-2nu)), and the lumped mass
 * m_v = sum of rho V0/4 over incident tets.  EBBX_E_DEGENERATE if a tet has
 * V0 <= 0.  Groups tets by keyfield if not yet grouped.  The FEM keeps views
 * of the key-field and the pinned field; reorder the relations (e.g. Morton)
 * before creating the domain: while it lives, ebbx_relation_reorder of tets or
 * verts fails with EBBX_E_STATE.  Synchronous. */
ebbx_status ebbx_fem_create(ebbx_relation tets, const char *keyfield, ebbx_relation verts,
                            const char *pos_field, const char *pinned_field,
                            const ebbx_fem_params *params, ebbx_fem *out);
ebbx_status ebbx_fem_destroy(ebbx_fem fem);

/* Change the scatter strategy and block size of an existing FEM. */
ebbx_status ebbx_fem_set_strategy(ebbx_fem fem, int32_t strategy, int32_t block);
/* Read back the strategy and block size in use (after AUTO resolution). */
ebbx_status ebbx_fem_get_strategy(ebbx_fem fem, int32_t *strategy, int32_t *block);

/* Autotuner (solver kernels are block-size sensitive; Performance
 * Evaluation, Vega): time the stiffness product at (d, u) under every
 * strategy and a set of block sizes, keep the fastest.  d, u: FP64 (3, nv)
 * device vectors or NULL (then d = 0, u = 1).  cache_path (nullable): a JSON
 * file of earlier choices, one entry per line, keyed by the device, model,
 * precision, material kind, sizes and a fingerprint of the tets' keys; a
 * hit skips the timing, a miss adds the choice (EBBX_E_ARG if the file
 * cannot be written).  results (nullable, room for cap entries) receives
 * the timings in microseconds per call; *n_results the number timed (0 on a
 * cache hit).  Synchronous; every candidate call overwrites library scratch
 * only.  Captured solver graphs are rebuilt on the next step. */
typedef struct {
    int32_t strategy;
    int32_t block;
    double us;
} ebbx_tune_entry;
ebbx_status ebbx_fem_autotune(ebbx_fem fem, const double *d, const double *u, const char *cache_path,
                              ebbx_tune_entry *results, int32_t cap, int32_t *n_results, ebbx_stream stream);

/* Internal elastic force at displacement d (x = X + d): per tet G = dD B with
 * dD = [d1-d0 | d2-d0 | d3-d0], F = I + G, first Piola-Kirchhoff stress P(F)
 * (StVK: P = F (2 mu E + lam tr(E) I), E = (G + G^T + G^T G)/2; NH: P =
 * mu (F - F^-T) + lam ln(J) F^-T), H = -V0 P B^T; columns of H go to corners
 * 1..3 and minus their sum to corner 0, reduced (+=) into f (Vega and
 * FreeFem++ workloads).  accumulate = 0 overwrites f, 1 adds to it (a reduce
 * phase field).  No gravity.  EBBX_E_PHASE if f aliases d.  An NH tet with
 * J <= 0 is counted in the FEM's device status (ebbx_fem_status). */
ebbx_status ebbx_fem_forces(ebbx_fem fem, const double *d, double *f, int32_t accumulate,
                            ebbx_stream stream);

/* Stiffness product y (+)= K u with K = df/dx at displacement d, evaluated
 * matrix-free per tet through dF = dU B and the directional derivative of P:
 * StVK dP = dF S + F (2 mu dE + lam tr(dE) I), dE = sym(F^T dF); NH dP =
 * mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam (F^-T : dF) F^-T; then
 * dH = -V0 dP B^T scattered as in ebbx_fem_forces.  No mass, no mask.
 * EBBX_E_PHASE if y aliases d or u. */
ebbx_status ebbx_fem_Kmul(ebbx_fem fem, const double *d, const double *u, double *y,
                          int32_t accumulate, ebbx_stream stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): ebbx_fem_Kmul with
 * the same arguments, kernels and results (bit for bit), except that the
 * call's scratch -- the shared-vertex partials of the block strategies, the
 * per-corner partials of SEG -- lives in a library-wide device array of
 * EBBX_NOALLOC_SCRATCH_MIB MiB per GPU instead of buffers of the domain.  The
 * call allocates nothing (the domain's tables are built when its strategy is
 * set).  EBBX_E_ARG when the domain needs more scratch than the array holds.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race; calls in one stream are ordered.  The
 * array keeps the last call's contents; a call writes every entry it reads. */
#define EBBX_NOALLOC_SCRATCH_MIB 64
ebbx_status ebbx_fem_Kmul_noalloc(ebbx_fem fem, const double *d, const double *u, double *y,
                                  int32_t accumulate, ebbx_stream stream);

/* Total strain energy W = sum V0 psi(F) into out_dev[0] (FP64):
 * StVK psi = mu E:E + lam tr(E)^2/2; NH psi = mu (tr(F^T F) - 3)/2 - mu ln J
 * + lam (ln J)^2/2. */
ebbx_status ebbx_fem_energy(ebbx_fem fem, const double *d, double *out_dev, ebbx_stream stream);

/* Jacobi diagonal of A = M - dt^2 K(d): diag[c][v] = m_v - dt^2 K[(v,c),(v,c)],
 * computed matrix-free from the 12 per-tet diagonal entries
 * -V0 dP(e_c b_a^T) : (e_c b_a^T), b_a the shape-function gradient of corner a
 * (rows of B for a = 1..3, minus their sum for a = 0).  FP64 (3, nv). */
ebbx_status ebbx_fem_jacobi_diag(ebbx_fem fem, const double *d, double dt, double *diag,
                                 ebbx_stream stream);

/* Copy the lumped mass (nv FP64) into mass_dev. */
ebbx_status ebbx_fem_mass(ebbx_fem fem, double *mass_dev, ebbx_stream stream);

/* Count of inverted NH tets seen by force/stiffness calls since the last
 * reset (reset = 1 clears it after reading).  Synchronises the stream. */
ebbx_status ebbx_fem_status(ebbx_fem fem, int64_t *n_inverted, int32_t reset, ebbx_stream stream);

enum { EBBX_PRECOND_NONE = 0, EBBX_PRECOND_JACOBI = 1 };

typedef struct {
    double dt;        /* time step, > 0 */
    double g[3];      /* body acceleration, e.g. (0, 0, -9.81) */
    double tol;       /* stop when ||r|| <= tol ||Pi b||; 0 runs exactly maxit iterations */
    int32_t maxit;    /* iteration cap, >= 0 */
    int32_t precond;  /* EBBX_PRECOND_* */
    double alpha;     /* Rayleigh mass damping, >= 0 (0: none) */
    double beta;      /* Rayleigh stiffness damping, >= 0 (0: none) */
} ebbx_step_params;

/* Solver report, written to device memory by ebbx_implicit_step. */
typedef struct {
    int32_t iters;        /* CG iterations run */
    int32_t status;       /* EBBX_OK, EBBX_E_NOT_SPD, EBBX_E_NOT_CONVERGED, EBBX_E_INVERTED */
    double rel_res;       /* ||r|| / ||Pi b|| at exit (0 if Pi b = 0) */
    int64_t n_inverted;   /* NH tets with J <= 0 at d_n */
} ebbx_step_stats;

/* One linearised backward-Euler step (Vega workload; Performance Evaluation:
 * each step computes the elastic forces, the stiffness and damping), with
 * Rayleigh damping D = alpha M - beta K(d) (K = df/dx, so -K is the
 * positive stiffness):
 *   A = (1 + dt alpha) M - (dt^2 + dt beta) K(d),
 *   b = dt (f(d) + M g - alpha M v + (dt + beta) K(d) v)
 * (alpha = beta = 0: A = M - dt^2 K, b = dt (f + M g + dt K v)),
 *   Pi zeroes pinned rows; masked PCG from dv = 0 on A dv = Pi b with
 *   alpha = r^T z / p^T A p, beta = r_new^T z_new / r^T z, z = D^-1 r (Jacobi)
 *   or z = r; stop when ||r|| <= tol ||Pi b|| or after maxit iterations;
 *   then v += dv, d += dt v.
 * d and v are FP64 (3, nv), updated in place.  CG scalars and dot products
 * stay in FP64 on the device; the iterations are replayed from captured HIP
 * graphs in chunks of up to 128.  With tol = 0 nothing synchronises the
 * host; with tol > 0 the host reads the device's convergence flag between
 * chunks.  stats_dev (device, nullable) receives the report.  If the solve
 * breaks down (p^T A p <= 0) d and v are left unchanged.  EBBX_E_PHASE if
 * d and v alias; EBBX_E_STATE on the union domain of a batch. */
ebbx_status ebbx_implicit_step(ebbx_fem fem, double *d, double *v, const ebbx_step_params *params,
                               ebbx_step_stats *stats_dev, ebbx_stream stream);


/* ---- stiffness assembled on edges ---------------------------------------- */

/* The Vega workload keeps its stiffness matrix on the mesh edges (Developing
 * Domain Libraries, "Example: FEM tetmesh"; Performance Evaluation).  The
 * edges relation of a domain holds every ordered vertex pair (i, j) that
 * shares a tet, i == j included, grouped by the tail i and sorted by the head
 * j: row_ptr (nv + 1 int32) and col (n_edges int32), a block-CSR pattern.  It
 * is built on the host from the grouping on first use (synchronous), once per
 * domain, with per-edge lists of the (tet, corner, corner) blocks that sum
 * into it.
 *
 * ebbx_fem_assemble: K(d) into one 3x3 block per edge, block(i, j)[r][c] =
 * df_{i,r}/dd_{j,c}, the sum over the tets holding i and j, in ascending tet
 * order, of the tet's corner block.  Each tet's 12 x 12 stiffness is computed
 * in FP64 from the same dP as ebbx_fem_Kmul (columns: unit corner
 * displacements); the blocks are stored at the domain's element precision,
 * nine columns of n_edges values.  The library owns a per-tet scratch of
 * 144 FP64 values per tet (about 1.2 KB/tet) and the blocks.  NH tets with
 * J <= 0 are counted as by ebbx_fem_forces.  Enqueued on stream (after the
 * synchronous first build). */
ebbx_status ebbx_fem_assemble(ebbx_fem fem, const double *d, ebbx_stream stream);

/* y (+)= K u with the blocks of the last ebbx_fem_assemble; FP64 (3, nv)
 * vectors, FP64 accumulation, each row summed in a fixed order.
 * EBBX_E_STATE before any assembly, EBBX_E_PHASE if y aliases u. */
ebbx_status ebbx_fem_spmv(ebbx_fem fem, const double *u, double *y, int32_t accumulate, ebbx_stream stream);

/* Number of directed edges (builds the edges relation if needed). */
ebbx_status ebbx_fem_edge_count(ebbx_fem fem, int64_t *n_edges);

/* Copies into caller device buffers (each nullable): row_ptr (nv + 1 int32),
 * col (n_edges int32), blocks (9, n_edges) FP64, column q = 3 r + c of every
 * block (EBBX_E_STATE for blocks before any assembly).  Enqueued on stream. */
ebbx_status ebbx_fem_edges_get(ebbx_fem fem, int32_t *row_ptr, int32_t *col, double *blocks, ebbx_stream stream);

/* ---- the spring-mass workload -------------------------------------------- */

/* The paper's introductory example (Ebb by example: a spring-mass simulation
 * on a tet mesh) on the same relational runtime: a spring on every row of
 * `edges`, whose arity-1 key-fields `tail` and `head` refer to rows of verts.
 * Creation groups the edges by tail (ebbx_relation_group_by), computes every
 * rest length |X_head - X_tail| from the FP64 (3, nv) field pos_field of verts
 * (the example's per-edge kernel) and keeps row-ordered copies of the heads
 * and rest lengths: later changes to the relations do not affect the domain.
 * Synchronous.  K: the spring constant (finite).  Calls on one domain share
 * its scratch (energy partials, the second position buffer and captured steps
 * of ebbx_springs_run): order them on one stream. */
ebbx_status ebbx_springs_create(ebbx_relation edges, const char *tail, const char *head, ebbx_relation verts,
                                const char *pos_field, double K, ebbx_springs *out);
ebbx_status ebbx_springs_destroy(ebbx_springs sp);

/* Rest lengths (FP64, one per edge) in the order of the edges grouped by tail
 * (each vertex's edges in increasing row order). */
ebbx_status ebbx_springs_rest(ebbx_springs sp, double *rest_dev, ebbx_stream stream);

/* force (+)= for every vertex v, the sum over the edges leaving v of
 * K (dq - L dq / |dq|), dq = q_head - q_v (0 if |dq| = 0): restoring springs,
 * minus the gradient of K (|dq| - L)^2 / 2 (the example's query loop over
 * v.edges reducing into v.force; the printed listing has the opposite sign).
 * FP64 (3, nv) vectors; each vertex's sum in a fixed order.  EBBX_E_PHASE if
 * force aliases q. */
ebbx_status ebbx_springs_forces(ebbx_springs sp, const double *q, double *force, int32_t accumulate,
                                ebbx_stream stream);

/* The example's exclusive per-vertex update: a = force / mass,
 * q += qd dt + a dt^2 / 2, qd += a dt, force = 0.  mass: FP64 (nv), positive.
 * EBBX_E_PHASE if q, qd and force alias. */
ebbx_status ebbx_springs_apply(ebbx_springs sp, const double *mass, double dt, double *q, double *qd,
                               double *force, ebbx_stream stream);

/* E_dev[0] += sum over vertices of mass |qd|^2 / 2 (a global +=; fixed-order
 * two-pass sum, bitwise reproducible). */
ebbx_status ebbx_springs_kinetic_energy(ebbx_springs sp, const double *mass, const double *qd, double *E_dev,
                                        ebbx_stream stream);

/* nsteps of (ebbx_springs_forces with accumulate = 1; ebbx_springs_apply),
 * with the same results bit for bit.  Each step runs as one fused kernel
 * (forces and update of every vertex) that writes the new positions to a
 * second position buffer, 3 nv FP64 owned by sp (allocated on the first call,
 * freed by ebbx_springs_destroy), and the next step writes them back; an odd
 * nsteps starts with one step of the two separate passes, so the result is
 * always in q.  Whole chunks of 32 steps are replayed from a HIP graph
 * captured on first use (recaptured when the pointers or dt change), the rest
 * launched directly.  The contents of force join the first step; force is
 * zero on return. */
ebbx_status ebbx_springs_run(ebbx_springs sp, const double *mass, double dt, int32_t nsteps, double *q,
                             double *qd, double *force, ebbx_stream stream);

/* ---- adjoint (vector-Jacobian products) ---------------------------------- */

/* T[a, w] = grad_x (w^T K(x) a) at displacement d: per tet the second
 * directional derivative Q = d2P[dF_a, dF_w] (dF_a = dA B, dF_w = dW B) of
 * the first Piola-Kirchhoff stress, scattered as -V0 Q B^T like the forces.
 * out (+)= T[a, w]; FP64 (3, nv).  EBBX_E_PHASE if out aliases d, a or w. */
ebbx_status ebbx_fem_Tmul(ebbx_fem fem, const double *d, const double *a, const double *w, double *out,
                          int32_t accumulate, ebbx_stream stream);

/* E_bar[t] += w_t . (dt f_t(d) + dt^2 K_t(d) v) / E_t for every tet (forces and
 * stiffness are linear in the per-tet Young's modulus at fixed Poisson ratio).
 * E_bar: FP64 (nt) device, accumulated.  E_t is the per-tet modulus in use (see
 * ebbx_fem_set_material) or the uniform one. */
ebbx_status ebbx_fem_E_grad(ebbx_fem fem, const double *d, const double *v, const double *w, double dt,
                            double *E_bar, ebbx_stream stream);

/* Vector-Jacobian products of the element maps; every output accumulates and
 * is nullable.  forces (f = f(d)):  d_bar += K(d) w,  E_bar[t] += w_t . f_t / E_t.
 * Kmul (y = K(d) u):  d_bar += T[u, w],  u_bar += K(d) w,  E_bar[t] += w_t . K_t u / E_t
 * (K is symmetric; f and K are linear in E_t at fixed nu).  FP64 (3, nv)
 * vectors, E_bar FP64 (nt).  EBBX_E_PHASE if an output aliases an input. */
ebbx_status ebbx_fem_forces_vjp(ebbx_fem fem, const double *d, const double *w, double *d_bar, double *E_bar,
                                ebbx_stream stream);
ebbx_status ebbx_fem_Kmul_vjp(ebbx_fem fem, const double *d, const double *u, const double *w, double *d_bar,
                              double *u_bar, double *E_bar, ebbx_stream stream);

/* Replace the material: per-tet E_tet_dev (nt FP64, borrowed and kept as the
 * E_t of ebbx_fem_E_grad) or uniform E; per-tet nu_tet_dev (nt FP64) or
 * uniform nu.  Enqueued on stream. */
ebbx_status ebbx_fem_set_material(ebbx_fem fem, const double *E_tet_dev, const double *nu_tet_dev, double E,
                                  double nu, ebbx_stream stream);

/* Vector-Jacobian product of one ebbx_implicit_step taken from (d_n, v_n) to
 * (d_{n+1}, v_{n+1}).  Given gx = dL/dd_{n+1} and gv = dL/dv_{n+1}:
 *   g^ = gv + dt gx;  solve A w = Pi g^ with the step's masked PCG
 *   (A = (1 + dt alpha) M - ck K(d_n), ck = dt^2 + dt beta, same params);
 *   d_bar = gx + dt K w + ck T[v_{n+1}, w]        (= dL/dd_n, overwritten)
 *   v_bar = g^ + ck K w - dt alpha M w            (= dL/dv_n, overwritten)
 *   E_bar[t] += w_t . (dt f_t + ck K_t v_{n+1}) / E_t   (nullable)
 * stats_dev (nullable) receives the adjoint solve's report.  Inputs must not
 * alias outputs (EBBX_E_PHASE). */
ebbx_status ebbx_implicit_step_vjp(ebbx_fem fem, const double *d_n, const double *v_np1,
                                   const ebbx_step_params *params, const double *gx, const double *gv,
                                   double *d_bar, double *v_bar, double *E_bar, ebbx_step_stats *stats_dev,
                                   ebbx_stream stream);

/* ---- batches of meshes ---------------------------------------------------- */

/* Many independent meshes in one set of relations (the relational model's
 * answer to batching: one `meshes` relation, key-fields tets.mesh and
 * verts.mesh into it).  Layout contract: verts and tets are sorted by mesh
 * id (non-decreasing), every tet's corners lie in the tet's mesh, and the
 * meshes relation holds FP64 fields E and nu (one value per mesh). */
typedef struct {
    const char *tet_verts;   /* key-field tets -> verts, arity 4 */
    const char *tet_mesh;    /* key-field tets -> meshes, arity 1 */
    const char *vert_mesh;   /* key-field verts -> meshes, arity 1 */
    const char *pos;         /* verts: FP64 x3 rest positions */
    const char *pinned;      /* verts: U8 x1 Dirichlet mask, nullable */
    const char *E;           /* meshes: FP64 x1 Young's modulus */
    const char *nu;          /* meshes: FP64 x1 Poisson ratio */
} ebbx_batch_fields;

/* Build the union domain of all meshes (model, element precision, rho,
 * strategy and block from params; params->E, nu ignored, E_field must be
 * NULL).  Synchronous.  EBBX_E_LAYOUT if the layout contract is broken,
 * EBBX_E_ARG for a mesh with E <= 0 or nu outside (-1, 0.5). */
ebbx_status ebbx_batch_create(ebbx_relation meshes, ebbx_relation tets, ebbx_relation verts,
                              const ebbx_batch_fields *fields, const ebbx_fem_params *params, ebbx_batch *out);
ebbx_status ebbx_batch_destroy(ebbx_batch batch);

/* The union domain (owned by the batch; ebbx_fem_destroy on it fails): the
 * element calls (forces, Kmul, diag, energy) act on every mesh at once. */
ebbx_status ebbx_batch_fem(ebbx_batch batch, ebbx_fem *out);

/* One implicit step (as ebbx_implicit_step) of every mesh, each with its
 * own CG scalars, stopping test and report: the meshes share every kernel
 * launch, and a mesh that has converged skips its share of the vector work.
 * per_mesh_dev: device array of nm ebbx_step_stats (nullable).  d and v are
 * FP64 (3, nv) over the union's vertices. */
ebbx_status ebbx_batch_implicit_step(ebbx_batch batch, double *d, double *v, const ebbx_step_params *params,
                                     ebbx_step_stats *per_mesh_dev, ebbx_stream stream);

/* Copy a device stats record to the host; synchronises the stream. */
ebbx_status ebbx_stats_fetch(const ebbx_step_stats *stats_dev, ebbx_step_stats *host,
                             ebbx_stream stream);

/* Stream `bytes` through a library-owned buffer to evict device caches
 * (including the memory-side Infinity Cache) before a cold measurement. */
ebbx_status ebbx_cache_flush(size_t bytes, ebbx_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* EBBX_H */
