// fem.h -- the tet-FEM domain object and the launchers of its kernels.
#pragma once

#include "internal.h"

struct ebbx_fem_s;

namespace ebbx {

enum ElemOp { OP_FORCE = 0, OP_KMUL = 1, OP_DIAG = 2 };

// Everything an element kernel reads; plain pointers, passed by value.
struct ElemArgs {
    int64_t nt, nv;
    const int32_t *keys;   // (4, nt) int32 key-field tets.v
    const void *B;         // (9, nt) element precision, B = Dm^-1 row-major
    const void *V0;        // (nt) element precision
    const void *mat;       // (2, nt) element precision (mu, lam) or NULL
    double mu, lam;        // uniform material when mat == NULL
    const double *d;       // (3, nv) displacement
    const double *u;       // (3, nv) direction (stiffness product)
    double *out;           // (3, nv) reduce target (atomic / block strategies)
    void *part;            // (nt, 12) element precision per-corner partials (segmented)
    unsigned long long *n_inv;  // inverted-element counter
    // block strategy
    const int32_t *blk_vptr;    // (nblk + 1) offsets into blk_verts
    const int32_t *blk_verts;   // global vertex ids per block, sorted
    const uint8_t *blk_own;     // 1 if every incident tet of that vertex is in the block
    const uint16_t *blk_local;  // (4, nt) local slot of each corner within its block
    const int *skip;            // nullable device flag: nonzero = return at once (converged solve)
};

// Launch the element map `op` with the FEM's current strategy; result into
// out (3, nv) (+= if accumulate).  For OP_DIAG, u is ignored and out receives
// the raw stiffness diagonal K[(v,c),(v,c)].
void elem_launch(ebbx_fem_s *F, ElemOp op, const double *d, const double *u, double *out, int accumulate,
                 hipStream_t s, const int *skip = nullptr);
// Total energy into out_dev[0].
void elem_energy(ebbx_fem_s *F, const double *d, double *out_dev, hipStream_t s);
// Rest-shape precompute; returns the number of degenerate tets.
int64_t elem_precompute(ebbx_fem_s *F, const double *X, const double *E_tet, hipStream_t s);
// Fill n doubles with a value (graph-safe, no memset node).
void fill_f64(double *p, int64_t n, double v, hipStream_t s);
// Build the tet-block tables of the BLOCK strategy.
void build_blocks(ebbx_fem_s *F, hipStream_t s);

}  // namespace ebbx

struct ebbx_fem_s {
    ebbx_relation_s *tets = nullptr, *verts = nullptr;
    std::string keyname;
    const int32_t *keys = nullptr;
    std::shared_ptr<ebbx::Grouping> group;
    int64_t nt = 0, nv = 0;
    int32_t model = EBBX_STVK, prec = EBBX_F64, strategy = EBBX_STRAT_ATOMIC, block = 256;
    double rho = 1000.0, E = 1e5, nu = 0.3, mu = 0.0, lam = 0.0;
    bool per_tet = false;
    size_t esize = 8;   // bytes of one element-precision value

    ebbx::DevBuf B, V0, mat, mass, pinned, part, status, scratch;
    // block strategy tables
    int32_t blk_tets = 0;      // tets per block
    int64_t nblk = 0;
    int32_t blk_maxv = 0;      // largest vertex count of one block
    int64_t blk_nverts = 0;    // entries of blk_verts (block lists, then isolated vertices)
    ebbx::DevBuf blk_vptr, blk_verts, blk_own, blk_local;
    bool blocks_built = false;

    // implicit-step state (allocated on first step)
    struct Step;
    std::unique_ptr<Step> step;
    ~ebbx_fem_s();
};
