// fem.h -- the tet-FEM domain object and the launchers of its kernels.
#pragma once

#include "internal.h"

struct ebbx_fem_s;

namespace ebbx {

enum ElemOp { OP_FORCE = 0, OP_KMUL = 1, OP_DIAG = 2, OP_TMUL = 3 };

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i on XCD i mod
// 8), each XCD with its own L2.  Give XCD x one contiguous range of tet blocks,
// so that neighbouring (Morton-adjacent) blocks, which share vertices, run under
// the same L2.  A bijection of [0, nblk).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblk) {
    const uint32_t q = nblk >> 3, r = nblk & 7u, x = b & 7u, i = b >> 3;
    return x * q + min(x, r) + i;
}

// The same with runs of 2^k consecutive blocks dealt to the XCDs in turn (k > 0),
// for a batch: there the blocks still working late in a solve are those of the
// few meshes that iterate longest, one contiguous stretch that a single range per
// XCD would leave to one XCD.  Blocks past the last whole round of 8 runs keep the
// contiguous mapping.  A bijection of [0, nblk).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblk, uint32_t k) {
    if (k == 0) return xcd_block(b, nblk);
    const uint32_t full = (nblk >> (k + 3)) << (k + 3);
    if (b >= full) return full + xcd_block(b - full, nblk - full);
    const uint32_t x = b & 7u, i = b >> 3;
    return ((((i >> k) << 3) + x) << k) + (i & ((1u << k) - 1u));
}

// The tet blocks of a batched solve still to evaluate, rebuilt from the meshes' finished flags
// at the start of every CG iteration: one range per unfinished mesh, in mesh order.  hdr[0] is
// the number of blocks, hdr[2] the number of unfinished meshes; range j covers list items
// [bpfx[j], bpfx[j+1]), the blocks bstart[j] + (i - bpfx[j]).  A block that two unfinished
// meshes share is listed once, in the first one's range.  Laid out as int32 [4 | nm + 1 | nm].
struct ActList {
    const int32_t *hdr, *bpfx, *bstart;
};
__host__ __device__ inline ActList act_list(const int32_t *p, int32_t nm) {
    return ActList{p, p + 4, p + 4 + (nm + 1)};
}
inline size_t act_list_ints(int64_t nm) { return (size_t)(4 + (nm + 1) + nm); }

// Everything an element kernel reads; plain pointers, passed by value.  Column
// stores are passed as one base pointer per component, so that a kernel
// addresses every column of a row with one 32-bit byte offset.
struct ElemArgs {
    uint32_t nt, nv;
    const int32_t *key[4];      // columns of the key-field tets.v
    const void *B[9];           // columns of B = Dm^-1 (row-major entries), element precision
    const void *V0;             // (nt) element precision
    const void *mu_t, *lam_t;   // per-tet Lame parameters (element precision) or NULL
    double mu, lam;             // uniform material when mu_t == NULL
    const double *X[3];         // rest positions (library copy), for B recomputed per block
    const double *d[3];         // displacement columns
    const double *u[3];         // direction columns (stiffness product; `a` of T[a, w])
    const double *w[3];         // second direction columns (`w` of T[a, w])
    double *out[3];             // reduce target columns
    void *part;                 // (nt, 12) per-corner partials (segmented reduction)
    unsigned long long *n_inv;  // inverted-element counters (one per mesh)
    const int32_t *tmesh;       // per-tet mesh ids selecting the counter, or NULL (one mesh)
    // block strategy
    // block tables at a fixed stride of blk_stride vertices per block (padded with vertex -1)
    const int32_t *blk_verts;   // global vertex ids of each block, sorted
    const uint16_t *blk_row;    // per block, blk_stride + 1 entries: vertex i's rows are [row[i], row[i+1])
    const uint32_t *blk_pos[2]; // per tet: rows of corners (0,1) and (2,3) within its block, 16 bits each
    const int32_t *blk_hpos;    // per block vertex: halo position, or -1 if the block owns it
    uint32_t blk_stride;
    const uint32_t *slot[2];    // packed corner slots within the block (one or two words per tet)
    double *halo;               // partial sums of shared vertices, 3 per entry, block-major
    const float *xf[3];         // FP32 elements, blocks of <= 256 vertices: block-local rest positions
                                // (stride blk_stride per block), or NULL
    uint32_t nblk;              // tet blocks
    // PIPE strategy
    const uint32_t *blk_run;    // per block vertex (stride blk_stride): run start | run end << 11 | acc index << 22
    const int32_t *sb_verts;    // per super-block (stride sb_stride): its vertices, -1 padded
    const int32_t *sb_hpos;     // per super-block vertex: halo position, or -1 if the super-block owns it
    uint32_t sb_g, nsb, sb_stride, stage_stride;
    uint32_t xcd_run_log2;      // 0: one contiguous range of blocks per XCD; k > 0: runs of 2^k
                                // consecutive blocks dealt to the XCDs in turn
    // owner strategy: block b owns vertices [b*own_vb, (b+1)*own_vb) and evaluates every
    // tet incident to them (tets on a block boundary are evaluated by each block they touch)
    const int32_t *own_tptr;    // (nblk + 1) offsets into own_meta
    const uint4 *own_meta;      // per (block, tet): tet id, then 4 x (11-bit slot | 13-bit sum position)
    const int32_t *own_gptr;    // (nblk + 1) offsets into own_ghost
    const int32_t *own_ghost;   // staged vertices not owned by the block, ascending
    const int64_t *rp;          // grouping row offsets (incidences of each vertex in (tet, corner) order)
    uint32_t own_vb, own_nblk;
    int accumulate;             // 1: out += result
    const int *skip;            // nullable device flag: nonzero = return at once (converged solve)
    const int *mdone;           // nullable per-mesh finished flags (batch): a block whose meshes are
                                // all finished returns at once (block strategies)
    const int32_t *act;         // nullable: the active list of a batched solve (k_block_list)
    int32_t act_nm;             // meshes of that batch (the list's array stride)
    // the fused step preamble (k_block_pre): f, K u and the stiffness diagonal, each into three
    // columns; shared vertices' partials go to halo9, 9 per entry (f, then K u, then diagonal)
    double *pre_out[3][3];
    double *halo9;
};

// Launch the element map `op` with the FEM's current strategy; result into
// out (3, nv) (+= if accumulate).  For OP_DIAG, u is ignored and out receives
// the raw stiffness diagonal K[(v,c),(v,c)].
// finish_halo = false (block strategies) leaves the shared vertices' sums in the
// halo for a consumer that reads them through elem_halo_view.  scratch (nullable): a
// device buffer of at least elem_scratch_bytes(F, op) bytes used in place of the
// domain's own halo (block strategies) or per-corner partials (SEG) for this call.
void elem_launch(ebbx_fem_s *F, ElemOp op, const double *d, const double *u, double *out, int accumulate,
                 hipStream_t s, const int *skip = nullptr, const double *w = nullptr, const int *mdone = nullptr,
                 bool finish_halo = true, void *scratch = nullptr, const int32_t *act = nullptr);
// Whether the element map `op` of F's strategy can run over an active list (act of
// elem_launch, batches only): the stiffness product of the BLOCK strategy, one tet per thread.
bool elem_list_ok(const ebbx_fem_s *F, ElemOp op);
// Device scratch one element map of the current strategy writes and reads besides its
// inputs, outputs and the domain's tables (0 for ATOMIC and OWNER).
size_t elem_scratch_bytes(const ebbx_fem_s *F, ElemOp op);

// The unfinished output of a block-strategy element map: vertex v's value is
// out[v] when row[v] < 0, else the sum of its halo entries (row r of the
// shared-vertex table, positions in block order; nc int4 chunks per row, or
// the CSR form ptr/pos when nc = 0).  row == NULL: nothing to finish.
struct HaloView {
    const int32_t *row;
    const int4 *tab;
    const int32_t *ptr, *pos;
    const double *halo;
    int nc;
};
HaloView elem_halo_view(const ebbx_fem_s *F);
// E_bar[t] += w_t . (cf f_t(d) + ck K_t(d) v) / E_t over the tets (no scatter; v unused if ck = 0).
void elem_egrad(ebbx_fem_s *F, const double *d, const double *v, const double *w, double cf, double ck,
                double *E_bar, hipStream_t s);
// Recompute the per-tet Lame parameters from per-tet (or uniform) E and nu.
void elem_set_material(ebbx_fem_s *F, const double *E_tet, const double *nu_tet, double E, double nu, hipStream_t s);
// The implicit step's three element maps at the state d in one pass of the block strategy
// (BLOCK, one tet per thread, incidence-order sums; elem_pre_ok): f(d) into f, K(d) u into y and
// the raw stiffness diagonal into diag, with the same per-tet arithmetic and summation order as
// the three separate maps.  Shared vertices stay in the 9-wide halo of elem_pre_halo for the
// consumer (elem_pre_prepare allocates it; call it outside stream capture).
bool elem_pre_ok(const ebbx_fem_s *F);
void elem_pre_prepare(ebbx_fem_s *F, hipStream_t s);
void elem_launch_pre(ebbx_fem_s *F, const double *d, const double *u, double *f, double *y, double *diag,
                     hipStream_t s);
HaloView elem_pre_halo(const ebbx_fem_s *F);
// Total energy into out_dev[0].
void elem_energy(ebbx_fem_s *F, const double *d, double *out_dev, hipStream_t s);
// Rest-shape precompute; returns the number of degenerate tets.
int64_t elem_precompute(ebbx_fem_s *F, const double *X, const double *E_tet, hipStream_t s);
// Fill n doubles with a value (graph-safe, no memset node).
void fill_f64(double *p, int64_t n, double v, hipStream_t s);
// Host form of the tet-block tables (blocks of bt consecutive tets): per block its
// sorted vertex list (CSR vptr/verts), each list entry's run of incidence rows
// (global running starts lptr), whether the block holds every incident tet of the
// entry's vertex (own), and per tet its corners' rows (pos, two 16-bit pairs) and
// slots (packed, w words).
struct HostBlocks {
    int32_t bt = 0, maxv = 0, w = 1;
    int64_t nblk = 0;
    std::vector<int32_t> vptr, verts, lptr;
    std::vector<uint8_t> own;
    std::vector<uint32_t> pos, packed;
};
HostBlocks host_blocks(const std::vector<int32_t> &keys, const std::vector<int64_t> &rp, int64_t nt, int32_t bt);
void download_keys(const ebbx_fem_s *F, std::vector<int32_t> &keys, std::vector<int64_t> &rp);
void upload(DevBuf &dst, const void *src, size_t bytes, hipStream_t s);
// Shared-vertex tables and halo buffer for units (blocks or super-blocks) whose vertex
// lists, in unit order, are verts (own: the unit holds every incident tet).
void build_halo(ebbx_fem_s *F, const std::vector<int32_t> &verts, const std::vector<uint8_t> &own,
                const std::vector<int64_t> &rp, std::vector<int32_t> &hpos, hipStream_t s);
void upload_block_tables(ebbx_fem_s *F, const HostBlocks &hb, const std::vector<int32_t> &hpos, hipStream_t s);
// Build the tet-block tables of the BLOCK strategy.
void build_blocks(ebbx_fem_s *F, int32_t tets_per_block, hipStream_t s);
// Build the super-block tables of the PIPE strategy (blocks of 256 tets, g blocks per
// super-block) and its halo.
void build_pipe(ebbx_fem_s *F, int32_t g, hipStream_t s);
// Launch the PIPE element kernel (pipe.hip); the halo pass is launched by the caller.
void launch_pipe(ebbx_fem_s *F, ElemOp op, const ElemArgs &a, hipStream_t s);
size_t pipe_shmem(const ebbx_fem_s *F, ElemOp op);
// The stiffness product of the LANES strategy (lanes.hip): four lanes per tet over the BLOCK
// tables; the halo pass is launched by the caller.
void launch_lanes(ebbx_fem_s *F, const ElemArgs &a, hipStream_t s);
size_t lanes_shmem(const ebbx_fem_s *F);
// Build the vertex-owned block tables of the OWNER strategy.
void build_owner(ebbx_fem_s *F, int32_t verts_per_block, hipStream_t s);
// Assembled stiffness on edges (assemble.hip): the edges relation (once per
// domain, synchronous), K(d) into the edge blocks, y (+)= K u over them, and
// copies of the relation and the blocks (FP64) into caller buffers.
void build_edges(ebbx_fem_s *F, hipStream_t s);
void assemble_stiffness(ebbx_fem_s *F, const double *d, hipStream_t s);
void assembled_spmv(ebbx_fem_s *F, const double *u, double *y, int accumulate, hipStream_t s);
void edges_copy(ebbx_fem_s *F, int32_t *row, int32_t *col, double *blocks, hipStream_t s);

// FEM handle registry (fem.hip).
ebbx_fem_s *check_fem(ebbx_fem f);
void fem_register(ebbx_fem_s *F);
void fem_unregister(ebbx_fem_s *F);
// Validate and build a FEM domain (synchronous); E_tet: per-tet modulus or NULL.
std::unique_ptr<ebbx_fem_s> fem_build(ebbx_relation_s *tr, const char *keyfield, ebbx_relation_s *vr,
                                      const char *pos_field, const char *pinned_field, const ebbx_fem_params &p,
                                      const double *E_tet);
// Select the scatter strategy and block size (builds block tables as needed).
void set_strategy(ebbx_fem_s *F, int32_t strategy, int32_t block, hipStream_t s);
// Drop the captured solver graphs (solve.hip); they bake in kernel arguments.
void step_drop_graphs(ebbx_fem_s *F);

inline bool overlap(const void *a, const void *b, size_t bytes) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

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
    const double *E_tet = nullptr;   // borrowed per-tet Young's modulus (nullable)
    // meshes of a batch: vertex ranges [mesh_vptr[m], mesh_vptr[m+1]); one mesh otherwise
    int64_t nm = 1;
    std::vector<int64_t> mesh_vptr;
    std::vector<int64_t> mesh_tptr;   // batches: tet ranges [mesh_tptr[m], mesh_tptr[m+1])
    const int32_t *tmesh = nullptr;  // per-tet mesh ids (batch) or NULL
    bool batch_owned = false;        // the union domain of a batch: destroyed with it
    size_t esize = 8;   // bytes of one element-precision value

    ebbx::DevBuf B, V0, mat, mass, pinned, part, status, scratch, Xc;
    // block strategy tables
    int32_t blk_tets = 0;      // tets per block
    int32_t blk_tpt = 1;       // tets per thread (block kernels run blk_tets / blk_tpt threads)
    int64_t nblk = 0;
    int32_t blk_maxv = 0;      // largest vertex count of one block
    int32_t blk_w = 1;         // 32-bit words of packed corner slots per tet
    int32_t blk_red = 0;       // 0: incidence-list sums (deterministic), 1: FP64 LDS atomics
    int64_t blk_nverts = 0;    // entries of blk_verts over all blocks
    int64_t sh_n = 0;          // vertices summed from the halo (shared or untouched)
    int64_t halo_n = 0;        // halo entries
    ebbx::DevBuf blk_xf;   // block-local FP32 rest positions (FP32 elements, blocks of <= 256 vertices)
    ebbx::DevBuf blk_vptr, blk_verts, blk_lptr, blk_pos, blk_hpos, blk_local, halo, sh_vert, sh_ptr, sh_pos, sh_tab,
        sh_row;
    ebbx::DevBuf halo9;        // the fused step preamble's halo (9 values per entry)
    int32_t sh_nc = 0;         // int4 chunks per row of sh_tab (0: use the CSR form)
    bool blocks_built = false;
    int32_t halo_level = -1;   // the halo and shared-vertex tables are of: 0 blocks, g >= 1 super-blocks of
                               // g blocks (PIPE), -1 none
    // PIPE strategy: super-blocks of pipe_g consecutive 256-tet blocks
    int32_t pipe_g = 0;
    int64_t nsb = 0;
    int32_t sb_maxv = 0;       // largest vertex count of one super-block (table stride)
    int32_t stage_stride = 0;  // staged vertices per block in LDS (128 or 256)
    ebbx::DevBuf blk_run, sb_verts, sb_hpos;
    // owner strategy tables
    int32_t own_vb = 0;        // owned vertices per block
    int64_t own_nblk = 0;
    int32_t own_maxv = 0;      // most staged vertices (owned + ghosts) of one block
    int32_t own_maxinc = 0;    // most owned incidences of one block
    int64_t own_ntb = 0;       // (block, tet) pairs over all blocks
    ebbx::DevBuf own_tptr, own_meta, own_gptr, own_ghost;
    // assembled stiffness: directed edges grouped by tail (built on first use)
    int64_t n_edges = -1;      // -1: not built
    bool assembled = false;    // e_blocks holds K(d) of an ebbx_fem_assemble call
    ebbx::DevBuf e_row, e_col, e_gptr, e_gent, e_blocks, e_ke;

    // implicit-step state (allocated on first step)
    struct Step;
    std::unique_ptr<Step> step;
    ebbx_fem_s();   // both defined where Step is complete (solve.hip)
    ~ebbx_fem_s();
};
