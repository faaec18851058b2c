// assemble.hip -- the stiffness matrix stored on the mesh edges.
//
// The Vega workload keeps its stiffness on the edges of the tet mesh, one 3x3
// block per pair of vertices that share a tet (Developing Domain Libraries,
// "Example: FEM tetmesh"; Performance Evaluation).  Here the edges relation
// holds every ordered pair (i, j), i == j included, grouped by the tail i and
// sorted by the head j, so that the blocks form a block-CSR matrix and K u is
// a sparse product instead of the matrix-free element map.
//
//  - k_elem_matrix: one thread per tet computes the tet's 12 x 12 stiffness in
//    FP64, column by column (a unit displacement of corner b along axis k gives
//    dF = e_k (x) grad N_b), with the element maps' own dP, and writes its
//    sixteen 3x3 corner blocks, rounded to the element precision, to a per-tet
//    record (the same rounding as the matrix-free map's per-tet corner results,
//    which are also summed in FP64), one block column at a time through LDS so
//    that the workgroup writes each tet's four blocks of that column (36
//    contiguous values) together (per-thread scattered stores of the record
//    wrote 2.45x its bytes);
//  - k_edge_gather: one thread per edge sums the corner blocks of the tets
//    holding both of its vertices in ascending tet order (deterministic) and
//    stores the edge block at the element precision, nine columns (SoA);
//  - k_bsr_spmv: sixteen lanes per vertex row; each lane takes edges of the row
//    (consecutive lanes read consecutive entries of each column) and the row
//    sum is a fixed butterfly over the sixteen lanes.
#include <algorithm>
#include <vector>

#include "fem.h"
#include "tetmath.h"

namespace ebbx {

namespace {

constexpr int SPMV_LANES = 16;

struct AsmArgs {
    uint32_t nt;
    const int32_t *key[4];
    const void *B[9];
    const void *mu_t, *lam_t;
    double mu, lam;
    const double *d[3];
    void *ke;                    // (nt, 16, 9) at the element precision: block (a, b) of tet t at
                                 // ke[(16 t + 4 b + a) * 9]
    unsigned long long *n_inv;
    const int32_t *tmesh;
};

constexpr int EM_THREADS = 128;   // tets per workgroup of the element-matrix kernel
constexpr int EM_STRIDE = 37;     // LDS doubles per tet for one block column (36, padded)

// Per-tet record: 144 values at the element precision, block (a, b) (rows of corner a, columns
// of corner b) at (4 b + a) * 9, row-major; so the four blocks of one column b are 36
// contiguous values.
template <class T, int MODEL>
__global__ __launch_bounds__(EM_THREADS) void k_elem_matrix(AsmArgs a) {
    __shared__ double s_col[EM_THREADS * EM_STRIDE];
    const uint32_t t0 = blockIdx.x * EM_THREADS, t = t0 + threadIdx.x;
    const bool in = t < a.nt;
    const uint32_t nloc = min((uint32_t)EM_THREADS, a.nt - t0);   // tets of this workgroup
    double b[9], G[9], gb[4][3], V0 = 1.0, mu = 0.0, lam = 0.0;
    if (in) {
#pragma unroll
        for (int k = 0; k < 9; ++k) b[k] = (double)ldc<T>(a.B[k], t);
        V0 = tet_V0(b);
        mu = a.mu_t ? (double)ldc<T>(a.mu_t, t) : a.mu;
        lam = a.lam_t ? (double)ldc<T>(a.lam_t, t) : a.lam;
        double qd[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t v = (uint32_t)a.key[c][t];
#pragma unroll
            for (int k = 0; k < 3; ++k) qd[c][k] = a.d[k][v];
        }
        grad_from(qd, b, G);
        // grad N_b: rows of B for corners 1..3, minus their sum for corner 0
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gb[1][j] = b[j];
            gb[2][j] = b[3 + j];
            gb[3][j] = b[6 + j];
            gb[0][j] = -(b[j] + b[3 + j] + b[6 + j]);
        }
    }
    bool ok = true;
    // one block column at a time: every tet's 36 values go through LDS, then the workgroup
    // writes each tet's 288 contiguous bytes of that column together
    for (int cb = 0; cb < 4; ++cb) {
        if (in) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double dF[9], dP[9], h[12];
#pragma unroll
                for (int q = 0; q < 9; ++q) dF[q] = 0.0;
                dF[3 * k] = gb[cb][0];
                dF[3 * k + 1] = gb[cb][1];
                dF[3 * k + 2] = gb[cb][2];
                ok = dstress_scaled<double, MODEL>(mu, lam, V0, G, dF, dP) && ok;
                corner_out(dP, b, h);   // h[3 a + r] = df_{a,r} / dd_{cb,k}
#pragma unroll
                for (int ca = 0; ca < 4; ++ca)
#pragma unroll
                    for (int r = 0; r < 3; ++r) s_col[threadIdx.x * EM_STRIDE + ca * 9 + 3 * r + k] = h[3 * ca + r];
            }
        }
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < nloc * 36u; e += EM_THREADS) {
            const uint32_t i = e / 36u, o = e - 36u * i;
            ((T *)a.ke)[(size_t)(t0 + i) * 144 + 36u * cb + o] = (T)s_col[i * EM_STRIDE + o];
        }
        __syncthreads();
    }
    if (MODEL == EBBX_NH && in && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
}

// blocks[q][e] = sum over the edge's (tet, a, b) entries, in tet order, of ke block q
template <class T>
__global__ __launch_bounds__(256) void k_edge_gather(const T *ke, const int32_t *gptr, const uint32_t *gent,
                                                     uint32_t ne, T *blocks) {
    // XCD x sums one contiguous range of edges (tails in mesh order), so the records of a tet,
    // which its four corners' edges all read, come into one L2 rather than up to four
    const uint32_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = 0.0;
    const int32_t j0 = gptr[e], j1 = gptr[e + 1];
    for (int32_t j = j0; j < j1; ++j) {
        const uint32_t c = gent[j];   // 16 t + 4 a + b: block (a, b) of tet t
        const T *blk = ke + (size_t)(c >> 4) * 144 + (4u * (c & 3u) + ((c >> 2) & 3u)) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) s[q] += (double)blk[q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) blocks[(size_t)q * ne + e] = (T)s[q];
}

template <class T> struct BsrArgs {
    const int32_t *row, *col;
    const T *k[9];
    const double *u[3];
    double *y[3];
    uint32_t nv;
    int accumulate;
};

template <class T>
__global__ __launch_bounds__(256) void k_bsr_spmv(BsrArgs<T> a) {
    // XCD x takes one contiguous range of rows, whose neighbours' u it shares in its L2
    const uint32_t g = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / SPMV_LANES;
    const uint32_t lane = threadIdx.x % SPMV_LANES;
    const uint32_t i = g < a.nv ? g : a.nv - 1;   // whole groups stay in the shuffles
    const int32_t e0 = a.row[i], e1 = g < a.nv ? a.row[i + 1] : e0;
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int32_t e = e0 + (int32_t)lane; e < e1; e += SPMV_LANES) {
        const uint32_t j = (uint32_t)a.col[e];
        const double u0 = a.u[0][j], u1 = a.u[1][j], u2 = a.u[2][j];
        y0 += (double)a.k[0][e] * u0 + (double)a.k[1][e] * u1 + (double)a.k[2][e] * u2;
        y1 += (double)a.k[3][e] * u0 + (double)a.k[4][e] * u1 + (double)a.k[5][e] * u2;
        y2 += (double)a.k[6][e] * u0 + (double)a.k[7][e] * u1 + (double)a.k[8][e] * u2;
    }
#pragma unroll
    for (int m = SPMV_LANES / 2; m >= 1; m >>= 1) {
        y0 += __shfl_xor(y0, m, SPMV_LANES);
        y1 += __shfl_xor(y1, m, SPMV_LANES);
        y2 += __shfl_xor(y2, m, SPMV_LANES);
    }
    if (lane == 0 && g < a.nv) {
        if (a.accumulate) {
            y0 += a.y[0][i];
            y1 += a.y[1][i];
            y2 += a.y[2][i];
        }
        a.y[0][i] = y0;
        a.y[1][i] = y1;
        a.y[2][i] = y2;
    }
}

unsigned grid_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Edges relation and gather lists, from the grouping (vertex -> (tet, corner)
// incidences in tet order).  Host side, once per domain.
void build_edges(ebbx_fem_s *F, hipStream_t s) {
    if (F->n_edges >= 0) return;
    const int64_t nt = F->nt, nv = F->nv;
    if (nt >= (int64_t(1) << 28)) fail(EBBX_E_ARG, "assembled stiffness: at most 2^28 tets");
    std::vector<int32_t> keys((size_t)(4 * nt));
    if (nt > 0) HIPCHK(hipMemcpy(keys.data(), F->keys, keys.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> rp((size_t)(nv + 1));
    HIPCHK(hipMemcpy(rp.data(), F->group->row_ptr.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> inc((size_t)std::max<int64_t>(4 * nt, 1));
    if (nt > 0) HIPCHK(hipMemcpy(inc.data(), F->group->inc.get(), (size_t)(4 * nt) * sizeof(int32_t),
                                 hipMemcpyDeviceToHost));
    std::vector<int32_t> row((size_t)(nv + 1), 0), col, gptr(1, 0);
    std::vector<uint32_t> gent;
    col.reserve((size_t)(16 * nv + 16));
    gent.reserve((size_t)(16 * nt));
    struct Ent {
        int32_t j;
        uint32_t code;   // 16 t + 4 a + b
    };
    std::vector<Ent> buf;
    for (int64_t i = 0; i < nv; ++i) {
        buf.clear();
        for (int64_t p = rp[(size_t)i]; p < rp[(size_t)i + 1]; ++p) {
            const uint32_t t = (uint32_t)inc[(size_t)p] >> 2, ca = (uint32_t)inc[(size_t)p] & 3u;
            for (uint32_t cb = 0; cb < 4; ++cb)
                buf.push_back({keys[(size_t)cb * nt + t], 16u * t + 4u * ca + cb});
        }
        std::sort(buf.begin(), buf.end(), [](const Ent &x, const Ent &y) {
            return x.j != y.j ? x.j < y.j : x.code < y.code;
        });
        for (size_t k = 0; k < buf.size(); ++k) {
            if (k == 0 || buf[k].j != buf[k - 1].j) {
                if (k > 0) gptr.push_back((int32_t)gent.size());
                col.push_back(buf[k].j);
            }
            gent.push_back(buf[k].code);
        }
        if (!buf.empty()) gptr.push_back((int32_t)gent.size());
        row[(size_t)i + 1] = (int32_t)col.size();
    }
    if (col.size() >= (size_t)(1u << 31)) fail(EBBX_E_ARG, "assembled stiffness: too many edges");
    F->n_edges = (int64_t)col.size();
    auto up = [&](DevBuf &dst, const void *src, size_t bytes) {
        dst.reset(std::max<size_t>(bytes, 8), s);
        if (bytes) HIPCHK(hipMemcpy(dst.get(), src, bytes, hipMemcpyHostToDevice));
    };
    up(F->e_row, row.data(), row.size() * sizeof(int32_t));
    up(F->e_col, col.data(), col.size() * sizeof(int32_t));
    up(F->e_gptr, gptr.data(), gptr.size() * sizeof(int32_t));
    up(F->e_gent, gent.data(), gent.size() * sizeof(uint32_t));
}

namespace {

template <class T> void launch_assemble(ebbx_fem_s *F, const double *d, hipStream_t s) {
    const int64_t nt = F->nt, nv = F->nv;
    const size_t es = sizeof(T);
    if (nt > 0) {
        AsmArgs a{};
        a.nt = (uint32_t)nt;
        for (int c = 0; c < 4; ++c) a.key[c] = F->keys + (size_t)c * nt;
        for (int k = 0; k < 9; ++k) a.B[k] = (const char *)F->B.get() + (size_t)k * nt * es;
        if (F->per_tet) {
            a.mu_t = F->mat.get();
            a.lam_t = (const char *)F->mat.get() + (size_t)nt * es;
        }
        a.mu = F->mu;
        a.lam = F->lam;
        for (int k = 0; k < 3; ++k) a.d[k] = d + (size_t)k * nv;
        a.ke = F->e_ke.get();
        a.n_inv = F->status.as<unsigned long long>();
        a.tmesh = F->tmesh;
        if (F->model == EBBX_STVK)
            hipLaunchKernelGGL((k_elem_matrix<T, EBBX_STVK>), dim3(grid_of(nt, EM_THREADS)), dim3(EM_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL((k_elem_matrix<T, EBBX_NH>), dim3(grid_of(nt, EM_THREADS)), dim3(EM_THREADS), 0, s, a);
        HIPCHK(hipGetLastError());
    }
    const int64_t ne = F->n_edges;
    if (ne > 0) {
        hipLaunchKernelGGL((k_edge_gather<T>), dim3(grid_of(ne, 256)), dim3(256), 0, s,
                           (const T *)F->e_ke.get(), F->e_gptr.as<int32_t>(), F->e_gent.as<uint32_t>(),
                           (uint32_t)ne, F->e_blocks.as<T>());
        HIPCHK(hipGetLastError());
    }
}

template <class T> void launch_spmv(ebbx_fem_s *F, const double *u, double *y, int accumulate, hipStream_t s) {
    const int64_t nv = F->nv, ne = F->n_edges;
    BsrArgs<T> a{};
    a.row = F->e_row.as<int32_t>();
    a.col = F->e_col.as<int32_t>();
    for (int q = 0; q < 9; ++q) a.k[q] = F->e_blocks.as<T>() + (size_t)q * ne;
    for (int k = 0; k < 3; ++k) {
        a.u[k] = u + (size_t)k * nv;
        a.y[k] = y + (size_t)k * nv;
    }
    a.nv = (uint32_t)nv;
    a.accumulate = accumulate;
    hipLaunchKernelGGL((k_bsr_spmv<T>), dim3(grid_of(nv * SPMV_LANES, 256)), dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
}

}  // namespace

void assemble_stiffness(ebbx_fem_s *F, const double *d, hipStream_t s) {
    build_edges(F, s);
    // the blocks and the per-tet scratch, on the first assembly
    const size_t blk_bytes = std::max<size_t>((size_t)9 * F->n_edges * F->esize, 8);
    const size_t ke_bytes = std::max<size_t>((size_t)F->nt * 144 * F->esize, 8);
    if (F->e_blocks.bytes() != blk_bytes) F->e_blocks.reset(blk_bytes, s);
    if (F->e_ke.bytes() != ke_bytes) F->e_ke.reset(ke_bytes, s);
    if (F->prec == EBBX_F32) launch_assemble<float>(F, d, s);
    else launch_assemble<double>(F, d, s);
    F->assembled = true;
}

void assembled_spmv(ebbx_fem_s *F, const double *u, double *y, int accumulate, hipStream_t s) {
    if (!F->assembled) fail(EBBX_E_STATE, "no assembled stiffness: call ebbx_fem_assemble first");
    if (F->nv == 0) return;
    if (F->prec == EBBX_F32) launch_spmv<float>(F, u, y, accumulate, s);
    else launch_spmv<double>(F, u, y, accumulate, s);
}

// Copies of the edges relation and the blocks (FP64) for inspection.
namespace {
template <class T>
__global__ void k_blocks_f64(const T *src, int64_t n, double *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}
}  // namespace

void edges_copy(ebbx_fem_s *F, int32_t *row, int32_t *col, double *blocks, hipStream_t s) {
    build_edges(F, s);
    const int64_t ne = F->n_edges, nv = F->nv;
    if (row) HIPCHK(hipMemcpyAsync(row, F->e_row.get(), (size_t)(nv + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (col && ne > 0) HIPCHK(hipMemcpyAsync(col, F->e_col.get(), (size_t)ne * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (blocks && ne > 0) {
        if (!F->assembled) fail(EBBX_E_STATE, "no assembled stiffness: call ebbx_fem_assemble first");
        const unsigned g = (unsigned)std::min<int64_t>(grid_of(9 * ne, 256), 1 << 16);
        if (F->prec == EBBX_F32)
            hipLaunchKernelGGL((k_blocks_f64<float>), dim3(g), dim3(256), 0, s, F->e_blocks.as<float>(), 9 * ne, blocks);
        else
            hipLaunchKernelGGL((k_blocks_f64<double>), dim3(g), dim3(256), 0, s, F->e_blocks.as<double>(), 9 * ne,
                               blocks);
        HIPCHK(hipGetLastError());
    }
}

}  // namespace ebbx

// ---- C ABI --------------------------------------------------------------------------

using namespace ebbx;

extern "C" ebbx_status ebbx_fem_assemble(ebbx_fem fem, const double *d, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (F->nv > 0 && !d) fail(EBBX_E_ARG, "d is NULL");
    assemble_stiffness(F, d, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_spmv(ebbx_fem fem, const double *u, double *y, int32_t accumulate,
                                     ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    const int64_t nv = F->nv;
    if (nv > 0 && (!u || !y)) fail(EBBX_E_ARG, "u or y is NULL");
    if (nv > 0 && overlap(u, y, (size_t)(3 * nv) * sizeof(double))) fail(EBBX_E_PHASE, "y aliases u");
    assembled_spmv(F, u, y, accumulate, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_edge_count(ebbx_fem fem, int64_t *n_edges) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (!n_edges) fail(EBBX_E_ARG, "n_edges is NULL");
    build_edges(F, nullptr);
    *n_edges = F->n_edges;
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_edges_get(ebbx_fem fem, int32_t *row_ptr, int32_t *col, double *blocks,
                                          ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    edges_copy(F, row_ptr, col, blocks, (hipStream_t)stream);
    EBBX_API_END
}
