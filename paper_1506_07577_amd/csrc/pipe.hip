// pipe.hip -- the element-parallel map over super-blocks of tet blocks, with the next
// block's vertex fields streamed into LDS while the current block is evaluated.
//
// The PIPE strategy keeps the BLOCK strategy's per-block work (a block of 256
// consecutive, Morton-ordered tets; its vertices' fields staged in LDS; each tet writes
// its corners to the rows of the block's incidence order; each block vertex sums its
// contiguous run of rows in FP64, in a fixed order) and changes two things:
//  - one workgroup walks a super-block of g consecutive blocks.  While it evaluates
//    block i, the gfx950 global-to-LDS loads bring block i+1's vertex fields (displacement,
//    direction(s), rest positions) into the other half of a double buffer: the loads hold
//    no registers, and the vertex gathers of the next block overlap the element math of
//    the current one instead of every workgroup alternating between the two;
//  - each block vertex's run sum is added to an FP64 accumulator of the super-block in
//    LDS (in block order), so only the vertices shared between super-blocks, not between
//    blocks, go through the halo: the super-block stores the vertices whose incident tets
//    it holds and writes one partial per shared vertex, which the halo pass sums in
//    super-block order.
// Every sum has a fixed order, so results are bitwise reproducible run to run.
#include <algorithm>
#include <vector>

#include "fem.h"
#include "tetmath.h"

namespace ebbx {

namespace {

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

constexpr int PB = 256;   // tets per block = threads per workgroup

// Vertex ids for the staging of block b: thread (wave wv, lane l) covers block-vertex
// entries wv*32 + 128 r + l/2 (r < nr), two lanes per entry; -1 past the block's list.
__device__ __forceinline__ void stage_ids(const ElemArgs &a, uint32_t b, uint32_t nr, int32_t (&vid)[2]) {
    const uint32_t S = a.blk_stride;
    const uint32_t e = (threadIdx.x >> 6) * 32u + ((threadIdx.x & 63u) >> 1);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t er = e + 128u * r;
        vid[r] = ((uint32_t)r < nr && er < S) ? ldc<int32_t>(a.blk_verts, b * S + er) : -1;
    }
}

// Stage the NC vertex columns `col` of one block into LDS columns of SP doubles at dst
// with global-to-LDS dword loads: lane l of wave wv loads dword (l & 1) of entry
// wv*32 + 128 r + l/2, so each wave instruction fills 256 contiguous bytes of one column.
// Entries past the block's list load vertex 0 (in bounds) into padding that no tet reads.
template <int NC>
__device__ __forceinline__ void stage_dma(const double *const (&col)[NC], double *dst, uint32_t SP, uint32_t nr,
                                          const int32_t (&vid)[2]) {
    const uint32_t hw = (threadIdx.x & 1u) * 4u, e0 = (threadIdx.x >> 6) * 32u;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if ((uint32_t)r >= nr) break;
        const uint32_t off = (uint32_t)max(vid[r], 0) * 8u + hw;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            __builtin_amdgcn_global_load_lds((gbl_void_t *)((const char *)col[c] + off),
                                             (lds_void_t *)(dst + c * SP + e0 + 128u * r), 4, 0, 0);
    }
}

template <class T, int MODEL, int OP>
__global__ __launch_bounds__(PB) void k_pipe(ElemArgs a) {
    extern __shared__ uint4 s_dyn4[];
    if (a.skip && *a.skip) return;   // uniform over the grid
    constexpr int NQ = OP == OP_TMUL ? 3 : OP == OP_KMUL ? 2 : 1;   // staged vertex fields
    constexpr int NC = 3 * NQ + 3;                                 // their columns, then the rest positions
    constexpr uint32_t LB = 4 * PB;                                // rows of one component column
    const uint32_t tid = threadIdx.x, nt = a.nt, S = a.blk_stride, SP = a.stage_stride, SV = a.sb_stride;
    const uint32_t nr = SP >> 7;
    const uint32_t sb = xcd_block(blockIdx.x, a.nsb, a.xcd_run_log2);
    const uint32_t b0 = sb * a.sb_g, nb = min(a.sb_g, a.nblk - b0);
    if (a.mdone) {   // a batch: skip the super-block once every mesh it touches has finished (uniform)
        const int32_t m0 = a.tmesh[b0 * PB], m1 = a.tmesh[min((b0 + nb) * PB, nt) - 1];
        bool all = true;
        for (int32_t m = m0; m <= m1; ++m) all = all && a.mdone[m] != 0;
        if (all) return;
    }
    double *stage = (double *)s_dyn4;                     // two buffers of NC columns of SP entries
    T *rows = (T *)(stage + 2 * NC * SP);                  // three columns of LB rows
    double *acc = (double *)(rows + 3 * LB);               // three columns of SV super-block vertices
    const double *col[NC];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        col[k] = a.d[k];
        if (NQ > 1) col[3 + k] = a.u[k];
        if (NQ > 2) col[6 + k] = a.w[k];
        col[3 * NQ + k] = a.X[k];
    }
    // the first block's staging, the next block's vertex ids, and the epilogue's tables
    int32_t vid[2], vnext[2] = {-1, -1};
    stage_ids(a, b0, nr, vid);
    stage_dma<NC>(col, stage, SP, nr, vid);
    if (nb > 1) stage_ids(a, b0 + 1, nr, vnext);
    for (uint32_t i = tid; i < 3 * SV; i += PB) acc[i] = 0.0;
    // per-tet streams (packed slots, corner rows, material) and the block vertex's run of block b
    auto load_block = [&](uint32_t b, uint32_t &sw, uint32_t &p0, uint32_t &p1, uint32_t &red, T &mu, T &lam) {
        const uint32_t t = b * PB + tid;
        sw = p0 = p1 = 0u;
        mu = (T)a.mu;
        lam = (T)a.lam;
        if (t < nt) {
            sw = ldc<uint32_t>(a.slot[0], t);
            p0 = ldc<uint32_t>(a.blk_pos[0], t);
            p1 = ldc<uint32_t>(a.blk_pos[1], t);
            if (a.mu_t) {
                mu = ldc<T>(a.mu_t, t);
                lam = ldc<T>(a.lam_t, t);
            }
        }
        red = tid < S ? ldc<uint32_t>(a.blk_run, b * S + tid) : 0u;
    };
    uint32_t sw, p0, p1, red;
    T mu, lam;
    load_block(b0, sw, p0, p1, red, mu, lam);
    for (uint32_t i = 0; i < nb; ++i) {
        const uint32_t b = b0 + i;
        // block i's staging has landed (and the previous block's run sums are done)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // start block i+1's staging into the other buffer; its streams and block i+2's ids
        uint32_t nsw = 0u, np0 = 0u, np1 = 0u, nred = 0u;
        T nmu = (T)a.mu, nlam = (T)a.lam;
        int32_t vn2[2] = {-1, -1};
        if (i + 1 < nb) {
            stage_dma<NC>(col, stage + ((i + 1) & 1u) * NC * SP, SP, nr, vnext);
            load_block(b + 1, nsw, np0, np1, nred, nmu, nlam);
            if (i + 2 < nb) stage_ids(a, b + 2, nr, vn2);
        }
        // evaluate this block's tets from its staged fields
        const double *sd = stage + (i & 1u) * NC * SP;
        const uint32_t t = b * PB + tid;
        if (t < nt) {
            const uint32_t sl[4] = {sw & 255u, (sw >> 8) & 255u, (sw >> 16) & 255u, sw >> 24};
            double qd[4][3], qu[4][3], qw[4][3];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    qd[c][k] = sd[k * SP + sl[c]];
                    qu[c][k] = NQ > 1 ? sd[(3 + k) * SP + sl[c]] : 0.0;
                    qw[c][k] = NQ > 2 ? sd[(6 + k) * SP + sl[c]] : 0.0;
                }
            T bm[9], V0;
            rest_B(sd + 3 * NQ * SP, SP, sl, bm, V0);
            T h[12];
            const bool ok = eval_tet<T, MODEL, OP>(mu, lam, bm, V0, qd, qu, h, qw);
            if (MODEL == EBBX_NH && OP == OP_FORCE && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
            const uint32_t p[4] = {p0 & 0xffffu, p0 >> 16, p1 & 0xffffu, p1 >> 16};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rows[p[c]] = h[3 * c];
                rows[LB + p[c]] = h[3 * c + 1];
                rows[2 * LB + p[c]] = h[3 * c + 2];
            }
        }
        __syncthreads();
        // each block vertex sums its run of rows (fixed order, FP64) into the super-block's
        // accumulator of that vertex (a vertex occurs once per block: no two threads collide)
        {
            const uint32_t j0 = red & 2047u, j1 = (red >> 11) & 2047u, ai = red >> 22;
            if (j1 > j0) {
                double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
                for (uint32_t j = j0; j < j1; ++j) {
                    a0 += (double)rows[j];
                    a1 += (double)rows[LB + j];
                    a2 += (double)rows[2 * LB + j];
                }
                acc[ai] += a0;
                acc[SV + ai] += a1;
                acc[2 * SV + ai] += a2;
            }
        }
        sw = nsw;
        p0 = np0;
        p1 = np1;
        red = nred;
        mu = nmu;
        lam = nlam;
        vnext[0] = vn2[0];
        vnext[1] = vn2[1];
    }
    __syncthreads();
    // the super-block's vertices: stored when it holds every incident tet, else one halo partial
    for (uint32_t k = tid; k < SV; k += PB) {
        const int32_t g = ldc<int32_t>(a.sb_verts, sb * SV + k);
        if (g < 0) break;   // the list is padded at its end
        const int32_t hp = ldc<int32_t>(a.sb_hpos, sb * SV + k);
        double v0 = acc[k], v1 = acc[SV + k], v2 = acc[2 * SV + k];
        const uint32_t gv = (uint32_t)g;
        if (hp < 0) {
            if (a.accumulate) {
                v0 += ldc<double>(a.out[0], gv);
                v1 += ldc<double>(a.out[1], gv);
                v2 += ldc<double>(a.out[2], gv);
            }
            stc<double>(a.out[0], gv, v0);
            stc<double>(a.out[1], gv, v1);
            stc<double>(a.out[2], gv, v2);
        } else {
            double *hq = a.halo + 3 * (size_t)hp;
            hq[0] = v0;
            hq[1] = v1;
            hq[2] = v2;
        }
    }
}

template <class T, int MODEL>
void launch_model(ElemOp op, const ElemArgs &a, unsigned grid, size_t shmem, hipStream_t s) {
    if (op == OP_FORCE) hipLaunchKernelGGL((k_pipe<T, MODEL, OP_FORCE>), dim3(grid), dim3(PB), shmem, s, a);
    else if (op == OP_KMUL) hipLaunchKernelGGL((k_pipe<T, MODEL, OP_KMUL>), dim3(grid), dim3(PB), shmem, s, a);
    else if (op == OP_TMUL) hipLaunchKernelGGL((k_pipe<T, MODEL, OP_TMUL>), dim3(grid), dim3(PB), shmem, s, a);
    else hipLaunchKernelGGL((k_pipe<T, MODEL, OP_DIAG>), dim3(grid), dim3(PB), shmem, s, a);
    HIPCHK(hipGetLastError());
}

}  // namespace

size_t pipe_shmem(const ebbx_fem_s *F, ElemOp op) {
    const int nq = op == OP_TMUL ? 3 : op == OP_KMUL ? 2 : 1;
    return (size_t)2 * (3 * nq + 3) * F->stage_stride * sizeof(double) + (size_t)12 * PB * F->esize +
           (size_t)3 * F->sb_maxv * sizeof(double);
}

void launch_pipe(ebbx_fem_s *F, ElemOp op, const ElemArgs &a0, hipStream_t s) {
    ElemArgs a = a0;
    a.blk_run = F->blk_run.as<uint32_t>();
    a.sb_verts = F->sb_verts.as<int32_t>();
    a.sb_hpos = F->sb_hpos.as<int32_t>();
    a.sb_g = (uint32_t)F->pipe_g;
    a.nsb = (uint32_t)F->nsb;
    a.sb_stride = (uint32_t)F->sb_maxv;
    a.stage_stride = (uint32_t)F->stage_stride;
    const size_t shmem = pipe_shmem(F, op);
    const unsigned grid = (unsigned)F->nsb;
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) launch_model<float, EBBX_STVK>(op, a, grid, shmem, s);
        else launch_model<float, EBBX_NH>(op, a, grid, shmem, s);
    } else {
        if (F->model == EBBX_STVK) launch_model<double, EBBX_STVK>(op, a, grid, shmem, s);
        else launch_model<double, EBBX_NH>(op, a, grid, shmem, s);
    }
}

// Super-blocks of g consecutive 256-tet blocks.  A super-block's vertex list is the
// sorted union of its blocks' lists; a vertex is owned by the super-block when the
// super-block holds every incident tet of it.  Per block vertex: its run of rows in the
// block (start, end) and its index in the super-block's list, packed in one word.
void build_pipe(ebbx_fem_s *F, int32_t g, hipStream_t s) {
    if (g < 1 || g > 16) fail(EBBX_E_ARG, "pipelined blocks: 1 to 16 blocks per workgroup (got %d)", g);
    std::vector<int32_t> keys;
    std::vector<int64_t> rp;
    download_keys(F, keys, rp);
    const HostBlocks hb = host_blocks(keys, rp, F->nt, PB);
    if (hb.w != 1)
        fail(EBBX_E_STATE, "pipelined blocks need at most 256 vertices per block of 256 tets (a block has %d): "
             "reorder the mesh (Morton) or use the block strategy", hb.maxv);
    const int64_t nblk = hb.nblk, nsb = std::max<int64_t>(1, (nblk + g - 1) / g);
    const size_t S = (size_t)hb.maxv;
    std::vector<int32_t> sv_all, sv_ptr(1, 0);
    std::vector<uint8_t> own_all;
    std::vector<uint32_t> red((size_t)std::max<int64_t>(nblk, 1) * S, 0u);
    std::vector<std::pair<int32_t, int32_t>> ent;   // (vertex, incidences in the block)
    int32_t maxsv = 1;
    for (int64_t q = 0; q < nsb; ++q) {
        const int64_t bb = q * g, be = std::min<int64_t>(nblk, bb + g);
        ent.clear();
        for (int64_t b = bb; b < be; ++b)
            for (int32_t k = hb.vptr[(size_t)b]; k < hb.vptr[(size_t)b + 1]; ++k)
                ent.push_back({hb.verts[(size_t)k], hb.lptr[(size_t)k + 1] - hb.lptr[(size_t)k]});
        std::sort(ent.begin(), ent.end());
        std::vector<int32_t> list;
        size_t i = 0;
        while (i < ent.size()) {
            size_t j = i;
            int64_t inc = 0;
            while (j < ent.size() && ent[j].first == ent[i].first) inc += ent[j++].second;
            const int32_t v = ent[i].first;
            list.push_back(v);
            own_all.push_back(inc == rp[(size_t)v + 1] - rp[(size_t)v] ? 1 : 0);
            i = j;
        }
        if (list.size() > 1023)
            fail(EBBX_E_ARG, "super-block %lld touches %zu vertices (limit 1023); use fewer blocks per workgroup",
                 (long long)q, list.size());
        maxsv = std::max(maxsv, (int32_t)list.size());
        for (int64_t b = bb; b < be; ++b) {
            const int32_t a0 = hb.vptr[(size_t)b], a1 = hb.vptr[(size_t)b + 1], base = hb.lptr[(size_t)a0];
            for (int32_t k = a0; k < a1; ++k) {
                const uint32_t j0 = (uint32_t)(hb.lptr[(size_t)k] - base), j1 = (uint32_t)(hb.lptr[(size_t)k + 1] - base);
                const uint32_t ai =
                    (uint32_t)(std::lower_bound(list.begin(), list.end(), hb.verts[(size_t)k]) - list.begin());
                red[(size_t)b * S + (size_t)(k - a0)] = j0 | (j1 << 11) | (ai << 22);
            }
        }
        sv_all.insert(sv_all.end(), list.begin(), list.end());
        sv_ptr.push_back((int32_t)sv_all.size());
    }
    std::vector<int32_t> hpos;
    build_halo(F, sv_all, own_all, rp, hpos, s);
    upload_block_tables(F, hb, {}, s);
    const size_t SV = (size_t)maxsv;
    std::vector<int32_t> pverts((size_t)nsb * SV, -1), phpos((size_t)nsb * SV, -1);
    for (int64_t q = 0; q < nsb; ++q)
        for (int32_t k = sv_ptr[(size_t)q]; k < sv_ptr[(size_t)q + 1]; ++k) {
            pverts[(size_t)q * SV + (size_t)(k - sv_ptr[(size_t)q])] = sv_all[(size_t)k];
            phpos[(size_t)q * SV + (size_t)(k - sv_ptr[(size_t)q])] = hpos[(size_t)k];
        }
    upload(F->blk_run, red.data(), red.size() * sizeof(uint32_t), s);
    upload(F->sb_verts, pverts.data(), pverts.size() * sizeof(int32_t), s);
    upload(F->sb_hpos, phpos.data(), phpos.size() * sizeof(int32_t), s);
    F->pipe_g = g;
    F->nsb = nsb;
    F->sb_maxv = maxsv;
    F->stage_stride = hb.maxv <= 128 ? 128 : 256;
    F->halo_level = g;
    F->blocks_built = false;   // the block tables are the PIPE ones now (no block-level halo)
}

}  // namespace ebbx
