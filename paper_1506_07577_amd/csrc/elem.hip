// elem.hip -- the element-parallel map over the tets relation.
//
// Each tet gathers the vertex fields of its four corners through the tets.v
// key-field, evaluates its hyperelastic element quantity and reduces (+=)
// twelve results into a vertex field (Runtime Implementation, "CPU/GPU
// Specialization" and "Reductions").  The per-tet quantities are those of the
// paper's Vega (StVK) and FreeFem++ (neo-Hookean) workloads (Performance
// Evaluation), written in the displacement-gradient form G = dD B, F = I + G,
// so that single precision keeps its accuracy near the rest shape (no F - I
// or F - F^-T cancellation).
//
// Four reductions:
//  - ATOMIC: one thread per tet, FP64 device-scope atomics (the paper's GPU
//    field reduction);
//  - SEG:    one thread per tet writes its per-corner partials, then one thread
//    per vertex sums them over the grouping's incidence in a fixed order;
//  - BLOCK:  a workgroup takes a block of consecutive (Morton-ordered) tets,
//    stages the block's vertices in LDS (the fields and, for blocks of at most 256
//    vertices, the rest positions, from which each tet recomputes B = Dm^-1
//    instead of streaming the stored B),
//    evaluates, writes each corner's result
//    to its row of the block's incidence order (FP64 rows overwrite the staging
//    after a barrier, so that they do not limit the workgroups per CU), sums each vertex's rows in a
//    fixed order, stores the vertices it owns outright and writes partials of
//    vertices shared with other blocks to a halo buffer that a vertex pass sums
//    in block order.  No global atomics (BLOCK_LDS: the in-block sums with LDS
//    atomics instead of rows);
//  - OWNER:  a workgroup owns a range of vertices and evaluates every tet that
//    touches them (boundary tets once per block), so no halo is needed.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "fem.h"
#include "tetmath.h"

namespace ebbx {

enum Scatter { SC_ATOMIC = 0, SC_PART = 1 };

// ---- one thread per tet: atomic or segmented reduction ------------------------------

template <class T, int MODEL, int OP, int SC>
__global__ __launch_bounds__(256) void k_elem(ElemArgs a) {
    if (a.skip && *a.skip) return;   // uniform over the grid
    const uint32_t nt = a.nt;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    T b[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) b[k] = ldc<T>(a.B[k], t);
    const T V0 = tet_V0(b);
    T mu, lam;
    if (a.mu_t) {
        mu = ldc<T>(a.mu_t, t);
        lam = ldc<T>(a.lam_t, t);
    } else {
        mu = (T)a.mu;
        lam = (T)a.lam;
    }
    uint32_t v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (uint32_t)ldc<int32_t>(a.key[c], t);
    double qd[4][3], qu[4][3], qw[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            qd[c][k] = ldc<double>(a.d[k], v[c]);
            qu[c][k] = (OP == OP_KMUL || OP == OP_TMUL) ? ldc<double>(a.u[k], v[c]) : 0.0;
            qw[c][k] = (OP == OP_TMUL) ? ldc<double>(a.w[k], v[c]) : 0.0;
        }
    T h[12];
    const bool ok = eval_tet<T, MODEL, OP>(mu, lam, b, V0, qd, qu, h, qw);
    if (MODEL == EBBX_NH && OP == OP_FORCE && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
    if (SC == SC_ATOMIC) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) atomicAdd(atc<double>(a.out[k], v[c]), (double)h[3 * c + k]);
    } else {
        T *pp = (T *)a.part + 12 * (size_t)t;
#pragma unroll
        for (int k = 0; k < 12; ++k) pp[k] = h[k];
    }
}

// ---- tet blocks staged in LDS --------------------------------------------------------
//
// Block b holds tets [b*BT, (b+1)*BT), BT = blockDim.x * TPT.  Its vertex list
// blk_verts[vptr[b] .. vptr[b+1]) is sorted; each corner carries its slot in
// that list (packed: 4 x 8 bits per word when every block has <= 256 vertices,
// else 2 x 16 bits in each of two words).

template <int W> __device__ __forceinline__ void unpack_slots(const ElemArgs &a, uint32_t t, uint32_t *s) {
    if (W == 1) {
        const uint32_t w = ldc<uint32_t>(a.slot[0], t);
        s[0] = w & 255u;
        s[1] = (w >> 8) & 255u;
        s[2] = (w >> 16) & 255u;
        s[3] = w >> 24;
    } else {
        const uint32_t w0 = ldc<uint32_t>(a.slot[0], t), w1 = ldc<uint32_t>(a.slot[1], t);
        s[0] = w0 & 65535u;
        s[1] = w0 >> 16;
        s[2] = w1 & 65535u;
        s[3] = w1 >> 16;
    }
}

// LDS layout: the block's vertex fields with one column per component (d, and
// u for the stiffness product), then the per-corner results, three columns
// (x, y, z) whose rows follow the block's incidence order (by vertex, then
// local tet, then corner): each tet writes its four corners to the rows the
// block tables give them, so every block vertex then sums one contiguous run
// of rows (fixed order, FP64) and either stores it (the block owns the vertex)
// or writes it to the halo.  Every global load that does not depend on another
// is issued at kernel start.
template <class T>
__device__ __forceinline__ void reduce_slot(const ElemArgs &a, const T *s_h, uint32_t LB, uint32_t gv, int32_t hp,
                                            int32_t j0, int32_t j1) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
    for (int32_t j = j0; j < j1; ++j) {   // this vertex's rows, in (local tet, corner) order
        a0 += (double)s_h[j];
        a1 += (double)s_h[LB + j];
        a2 += (double)s_h[2 * LB + j];
    }
    if (hp < 0) {
        // every incident tet is in this block: sole writer
        if (a.accumulate) {
            a0 += ldc<double>(a.out[0], gv);
            a1 += ldc<double>(a.out[1], gv);
            a2 += ldc<double>(a.out[2], gv);
        }
        stc<double>(a.out[0], gv, a0);
        stc<double>(a.out[1], gv, a1);
        stc<double>(a.out[2], gv, a2);
    } else {
        double *hq = a.halo + 3 * (size_t)hp;
        hq[0] = a0;
        hq[1] = a1;
        hq[2] = a2;
    }
}

// Gradient dD B of a vertex field staged in LDS (3 columns of S block vertices) over the
// tet whose corners sit in slots sl.
template <class T>
__device__ __forceinline__ void staged_grad(const double *s, uint32_t S, const uint32_t *sl, const T *b, T *G) {
    double q[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) q[c][k] = s[k * S + sl[c]];
    grad_from(q, b, G);
}

// One tet block (blk) of the BLOCK strategies, evaluated by the whole workgroup.
template <class T, int MODEL, int OP, int TPT, int W, int RED>
__device__ __forceinline__ void block_body(const ElemArgs &a, uint32_t blk, uint32_t tid) {
    extern __shared__ uint4 s_dyn4[];
    const uint32_t nt = a.nt;
    const uint32_t nthr = blockDim.x, BT = nthr * TPT;
    const uint32_t LB = 4 * BT;   // rows of one component column of the per-corner results
    // block tables at a fixed stride S (padded with vertex -1): no dependent offset load
    const uint32_t S = a.blk_stride;
    const int32_t *bverts = a.blk_verts + (size_t)blk * S;
    const int32_t *bhpos = a.blk_hpos + (size_t)blk * S;
    const uint16_t *brow = a.blk_row + (size_t)blk * (S + 1);
    const uint32_t t0 = blk * BT;
    // RED == 0: per-corner result rows in the block's incidence order (deterministic sums);
    // RED == 1: FP64 LDS atomics into one accumulator per block vertex
    constexpr int NQ = OP == OP_TMUL ? 3 : OP == OP_KMUL ? 2 : 1;   // staged vertex fields
    double *s_d = (double *)s_dyn4;
    double *s_u = s_d + 3 * S;
    double *s_w = s_u + 3 * S;
    // blocks of at most 256 vertices (8-bit corner slots, a well-ordered mesh) stage the rest
    // positions and recompute B per tet; others stream the stored B (their vertex gathers are
    // scattered, and the 24 B per block vertex would cost more than the 36-72 B per tet)
    constexpr bool XB = W == 1;
    // FP32 elements stage the block-local FP32 rest positions of a precomputed table (read
    // contiguously, without waiting for the block's vertex ids) instead of gathering X
    constexpr bool XF = XB && sizeof(T) == 4;
    double *s_x = s_d + 3 * NQ * S;   // rest positions of the block's vertices (XB)
    float *s_xf = (float *)s_x;       // their block-local FP32 form (XF)
    const float *xf[3] = {nullptr, nullptr, nullptr};
    if (XF)
#pragma unroll
        for (int k = 0; k < 3; ++k) xf[k] = a.xf[k] + (size_t)blk * S;
    // rows (moved to the LDS start when REUSE); after the FP32 rest positions they start at a
    // multiple of 4 floats
    T *s_h = XF ? (T *)(s_xf + ((3 * S + 3) & ~3u)) : (T *)(s_x + (XB ? 3 * S : 0));
    double *s_acc = (double *)s_h;

    // this thread's first block vertex
    const int32_t gvs0 = tid < S ? bverts[tid] : -1;
    const bool has = gvs0 >= 0;
    const uint32_t gv0 = has ? (uint32_t)gvs0 : 0u;
    int32_t hp0 = -1, j00 = 0, j10 = 0;
    if (has) {
        hp0 = bhpos[tid];
        if (RED == 0) {
            j00 = brow[tid];
            j10 = brow[tid + 1];
        }
    }
    // per-tet streams
    T b[TPT][9], V0[TPT], mu[TPT], lam[TPT];
    uint32_t sl[TPT][4], pw[TPT][2];
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
        const uint32_t t = t0 + r * nthr + tid;
        if (t < nt) {
            if (!XB) {
#pragma unroll
                for (int k = 0; k < 9; ++k) b[r][k] = ldc<T>(a.B[k], t);
                V0[r] = tet_V0(b[r]);
            }
            if (a.mu_t) {
                mu[r] = ldc<T>(a.mu_t, t);
                lam[r] = ldc<T>(a.lam_t, t);
            } else {
                mu[r] = (T)a.mu;
                lam[r] = (T)a.lam;
            }
            unpack_slots<W>(a, t, sl[r]);
            if (RED == 0) {
                pw[r][0] = ldc<uint32_t>(a.blk_pos[0], t);
                pw[r][1] = ldc<uint32_t>(a.blk_pos[1], t);
            }
        }
    }
    if (has) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_d[k * S + tid] = ldc<double>(a.d[k], gv0);
            if (XF) s_xf[k * S + tid] = xf[k][tid];
            else if (XB) s_x[k * S + tid] = ldc<double>(a.X[k], gv0);
            if (NQ > 1) s_u[k * S + tid] = ldc<double>(a.u[k], gv0);
            if (NQ > 2) s_w[k * S + tid] = ldc<double>(a.w[k], gv0);
            if (RED == 1) s_acc[k * S + tid] = 0.0;
        }
    }
    for (uint32_t i = tid + nthr; i < S; i += nthr) {
        const int32_t gvs = bverts[i];
        if (gvs < 0) continue;
        const uint32_t gv = (uint32_t)gvs;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_d[k * S + i] = ldc<double>(a.d[k], gv);
            if (XF) s_xf[k * S + i] = xf[k][i];
            else if (XB) s_x[k * S + i] = ldc<double>(a.X[k], gv);
            if (NQ > 1) s_u[k * S + i] = ldc<double>(a.u[k], gv);
            if (NQ > 2) s_w[k * S + i] = ldc<double>(a.w[k], gv);
            if (RED == 1) s_acc[k * S + i] = 0.0;
        }
    }
    __syncthreads();
    // FP64 per-corner rows (24 KiB per 256 tets) would cap the workgroups per CU when added to
    // the staging: there every tet first takes its gradients from the staged fields into
    // registers, and after a barrier the rows overwrite the staging from the start of the LDS.
    // FP32 rows are half as large and keep the single pass.
    constexpr bool REUSE = sizeof(T) == 8 && RED == 0;
    if (REUSE) {
        T G[TPT][9], D1[TPT][9], D2[TPT][9];
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const uint32_t t = t0 + r * nthr + tid;
            if (t < nt) {
                if (XB) rest_B(s_x, S, sl[r], b[r], V0[r]);
                staged_grad(s_d, S, sl[r], b[r], G[r]);
                if (NQ > 1) staged_grad(s_u, S, sl[r], b[r], D1[r]);
                if (NQ > 2) staged_grad(s_w, S, sl[r], b[r], D2[r]);
            }
        }
        __syncthreads();
        T *s_r = (T *)s_dyn4;
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const uint32_t t = t0 + r * nthr + tid;
            if (t < nt) {
                T h[12];
                bool ok = true;
                if (OP == OP_TMUL) {
                    T Q[9];
                    ok = d2stress_scaled<T, MODEL>(mu[r], lam[r], V0[r], G[r], D1[r], D2[r], Q);
                    corner_out(Q, b[r], h);
                } else if (OP == OP_FORCE) {
                    T P[9];
                    ok = stress_scaled<T, MODEL>(mu[r], lam[r], V0[r], G[r], P);
                    corner_out(P, b[r], h);
                } else if (OP == OP_KMUL) {
                    T dP[9];
                    ok = dstress_scaled<T, MODEL>(mu[r], lam[r], V0[r], G[r], D1[r], dP);
                    corner_out(dP, b[r], h);
                } else {
                    ok = diag12<T, MODEL>(mu[r], lam[r], G[r], b[r], V0[r], h);
                }
                if (MODEL == EBBX_NH && OP == OP_FORCE && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
                const uint32_t p[4] = {pw[r][0] & 0xffffu, pw[r][0] >> 16, pw[r][1] & 0xffffu, pw[r][1] >> 16};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    s_r[p[c]] = h[3 * c];
                    s_r[LB + p[c]] = h[3 * c + 1];
                    s_r[2 * LB + p[c]] = h[3 * c + 2];
                }
            }
        }
        s_h = s_r;
    } else {
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const uint32_t tl = r * nthr + tid, t = t0 + tl;
            if (t < nt) {
                double qd[4][3], qu[4][3], qw[4][3];
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        qd[c][k] = s_d[k * S + sl[r][c]];
                        qu[c][k] = (NQ > 1) ? s_u[k * S + sl[r][c]] : 0.0;
                        qw[c][k] = (NQ > 2) ? s_w[k * S + sl[r][c]] : 0.0;
                    }
                if constexpr (XF) rest_B_local(s_xf, S, sl[r], b[r], V0[r]);
                else if (XB) rest_B(s_x, S, sl[r], b[r], V0[r]);
                T h[12];
                const bool ok = eval_tet<T, MODEL, OP>(mu[r], lam[r], b[r], V0[r], qd, qu, h, qw);
                if (MODEL == EBBX_NH && OP == OP_FORCE && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
                if (RED == 0) {
                    const uint32_t p[4] = {pw[r][0] & 0xffffu, pw[r][0] >> 16, pw[r][1] & 0xffffu, pw[r][1] >> 16};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        s_h[p[c]] = h[3 * c];
                        s_h[LB + p[c]] = h[3 * c + 1];
                        s_h[2 * LB + p[c]] = h[3 * c + 2];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int k = 0; k < 3; ++k) atomicAdd(&s_acc[k * S + sl[r][c]], (double)h[3 * c + k]);
                }
            }
        }
    }
    __syncthreads();
    if (RED == 0) {
        if (has) reduce_slot<T>(a, s_h, LB, gv0, hp0, j00, j10);
        for (uint32_t i = tid + nthr; i < S; i += nthr) {
            const int32_t gvs = bverts[i];
            if (gvs >= 0) reduce_slot<T>(a, s_h, LB, (uint32_t)gvs, bhpos[i], brow[i], brow[i + 1]);
        }
    } else {
        for (uint32_t i = tid; i < S; i += nthr) {
            const int32_t gvs = i == tid ? gvs0 : bverts[i];
            if (gvs < 0) continue;
            const uint32_t gv = (uint32_t)gvs;
            const int32_t hp = i == tid ? hp0 : bhpos[i];
            double v0 = s_acc[i], v1 = s_acc[S + i], v2 = s_acc[2 * S + i];
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
}

template <class T, int MODEL, int OP, int TPT, int W, int RED>
__global__ __launch_bounds__(512) void k_block(ElemArgs a) {
    if (a.skip && *a.skip) return;   // uniform over the grid
    const uint32_t blk = xcd_block(blockIdx.x, a.nblk, a.xcd_run_log2);
    if (a.mdone) {   // a batch: skip the block once every mesh it touches has finished (uniform)
        const uint32_t BT = blockDim.x * TPT, t0 = blk * BT;
        const int32_t m0 = a.tmesh[t0], m1 = a.tmesh[min(t0 + BT, a.nt) - 1];
        bool all = true;
        for (int32_t m = m0; m <= m1; ++m) all = all && a.mdone[m] != 0;
        if (all) return;
    }
    block_body<T, MODEL, OP, TPT, W, RED>(a, blk, threadIdx.x);
}

// The block kernel of a batched solve over the list of the blocks of its unfinished meshes
// (a.act; see ActList): a fixed grid of workgroups, each taking one contiguous stretch of the
// list (XCD x's workgroups, x = workgroup mod 8, one contiguous eighth of it), so iterations in
// which few meshes still iterate dispatch no workgroups for the finished ones.
// The loop costs registers: the FP32 products would need 80-88 VGPRs (5 waves per SIMD)
// against 55-69 for k_block; they are held to 6 waves (80 VGPRs, at most a couple spilled).
template <class T, int MODEL, int OP, int W>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) void k_block_list(ElemArgs a) {
    __shared__ int32_t s_m[1];
    if (a.skip && *a.skip) return;   // uniform over the grid
    const ActList L = act_list(a.act, a.act_nm);
    const uint32_t n = (uint32_t)L.hdr[0], G = gridDim.x;
    const uint32_t r = (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);   // G is a multiple of 8
    const uint32_t i0 = (uint32_t)(((uint64_t)r * n) / G), i1 = (uint32_t)(((uint64_t)(r + 1) * n) / G);
    if (i0 >= i1) return;
    // the list range holding item i0 (bpfx is ascending; ranges may be empty)
    const int32_t nam = L.hdr[2];
    if (threadIdx.x == 0) s_m[0] = 0;
    __syncthreads();
    for (int32_t j = threadIdx.x; j < nam; j += blockDim.x)
        if ((uint32_t)L.bpfx[j] <= i0 && i0 < (uint32_t)L.bpfx[j + 1]) s_m[0] = j;
    __syncthreads();
    // list positions are the same in every lane: keep them in scalar registers, so that the
    // block's table addresses stay scalar as in k_block
    int32_t j = __builtin_amdgcn_readfirstlane(s_m[0]);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane(L.bpfx[j]);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane(L.bpfx[j + 1]);
    for (uint32_t i = i0; i < i1; ++i) {
        while (i >= hi) {
            ++j;
            lo = hi;
            hi = (uint32_t)__builtin_amdgcn_readfirstlane(L.bpfx[j + 1]);
        }
        if (i > i0) __syncthreads();   // the previous block is done with the LDS
        const uint32_t blk = (uint32_t)__builtin_amdgcn_readfirstlane(L.bstart[j]) + (i - lo);
        // the thread index passes through an empty asm statement, so that the compiler does not
        // hoist the per-thread values the body derives from it out of the loop and keep them
        // live across blocks (98 VGPRs against the body's 69 for the FP32 neo-Hookean product)
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        block_body<T, MODEL, OP, 1, W, 0>(a, blk, tid);
    }
}

// The run sum of one block vertex for output column set `out` (owned) or halo slot `hq`
// (shared), as reduce_slot, overwriting (the step preamble does not accumulate).
template <class T>
__device__ __forceinline__ void reduce_pre(const T *s_h, uint32_t LB, uint32_t gv, double *const *out, double *hq,
                                           int32_t j0, int32_t j1) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
    for (int32_t j = j0; j < j1; ++j) {
        a0 += (double)s_h[j];
        a1 += (double)s_h[LB + j];
        a2 += (double)s_h[2 * LB + j];
    }
    if (!hq) {
        stc<double>(out[0], gv, a0);
        stc<double>(out[1], gv, a1);
        stc<double>(out[2], gv, a2);
    } else {
        hq[0] = a0;
        hq[1] = a1;
        hq[2] = a2;
    }
}

// The implicit step's preamble for one tet block: the forces f(d), the product K(d) u and the
// raw stiffness diagonal.  The block's d and u (and rest positions) are staged once, and each
// tet's rest shape and gradients are formed once; the three per-corner results then pass through
// the incidence-order rows one after another (rows, barrier, run sums, barrier), so each output
// is summed exactly as its own element map would sum it.  Owned vertices store f, K u and the
// diagonal; a shared vertex writes its three partials to one 9-wide halo entry.
template <class T, int MODEL, int W>
__device__ __forceinline__ void block_body_pre(const ElemArgs &a, uint32_t blk, uint32_t tid) {
    extern __shared__ uint4 s_dyn4[];
    const uint32_t nt = a.nt, BT = blockDim.x, LB = 4 * BT;
    const uint32_t S = a.blk_stride;
    const int32_t *bverts = a.blk_verts + (size_t)blk * S;
    const int32_t *bhpos = a.blk_hpos + (size_t)blk * S;
    const uint16_t *brow = a.blk_row + (size_t)blk * (S + 1);
    const uint32_t t = blk * BT + tid;
    const bool in = t < nt;
    // the LDS layout of the stiffness product's block kernel (d, u, then the rest positions)
    constexpr bool XB = W == 1;
    constexpr bool XF = XB && sizeof(T) == 4;
    constexpr bool REUSE = sizeof(T) == 8;   // FP64 rows overwrite the staging
    double *s_d = (double *)s_dyn4;
    double *s_u = s_d + 3 * S;
    double *s_x = s_u + 3 * S;
    float *s_xf = (float *)s_x;
    T *s_h = REUSE ? (T *)s_dyn4 : XF ? (T *)(s_xf + ((3 * S + 3) & ~3u)) : (T *)(s_x + (XB ? 3 * S : 0));

    const int32_t gvs0 = tid < S ? bverts[tid] : -1;
    const bool has = gvs0 >= 0;
    const uint32_t gv0 = has ? (uint32_t)gvs0 : 0u;
    int32_t hp0 = -1, j00 = 0, j10 = 0;
    if (has) {
        hp0 = bhpos[tid];
        j00 = brow[tid];
        j10 = brow[tid + 1];
    }
    T b[9], V0 = T(1), mu = T(0), lam = T(0);
    uint32_t sl[4] = {0, 0, 0, 0}, pw[2] = {0, 0};
    if (in) {
        if (!XB) {
#pragma unroll
            for (int k = 0; k < 9; ++k) b[k] = ldc<T>(a.B[k], t);
            V0 = tet_V0(b);
        }
        if (a.mu_t) {
            mu = ldc<T>(a.mu_t, t);
            lam = ldc<T>(a.lam_t, t);
        } else {
            mu = (T)a.mu;
            lam = (T)a.lam;
        }
        unpack_slots<W>(a, t, sl);
        pw[0] = ldc<uint32_t>(a.blk_pos[0], t);
        pw[1] = ldc<uint32_t>(a.blk_pos[1], t);
    }
    const float *xf[3] = {nullptr, nullptr, nullptr};
    if (XF)
#pragma unroll
        for (int k = 0; k < 3; ++k) xf[k] = a.xf[k] + (size_t)blk * S;
    for (uint32_t i = tid; i < S; i += BT) {
        const int32_t gvs = i == tid ? gvs0 : bverts[i];
        if (gvs < 0) continue;
        const uint32_t gv = (uint32_t)gvs;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_d[k * S + i] = ldc<double>(a.d[k], gv);
            s_u[k * S + i] = ldc<double>(a.u[k], gv);
            if (XF) s_xf[k * S + i] = xf[k][i];
            else if (XB) s_x[k * S + i] = ldc<double>(a.X[k], gv);
        }
    }
    __syncthreads();
    T G[9], dF[9];
    if (in) {
        if constexpr (XF) rest_B_local(s_xf, S, sl, b, V0);
        else if (XB) rest_B(s_x, S, sl, b, V0);
        staged_grad(s_d, S, sl, b, G);
        staged_grad(s_u, S, sl, b, dF);
    }
    const uint32_t p[4] = {pw[0] & 0xffffu, pw[0] >> 16, pw[1] & 0xffffu, pw[1] >> 16};
    // unrolled: each phase keeps only the registers it needs (78 VGPRs for the FP32 neo-Hookean
    // pass against 102 with one loop body)
#pragma unroll
    for (int ph = 0; ph < 3; ++ph) {
        __syncthreads();   // the staging (REUSE) or the previous phase's rows are no longer read
        if (in) {
            T h[12];
            if (ph == 0) {
                T P[9];
                const bool ok = stress_scaled<T, MODEL>(mu, lam, V0, G, P);
                corner_out(P, b, h);
                if (MODEL == EBBX_NH && !ok) atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
            } else if (ph == 1) {
                T dP[9];
                dstress_scaled<T, MODEL>(mu, lam, V0, G, dF, dP);
                corner_out(dP, b, h);
            } else {
                diag12<T, MODEL>(mu, lam, G, b, V0, h);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                s_h[p[c]] = h[3 * c];
                s_h[LB + p[c]] = h[3 * c + 1];
                s_h[2 * LB + p[c]] = h[3 * c + 2];
            }
        }
        __syncthreads();
        double *const *out = a.pre_out[ph];
        if (has) reduce_pre<T>(s_h, LB, gv0, out, hp0 < 0 ? nullptr : a.halo9 + 9 * (size_t)hp0 + 3 * ph, j00, j10);
        for (uint32_t i = tid + BT; i < S; i += BT) {
            const int32_t gvs = bverts[i];
            if (gvs < 0) continue;
            const int32_t hp = bhpos[i];
            reduce_pre<T>(s_h, LB, (uint32_t)gvs, out, hp < 0 ? nullptr : a.halo9 + 9 * (size_t)hp + 3 * ph, brow[i],
                          brow[i + 1]);
        }
    }
}

template <class T, int MODEL, int W>
__global__ __launch_bounds__(512) void k_block_pre(ElemArgs a) {
    block_body_pre<T, MODEL, W>(a, xcd_block(blockIdx.x, a.nblk, a.xcd_run_log2), threadIdx.x);
}

// OWNER strategy: workgroup = one block of owned vertices.  The block stages
// the fields of its vertices (owned, then ghosts) in LDS, evaluates every tet
// listed for it, writes the rows of owned corners to their positions in the
// block's incidence order, and each owned vertex sums its contiguous run of
// rows in FP64 (the grouping's (tet, corner) order) and stores the result.
template <class T, int MODEL, int OP>
__global__ __launch_bounds__(256) void k_owner(ElemArgs a) {
    extern __shared__ double s_own[];
    if (a.skip && *a.skip) return;   // uniform over the grid
    const uint32_t tid = threadIdx.x;
    const uint32_t blk = xcd_block(blockIdx.x, a.own_nblk);
    const uint32_t v0 = blk * a.own_vb;
    const uint32_t nown = min(a.own_vb, a.nv - v0);
    const uint32_t g0 = (uint32_t)a.own_gptr[blk], ngh = (uint32_t)a.own_gptr[blk + 1] - g0;
    const uint32_t nvb = nown + ngh;
    const uint32_t tb = (uint32_t)a.own_tptr[blk], ntb = (uint32_t)a.own_tptr[blk + 1] - tb;
    if (a.mdone && ntb > 0) {   // a batch: skip once every mesh of the block's tets has finished (uniform)
        const int32_t m0 = a.tmesh[a.own_meta[tb].x], m1 = a.tmesh[a.own_meta[tb + ntb - 1].x];
        bool all = true;
        for (int32_t m = m0; m <= m1; ++m) all = all && a.mdone[m] != 0;
        if (all) return;
    }
    const int64_t rbase = a.rp[v0];
    const uint32_t ninc = (uint32_t)(a.rp[v0 + nown] - rbase);
    constexpr int NQ = OP == OP_TMUL ? 3 : OP == OP_KMUL ? 2 : 1;
    double *s_d = s_own;
    double *s_u = s_d + 3 * nvb;
    double *s_w = s_u + 3 * nvb;
    T *s_h = (T *)(s_d + 3 * NQ * nvb);   // 3 columns of ninc rows
    // this thread's owned vertex: its incidence run
    uint32_t e0 = 0, e1 = 0;
    if (tid < nown) {
        e0 = (uint32_t)(a.rp[v0 + tid] - rbase);
        e1 = (uint32_t)(a.rp[v0 + tid + 1] - rbase);
    }
    for (uint32_t i = tid; i < nvb; i += blockDim.x) {
        const uint32_t gv = i < nown ? v0 + i : (uint32_t)a.own_ghost[g0 + i - nown];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_d[k * nvb + i] = ldc<double>(a.d[k], gv);
            if (NQ > 1) s_u[k * nvb + i] = ldc<double>(a.u[k], gv);
            if (NQ > 2) s_w[k * nvb + i] = ldc<double>(a.w[k], gv);
        }
    }
    __syncthreads();
    for (uint32_t j = tid; j < ntb; j += blockDim.x) {
        const uint4 m = a.own_meta[tb + j];
        const uint32_t t = m.x;
        T b[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) b[k] = ldc<T>(a.B[k], t);
        const T V0 = tet_V0(b);
        T mu, lam;
        if (a.mu_t) {
            mu = ldc<T>(a.mu_t, t);
            lam = ldc<T>(a.lam_t, t);
        } else {
            mu = (T)a.mu;
            lam = (T)a.lam;
        }
        // corners: 24 bits each over (y, z, w): 11-bit slot | 13-bit position (0x1fff: not owned)
        const uint64_t lo = (uint64_t)m.y | ((uint64_t)m.z << 32);
        const uint32_t cw[4] = {(uint32_t)(lo & 0xffffffu), (uint32_t)((lo >> 24) & 0xffffffu),
                                (uint32_t)((lo >> 48) | ((uint64_t)(m.w & 0xffu) << 16)), m.w >> 8};
        double qd[4][3], qu[4][3], qw[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t sl = cw[c] & 0x7ffu;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qd[c][k] = s_d[k * nvb + sl];
                qu[c][k] = (NQ > 1) ? s_u[k * nvb + sl] : 0.0;
                qw[c][k] = (NQ > 2) ? s_w[k * nvb + sl] : 0.0;
            }
        }
        T h[12];
        const bool ok = eval_tet<T, MODEL, OP>(mu, lam, b, V0, qd, qu, h, qw);
        // the block owning corner 0 counts an inverted tet (exactly once over all blocks)
        if (MODEL == EBBX_NH && OP == OP_FORCE && !ok && (cw[0] >> 11) != 0x1fffu)
            atomicAdd(a.n_inv + (a.tmesh ? a.tmesh[t] : 0), 1ull);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t p = cw[c] >> 11;
            if (p != 0x1fffu) {
                s_h[p] = h[3 * c];
                s_h[ninc + p] = h[3 * c + 1];
                s_h[2 * ninc + p] = h[3 * c + 2];
            }
        }
    }
    __syncthreads();
    if (tid < nown) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (uint32_t e = e0; e < e1; ++e) {
            a0 += (double)s_h[e];
            a1 += (double)s_h[ninc + e];
            a2 += (double)s_h[2 * ninc + e];
        }
        const uint32_t gv = v0 + tid;
        if (a.accumulate) {
            a0 += ldc<double>(a.out[0], gv);
            a1 += ldc<double>(a.out[1], gv);
            a2 += ldc<double>(a.out[2], gv);
        }
        stc<double>(a.out[0], gv, a0);
        stc<double>(a.out[1], gv, a1);
        stc<double>(a.out[2], gv, a2);
    }
}

template <class T, int MODEL>
static void launch_owner(ElemOp op, const ElemArgs &a, unsigned grid, size_t shmem, hipStream_t s) {
    if (op == OP_FORCE) hipLaunchKernelGGL((k_owner<T, MODEL, OP_FORCE>), dim3(grid), dim3(256), shmem, s, a);
    else if (op == OP_KMUL) hipLaunchKernelGGL((k_owner<T, MODEL, OP_KMUL>), dim3(grid), dim3(256), shmem, s, a);
    else if (op == OP_TMUL) hipLaunchKernelGGL((k_owner<T, MODEL, OP_TMUL>), dim3(grid), dim3(256), shmem, s, a);
    else hipLaunchKernelGGL((k_owner<T, MODEL, OP_DIAG>), dim3(grid), dim3(256), shmem, s, a);
    HIPCHK(hipGetLastError());
}

// Sum each shared vertex's halo entries (its blocks' partials, in block order).
__global__ __launch_bounds__(256) void k_halo_reduce(const double *halo, const int32_t *sh_vert, const int32_t *sh_ptr,
                                                     const int32_t *sh_pos, uint32_t S, double *o0, double *o1,
                                                     double *o2, int accumulate, const int *skip) {
    if (skip && *skip) return;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)sh_vert[s];
        const int32_t j0 = sh_ptr[s], j1 = sh_ptr[s + 1];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int32_t j = j0; j < j1; ++j) {
            const double *hq = halo + 3 * (size_t)sh_pos[j];
            a0 += hq[0];
            a1 += hq[1];
            a2 += hq[2];
        }
        if (accumulate) {
            a0 += ldc<double>(o0, v);
            a1 += ldc<double>(o1, v);
            a2 += ldc<double>(o2, v);
        }
        stc<double>(o0, v, a0);
        stc<double>(o1, v, a1);
        stc<double>(o2, v, a2);
    }
}

// The same sum with each shared vertex's halo positions in one fixed-width row
// (NC x 4 entries, -1 padded, in block order): one dependent load fewer.
template <int NC>
__global__ __launch_bounds__(256) void k_halo_tab(const double *halo, const int32_t *sh_vert, const int4 *tab,
                                                  uint32_t S, double *o0, double *o1, double *o2, int accumulate,
                                                  const int *skip) {
    if (skip && *skip) return;
    // XCD x sums one contiguous eighth of the shared vertices (sorted by id), those of its own
    // eighth of the Morton-ordered blocks, whose halo entries that XCD wrote
    const uint32_t wg = xcd_block(blockIdx.x, gridDim.x);
    for (uint32_t s = wg * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)sh_vert[s];
        int4 q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = tab[(size_t)s * NC + c];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int32_t p[4] = {q[c].x, q[c].y, q[c].z, q[c].w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (p[k] >= 0) {
                    const double *hq = halo + 3 * (size_t)p[k];
                    a0 += hq[0];
                    a1 += hq[1];
                    a2 += hq[2];
                }
        }
        if (accumulate) {
            a0 += ldc<double>(o0, v);
            a1 += ldc<double>(o1, v);
            a2 += ldc<double>(o2, v);
        }
        stc<double>(o0, v, a0);
        stc<double>(o1, v, a1);
        stc<double>(o2, v, a2);
    }
}

// Vertex-owned reduction of per-corner partials over the grouping (CSR rows in
// increasing (tet, corner) order: a fixed summation order, so the result is
// bitwise reproducible).
template <class T>
__global__ __launch_bounds__(256) void k_seg_gather(const T *part, const int64_t *row_ptr, const int32_t *inc,
                                                    int64_t nv, double *out, int accumulate) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        const int64_t e1 = row_ptr[v + 1];
        for (int64_t j = row_ptr[v]; j < e1; ++j) {
            const int e = inc[j];
            const T *p = part + 12 * (int64_t)(e >> 2) + 3 * (e & 3);
            s0 += (double)p[0];
            s1 += (double)p[1];
            s2 += (double)p[2];
        }
        if (accumulate) {
            out[v] += s0;
            out[nv + v] += s1;
            out[2 * nv + v] += s2;
        } else {
            out[v] = s0;
            out[nv + v] = s1;
            out[2 * nv + v] = s2;
        }
    }
}

__global__ void k_fill(double *p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_n(int64_t n, int threads, int64_t cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

void fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_n(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    HIPCHK(hipGetLastError());
}

// ---- dispatch ---------------------------------------------------------------------------

template <class T, int MODEL, int OP>
static void launch_flat(int sc, const ElemArgs &a, int block, hipStream_t s) {
    const unsigned grid = grid_n(a.nt, block, 1ll << 31);
    if (sc == SC_ATOMIC) hipLaunchKernelGGL((k_elem<T, MODEL, OP, SC_ATOMIC>), dim3(grid), dim3(block), 0, s, a);
    else hipLaunchKernelGGL((k_elem<T, MODEL, OP, SC_PART>), dim3(grid), dim3(block), 0, s, a);
    HIPCHK(hipGetLastError());
}

template <class T, int MODEL, int OP, int W>
static void launch_block_w(int tpt, int red, const ElemArgs &a, int threads, unsigned grid, size_t shmem,
                           hipStream_t s) {
    if (red == 0) {
        if (tpt == 1) hipLaunchKernelGGL((k_block<T, MODEL, OP, 1, W, 0>), dim3(grid), dim3(threads), shmem, s, a);
        else hipLaunchKernelGGL((k_block<T, MODEL, OP, 2, W, 0>), dim3(grid), dim3(threads), shmem, s, a);
    } else {
        if (tpt == 1) hipLaunchKernelGGL((k_block<T, MODEL, OP, 1, W, 1>), dim3(grid), dim3(threads), shmem, s, a);
        else hipLaunchKernelGGL((k_block<T, MODEL, OP, 2, W, 1>), dim3(grid), dim3(threads), shmem, s, a);
    }
    HIPCHK(hipGetLastError());
}

template <class T, int MODEL, int OP>
static void launch_block(int tpt, int w, int red, const ElemArgs &a, int threads, unsigned grid, size_t shmem,
                         hipStream_t s) {
    if (w == 1) launch_block_w<T, MODEL, OP, 1>(tpt, red, a, threads, grid, shmem, s);
    else launch_block_w<T, MODEL, OP, 2>(tpt, red, a, threads, grid, shmem, s);
}

template <class T, int MODEL>
static void launch_model(bool block, ElemOp op, int sc, int tpt, int w, int red, const ElemArgs &a, int threads,
                         unsigned grid, size_t shmem, hipStream_t s) {
    if (block) {
        if (op == OP_FORCE) launch_block<T, MODEL, OP_FORCE>(tpt, w, red, a, threads, grid, shmem, s);
        else if (op == OP_KMUL) launch_block<T, MODEL, OP_KMUL>(tpt, w, red, a, threads, grid, shmem, s);
        else if (op == OP_TMUL) launch_block<T, MODEL, OP_TMUL>(tpt, w, red, a, threads, grid, shmem, s);
        else launch_block<T, MODEL, OP_DIAG>(tpt, w, red, a, threads, grid, shmem, s);
    } else {
        if (op == OP_FORCE) launch_flat<T, MODEL, OP_FORCE>(sc, a, threads, s);
        else if (op == OP_KMUL) launch_flat<T, MODEL, OP_KMUL>(sc, a, threads, s);
        else if (op == OP_TMUL) launch_flat<T, MODEL, OP_TMUL>(sc, a, threads, s);
        else launch_flat<T, MODEL, OP_DIAG>(sc, a, threads, s);
    }
}

bool elem_list_ok(const ebbx_fem_s *F, ElemOp op) {
    return op == OP_KMUL && F->strategy == EBBX_STRAT_BLOCK && F->blk_red == 0 && F->blk_tpt == 1 &&
           F->blk_tets <= 512;
}

// The list-driven block kernel runs as many workgroups as fit on the device at once (a
// multiple of 8, one share per XCD), so that each takes one stretch of the list.
template <class T, int MODEL>
static void launch_block_list(ebbx_fem_s *F, const ElemArgs &a, int threads, size_t shmem, hipStream_t s) {
    auto run = [&](auto kern) {
        int per_cu = 0, dev = 0, ncu = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, shmem));
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        const int64_t g = (int64_t)std::max(per_cu, 1) * std::max(ncu, 1);
        const unsigned grid = (unsigned)std::max<int64_t>(8, std::min<int64_t>(g, ((int64_t)F->nblk + 7) / 8 * 8) / 8 * 8);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), shmem, s, a);
        HIPCHK(hipGetLastError());
    };
    if (F->blk_w == 1) run(k_block_list<T, MODEL, OP_KMUL, 1>);
    else run(k_block_list<T, MODEL, OP_KMUL, 2>);
}

static ElemArgs base_args(ebbx_fem_s *F) {
    ElemArgs a{};
    const uint32_t nt = (uint32_t)F->nt, nv = (uint32_t)F->nv;
    const size_t es = F->esize;
    a.nt = nt;
    a.nv = nv;
    for (int c = 0; c < 4; ++c) a.key[c] = F->keys + (size_t)c * nt;
    for (int k = 0; k < 9; ++k) a.B[k] = (const char *)F->B.get() + (size_t)k * nt * es;
    a.V0 = F->V0.get();
    if (F->per_tet) {
        a.mu_t = F->mat.get();
        a.lam_t = (const char *)F->mat.get() + (size_t)nt * es;
    }
    a.mu = F->mu;
    a.lam = F->lam;
    for (int k = 0; k < 3; ++k) a.X[k] = F->Xc.as<double>() + (size_t)k * nv;
    a.n_inv = F->status.as<unsigned long long>();
    a.tmesh = F->tmesh;
    a.blk_verts = F->blk_verts.as<int32_t>();
    a.blk_row = F->blk_lptr.as<uint16_t>();
    a.blk_stride = (uint32_t)F->blk_maxv;
    a.blk_pos[0] = F->blk_pos.as<uint32_t>();
    a.blk_pos[1] = F->blk_pos.as<uint32_t>() + nt;
    a.blk_hpos = F->blk_hpos.as<int32_t>();
    a.slot[0] = F->blk_local.as<uint32_t>();
    a.slot[1] = F->blk_local.as<uint32_t>() + (F->blk_w == 2 ? nt : 0);
    a.halo = F->halo.as<double>();
    a.nblk = (uint32_t)F->nblk;
    for (int k = 0; k < 3; ++k)
        a.xf[k] = F->blk_xf.get() ? F->blk_xf.as<float>() + (size_t)k * F->nblk * F->blk_maxv : nullptr;
    // a batch deals runs of 64 blocks to the XCDs in turn (see xcd_block; runs of 16, 64
    // and 256 blocks measured 19.0, 19.1 and 19.5 ms per 256-mesh step against 20.8 ms
    // for one range per XCD); one mesh keeps one range per XCD
    a.xcd_run_log2 = F->tmesh ? 6u : 0u;
    a.own_tptr = F->own_tptr.as<int32_t>();
    a.own_meta = F->own_meta.as<uint4>();
    a.own_gptr = F->own_gptr.as<int32_t>();
    a.own_ghost = F->own_ghost.as<int32_t>();
    a.rp = F->group ? F->group->row_ptr.as<int64_t>() : nullptr;
    a.own_vb = (uint32_t)F->own_vb;
    a.own_nblk = (uint32_t)F->own_nblk;
    return a;
}

static void set_vec(const double *(&dst)[3], const double *p, uint32_t nv) {
    for (int k = 0; k < 3; ++k) dst[k] = p ? p + (size_t)k * nv : nullptr;
}

size_t block_shmem(const ebbx_fem_s *F, ElemOp op) {
    const int nq = op == OP_TMUL ? 3 : op == OP_KMUL ? 2 : 1;
    // rest positions staged on blocks of <= 256 vertices: FP32 block-local offsets for FP32
    // elements (3 columns, padded to a multiple of 4 floats), else FP64
    const size_t nx = F->blk_w != 1 ? 0
                      : F->prec == EBBX_F32 ? (((size_t)3 * F->blk_maxv + 3) & ~(size_t)3) * sizeof(float)
                                            : (size_t)3 * F->blk_maxv * sizeof(double);
    const size_t stage = (size_t)3 * nq * F->blk_maxv * sizeof(double) + nx;
    if (F->blk_red == 1) return stage + (size_t)3 * F->blk_maxv * sizeof(double);
    if (F->esize == 8) return std::max(stage, (size_t)12 * F->blk_tets * F->esize);   // rows reuse the staging
    return stage + (size_t)12 * F->blk_tets * F->esize;
}

// LDS a workgroup may allocate on the current device (160 KiB on gfx950).
static size_t lds_limit() {
    int dev = 0, v = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return v > 0 ? (size_t)v : (size_t)64 * 1024;
}

// Sum each shared vertex's halo entries into out (the second pass of the block strategies).
static void launch_halo(ebbx_fem_s *F, const double *hl, double *out, int accumulate, const int *skip, hipStream_t s) {
    if (F->sh_n <= 0) return;
    const int64_t nv = F->nv;
    // one wave per workgroup: the pass is a single round of two dependent loads per vertex, and
    // smaller workgroups measured 0.5 us faster than 256-thread ones (more of them in flight
    // per CU, dealt to the XCDs more finely)
    const unsigned T = 64;
    const dim3 g(grid_n(F->sh_n, T, 1ll << 20));
    const int32_t *sv = F->sh_vert.as<int32_t>();
    const int4 *tb = F->sh_tab.as<int4>();
    const uint32_t sn = (uint32_t)F->sh_n;
    switch (F->sh_nc) {
    case 1: hipLaunchKernelGGL(k_halo_tab<1>, g, dim3(T), 0, s, hl, sv, tb, sn, out, out + nv, out + 2 * nv, accumulate, skip); break;
    case 2: hipLaunchKernelGGL(k_halo_tab<2>, g, dim3(T), 0, s, hl, sv, tb, sn, out, out + nv, out + 2 * nv, accumulate, skip); break;
    case 3: hipLaunchKernelGGL(k_halo_tab<3>, g, dim3(T), 0, s, hl, sv, tb, sn, out, out + nv, out + 2 * nv, accumulate, skip); break;
    case 4: hipLaunchKernelGGL(k_halo_tab<4>, g, dim3(T), 0, s, hl, sv, tb, sn, out, out + nv, out + 2 * nv, accumulate, skip); break;
    default:
        hipLaunchKernelGGL(k_halo_reduce, g, dim3(T), 0, s, hl, sv, F->sh_ptr.as<int32_t>(),
                           F->sh_pos.as<int32_t>(), sn, out, out + nv, out + 2 * nv, accumulate, skip);
    }
    HIPCHK(hipGetLastError());
}

void elem_launch(ebbx_fem_s *F, ElemOp op, const double *d, const double *u, double *out, int accumulate,
                 hipStream_t s, const int *skip, const double *w, const int *mdone, bool finish_halo,
                 void *scratch, const int32_t *act) {
    const int64_t nt = F->nt, nv = F->nv;
    if (nv == 0) return;
    if (nt == 0) {
        if (!accumulate) fill_f64(out, 3 * nv, 0.0, s);
        return;
    }
    ElemArgs a = base_args(F);
    set_vec(a.d, d, (uint32_t)nv);
    set_vec(a.u, u, (uint32_t)nv);
    set_vec(a.w, w, (uint32_t)nv);
    for (int k = 0; k < 3; ++k) a.out[k] = out + (size_t)k * nv;
    a.part = F->part.get();
    if (scratch) {   // the caller's buffer replaces the domain's halo (block strategies) or partials (SEG)
        a.halo = (double *)scratch;
        a.part = scratch;
    }
    a.skip = skip;
    a.mdone = F->tmesh ? mdone : nullptr;
    a.act = F->tmesh ? act : nullptr;
    a.act_nm = (int32_t)F->nm;
    a.accumulate = accumulate;
    if (F->strategy == EBBX_STRAT_OWNER) {
        const int nq = op == OP_TMUL ? 3 : op == OP_KMUL ? 2 : 1;
        const size_t shmem = (size_t)3 * nq * F->own_maxv * sizeof(double) + (size_t)3 * F->own_maxinc * F->esize;
        if (shmem > lds_limit())
            fail(EBBX_E_STATE, "owner strategy needs %zu bytes of LDS per block; use fewer vertices per block",
                 shmem);
        const unsigned grid = (unsigned)F->own_nblk;
        if (F->prec == EBBX_F32) {
            if (F->model == EBBX_STVK) launch_owner<float, EBBX_STVK>(op, a, grid, shmem, s);
            else launch_owner<float, EBBX_NH>(op, a, grid, shmem, s);
        } else {
            if (F->model == EBBX_STVK) launch_owner<double, EBBX_STVK>(op, a, grid, shmem, s);
            else launch_owner<double, EBBX_NH>(op, a, grid, shmem, s);
        }
        return;
    }
    if (F->strategy == EBBX_STRAT_PIPE) {
        const size_t shmem = pipe_shmem(F, op);
        if (shmem > lds_limit())
            fail(EBBX_E_STATE, "pipelined blocks need %zu bytes of LDS per workgroup; use fewer blocks per "
                 "workgroup", shmem);
        launch_pipe(F, op, a, s);
        if (finish_halo) launch_halo(F, a.halo, out, accumulate, skip, s);
        return;
    }
    if (F->strategy == EBBX_STRAT_LANES && op == OP_KMUL) {
        const size_t shmem = lanes_shmem(F);
        if (shmem > lds_limit())
            fail(EBBX_E_STATE, "the multi-lane product needs %zu bytes of LDS per block; use smaller blocks", shmem);
        launch_lanes(F, a, s);
        if (finish_halo) launch_halo(F, a.halo, out, accumulate, skip, s);
        return;
    }
    if (F->strategy == EBBX_STRAT_BLOCK || F->strategy == EBBX_STRAT_BLOCK_LDS || F->strategy == EBBX_STRAT_LANES) {
        const size_t shmem = block_shmem(F, op);
        if (shmem > lds_limit())
            fail(EBBX_E_STATE, "block strategy needs %zu bytes of LDS per block (%d vertices); reorder the mesh "
                 "(Morton) or use smaller blocks", shmem, F->blk_maxv);
        const int tpt = F->blk_tpt, threads = F->blk_tets / tpt;
        if (threads > 512 || tpt > 2) fail(EBBX_E_ARG, "block strategy: at most 1024 tets per block");
        if (a.act && elem_list_ok(F, op)) {
            if (F->prec == EBBX_F32) {
                if (F->model == EBBX_STVK) launch_block_list<float, EBBX_STVK>(F, a, threads, shmem, s);
                else launch_block_list<float, EBBX_NH>(F, a, threads, shmem, s);
            } else {
                if (F->model == EBBX_STVK) launch_block_list<double, EBBX_STVK>(F, a, threads, shmem, s);
                else launch_block_list<double, EBBX_NH>(F, a, threads, shmem, s);
            }
            if (finish_halo) launch_halo(F, a.halo, out, accumulate, skip, s);
            return;
        }
        const unsigned grid = (unsigned)F->nblk;
        if (F->prec == EBBX_F32) {
            if (F->model == EBBX_STVK) launch_model<float, EBBX_STVK>(true, op, 0, tpt, F->blk_w, F->blk_red, a, threads, grid, shmem, s);
            else launch_model<float, EBBX_NH>(true, op, 0, tpt, F->blk_w, F->blk_red, a, threads, grid, shmem, s);
        } else {
            if (F->model == EBBX_STVK) launch_model<double, EBBX_STVK>(true, op, 0, tpt, F->blk_w, F->blk_red, a, threads, grid, shmem, s);
            else launch_model<double, EBBX_NH>(true, op, 0, tpt, F->blk_w, F->blk_red, a, threads, grid, shmem, s);
        }
        if (finish_halo) launch_halo(F, a.halo, out, accumulate, skip, s);
        return;
    }
    const int sc = F->strategy == EBBX_STRAT_SEG ? SC_PART : SC_ATOMIC;
    const int threads = F->block > 0 ? F->block : 256;
    if (sc == SC_ATOMIC && !accumulate) fill_f64(out, 3 * nv, 0.0, s);
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) launch_model<float, EBBX_STVK>(false, op, sc, 1, 1, 0, a, threads, 0, 0, s);
        else launch_model<float, EBBX_NH>(false, op, sc, 1, 1, 0, a, threads, 0, 0, s);
    } else {
        if (F->model == EBBX_STVK) launch_model<double, EBBX_STVK>(false, op, sc, 1, 1, 0, a, threads, 0, 0, s);
        else launch_model<double, EBBX_NH>(false, op, sc, 1, 1, 0, a, threads, 0, 0, s);
    }
    if (sc == SC_PART) {
        const unsigned g = grid_n(nv, 256, 1ll << 31);
        if (F->prec == EBBX_F32)
            hipLaunchKernelGGL(k_seg_gather<float>, dim3(g), dim3(256), 0, s, (const float *)a.part,
                               F->group->row_ptr.as<int64_t>(), F->group->inc.as<int32_t>(), nv, out, accumulate);
        else
            hipLaunchKernelGGL(k_seg_gather<double>, dim3(g), dim3(256), 0, s, (const double *)a.part,
                               F->group->row_ptr.as<int64_t>(), F->group->inc.as<int32_t>(), nv, out, accumulate);
        HIPCHK(hipGetLastError());
    }
}

size_t elem_scratch_bytes(const ebbx_fem_s *F, ElemOp op) {
    if (F->nv == 0 || F->nt == 0) return 0;
    switch (F->strategy) {
    case EBBX_STRAT_SEG: return (size_t)F->nt * 12 * F->esize;
    case EBBX_STRAT_BLOCK:
    case EBBX_STRAT_BLOCK_LDS:
    case EBBX_STRAT_LANES:
    case EBBX_STRAT_PIPE: return (size_t)F->halo_n * 3 * sizeof(double);
    default: (void)op; return 0;   // ATOMIC, OWNER: no scratch
    }
}

// ---- energy ------------------------------------------------------------------------------

template <class T, int MODEL>
__global__ __launch_bounds__(256) void k_energy(ElemArgs a, double *part) {
    __shared__ double s_w[4];
    const uint32_t nt = a.nt;
    double acc = 0.0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
        double b[9];
        for (int k = 0; k < 9; ++k) b[k] = (double)ldc<T>(a.B[k], t);
        const double V0 = (double)ldc<T>(a.V0, t);
        double mu = a.mu, lam = a.lam;
        if (a.mu_t) {
            mu = (double)ldc<T>(a.mu_t, t);
            lam = (double)ldc<T>(a.lam_t, t);
        }
        double q[4][3];
        for (int c = 0; c < 4; ++c) {
            const uint32_t v = (uint32_t)ldc<int32_t>(a.key[c], t);
            for (int k = 0; k < 3; ++k) q[c][k] = ldc<double>(a.d[k], v);
        }
        double G[9];
        grad_from(q, b, G);
        double psi;
        if (MODEL == EBBX_STVK) {
            double GtG[9], E[9];
            mulTN3(G, G, GtG);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) E[3 * i + j] = 0.5 * (G[3 * i + j] + G[3 * j + i] + GtG[3 * i + j]);
            double ee = 0.0;
            for (int k = 0; k < 9; ++k) ee += E[k] * E[k];
            const double tr = E[0] + E[4] + E[8];
            psi = mu * ee + 0.5 * lam * tr * tr;
        } else {
            // psi = mu (2 tr G + tr(G^T G))/2 - mu ln J + lam (ln J)^2 / 2
            double gg = 0.0;
            for (int k = 0; k < 9; ++k) gg += G[k] * G[k];
            const double lnJ = log1p(jm1_of(G));
            psi = 0.5 * mu * (2.0 * (G[0] + G[4] + G[8]) + gg) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
        }
        acc += V0 * psi;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

__global__ void k_sum_parts(const double *part, int n, double *out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

void elem_energy(ebbx_fem_s *F, const double *d, double *out_dev, hipStream_t s) {
    ElemArgs a = base_args(F);
    set_vec(a.d, d, (uint32_t)F->nv);
    const unsigned g = 1024;
    double *part = F->scratch.as<double>();   // scratch holds >= 4096 doubles
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) hipLaunchKernelGGL((k_energy<float, EBBX_STVK>), dim3(g), dim3(256), 0, s, a, part);
        else hipLaunchKernelGGL((k_energy<float, EBBX_NH>), dim3(g), dim3(256), 0, s, a, part);
    } else {
        if (F->model == EBBX_STVK) hipLaunchKernelGGL((k_energy<double, EBBX_STVK>), dim3(g), dim3(256), 0, s, a, part);
        else hipLaunchKernelGGL((k_energy<double, EBBX_NH>), dim3(g), dim3(256), 0, s, a, part);
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double *)part, (int)g, out_dev);
    HIPCHK(hipGetLastError());
}

// ---- gradient with respect to per-tet Young's modulus ------------------------------------------
//
// Forces and stiffness are linear in (mu, lam), and both are proportional to
// E at fixed nu, so d(f_t)/dE_t = f_t / E_t and d(K_t)/dE_t = K_t / E_t:
//   E_bar[t] += w_t . (dt f_t + dt^2 K_t v) / E_t.
template <class T, int MODEL>
__global__ __launch_bounds__(256) void k_egrad(ElemArgs a, const double *E_tet, double E, double cf, double ck,
                                               double *E_bar) {
    const uint32_t nt = a.nt;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    T b[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) b[k] = ldc<T>(a.B[k], t);
    const T V0 = tet_V0(b);
    T mu, lam;
    if (a.mu_t) {
        mu = ldc<T>(a.mu_t, t);
        lam = ldc<T>(a.lam_t, t);
    } else {
        mu = (T)a.mu;
        lam = (T)a.lam;
    }
    uint32_t v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (uint32_t)ldc<int32_t>(a.key[c], t);
    const bool with_k = ck != 0.0;   // uniform: the stiffness term (and its direction) is optional
    double qd[4][3], qv[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            qd[c][k] = ldc<double>(a.d[k], v[c]);
            qv[c][k] = with_k ? ldc<double>(a.u[k], v[c]) : 0.0;
        }
    T G[9], dF[9], P[9], dP[9], hf[12], hk[12];
    grad_from(qd, b, G);
    stress_scaled<T, MODEL>(mu, lam, V0, G, P);
    corner_out(P, b, hf);
    if (with_k) {
        grad_from(qv, b, dF);
        dstress_scaled<T, MODEL>(mu, lam, V0, G, dF, dP);
        corner_out(dP, b, hk);
    } else {
#pragma unroll
        for (int j = 0; j < 12; ++j) hk[j] = (T)0;
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            acc += ldc<double>(a.w[k], v[c]) * (cf * (double)hf[3 * c + k] + ck * (double)hk[3 * c + k]);
    const double Et = E_tet ? E_tet[t] : E;
    E_bar[t] += acc / Et;
}

void elem_egrad(ebbx_fem_s *F, const double *d, const double *v, const double *w, double cf, double ck,
                double *E_bar, hipStream_t s) {
    if (F->nt == 0) return;
    ElemArgs a = base_args(F);
    set_vec(a.d, d, (uint32_t)F->nv);
    set_vec(a.u, v, (uint32_t)F->nv);
    set_vec(a.w, w, (uint32_t)F->nv);
    const unsigned g = grid_n(F->nt, 256, 1ll << 31);
    const double *Et = F->per_tet ? F->E_tet : nullptr;
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) hipLaunchKernelGGL((k_egrad<float, EBBX_STVK>), dim3(g), dim3(256), 0, s, a, Et, F->E, cf, ck, E_bar);
        else hipLaunchKernelGGL((k_egrad<float, EBBX_NH>), dim3(g), dim3(256), 0, s, a, Et, F->E, cf, ck, E_bar);
    } else {
        if (F->model == EBBX_STVK) hipLaunchKernelGGL((k_egrad<double, EBBX_STVK>), dim3(g), dim3(256), 0, s, a, Et, F->E, cf, ck, E_bar);
        else hipLaunchKernelGGL((k_egrad<double, EBBX_NH>), dim3(g), dim3(256), 0, s, a, Et, F->E, cf, ck, E_bar);
    }
    HIPCHK(hipGetLastError());
}

template <class T>
__global__ void k_material(const double *E_tet, const double *nu_tet, double E, double nu, int64_t nt, T *mat) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const double Et = E_tet ? E_tet[t] : E, nt_ = nu_tet ? nu_tet[t] : nu;
        mat[t] = (T)(Et / (2.0 * (1.0 + nt_)));
        mat[nt + t] = (T)(Et * nt_ / ((1.0 + nt_) * (1.0 - 2.0 * nt_)));
    }
}

void elem_set_material(ebbx_fem_s *F, const double *E_tet, const double *nu_tet, double E, double nu, hipStream_t s) {
    const int64_t nt = std::max<int64_t>(F->nt, 1);
    if (!F->mat.get()) F->mat.reset((size_t)nt * 2 * F->esize, s);
    F->per_tet = true;
    F->E_tet = E_tet;
    F->E = E;
    F->nu = nu;
    if (F->nt == 0) return;
    const unsigned g = grid_n(F->nt, 256, 16384);
    if (F->prec == EBBX_F32)
        hipLaunchKernelGGL(k_material<float>, dim3(g), dim3(256), 0, s, E_tet, nu_tet, E, nu, F->nt, F->mat.as<float>());
    else
        hipLaunchKernelGGL(k_material<double>, dim3(g), dim3(256), 0, s, E_tet, nu_tet, E, nu, F->nt, F->mat.as<double>());
    HIPCHK(hipGetLastError());
}

// ---- rest-shape precompute -----------------------------------------------------------------

template <class T>
__global__ void k_precompute(const double *X, const int32_t *keys, int64_t nt, int64_t nv, const double *E_tet,
                             double E, double nu, T *B, T *V0, T *mat, double *V0d, unsigned long long *n_bad) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        double x[4][3];
        for (int c = 0; c < 4; ++c) {
            const int64_t v = keys[c * nt + t];
            for (int k = 0; k < 3; ++k) x[c][k] = X[k * nv + v];
        }
        double Dm[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Dm[3 * r + c] = x[c + 1][r] - x[0][r];
        const double det = det3(Dm);
        V0d[t] = det / 6.0;
        if (!(det > 0.0)) {
            atomicAdd(n_bad, 1ull);
            for (int k = 0; k < 9; ++k) B[k * nt + t] = (T)0;
            V0[t] = (T)0;
            continue;
        }
        // B = Dm^-1 = adj(Dm) / det
        double C[9];
        C[0] = Dm[4] * Dm[8] - Dm[5] * Dm[7];
        C[1] = Dm[2] * Dm[7] - Dm[1] * Dm[8];
        C[2] = Dm[1] * Dm[5] - Dm[2] * Dm[4];
        C[3] = Dm[5] * Dm[6] - Dm[3] * Dm[8];
        C[4] = Dm[0] * Dm[8] - Dm[2] * Dm[6];
        C[5] = Dm[2] * Dm[3] - Dm[0] * Dm[5];
        C[6] = Dm[3] * Dm[7] - Dm[4] * Dm[6];
        C[7] = Dm[1] * Dm[6] - Dm[0] * Dm[7];
        C[8] = Dm[0] * Dm[4] - Dm[1] * Dm[3];
        for (int k = 0; k < 9; ++k) B[k * nt + t] = (T)(C[k] / det);
        V0[t] = (T)(det / 6.0);
        if (mat) {
            const double Et = E_tet ? E_tet[t] : E;
            mat[t] = (T)(Et / (2.0 * (1.0 + nu)));
            mat[nt + t] = (T)(Et * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)));
        }
    }
}

// m_v = sum over the vertex's incidences (in grouping order) of rho V0 / 4
__global__ void k_lumped_mass(const double *V0d, const int64_t *row_ptr, const int32_t *inc, int64_t nv, double rho,
                              double *mass) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        double m = 0.0;
        for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) m += rho * V0d[inc[j] >> 2] / 4.0;
        mass[v] = m;
    }
}

int64_t elem_precompute(ebbx_fem_s *F, const double *X, const double *E_tet, hipStream_t s) {
    const int64_t nt = F->nt, nv = F->nv;
    DevBuf V0d((size_t)std::max<int64_t>(nt, 1) * sizeof(double), s);
    DevBuf bad(sizeof(unsigned long long), s);
    HIPCHK(hipMemsetAsync(bad.get(), 0, sizeof(unsigned long long), s));
    if (nt > 0) {
        const unsigned g = grid_n(nt, 256, 16384);
        if (F->prec == EBBX_F32)
            hipLaunchKernelGGL(k_precompute<float>, dim3(g), dim3(256), 0, s, X, F->keys, nt, nv, E_tet, F->E, F->nu,
                               F->B.as<float>(), F->V0.as<float>(), F->per_tet ? F->mat.as<float>() : nullptr,
                               V0d.as<double>(), bad.as<unsigned long long>());
        else
            hipLaunchKernelGGL(k_precompute<double>, dim3(g), dim3(256), 0, s, X, F->keys, nt, nv, E_tet, F->E, F->nu,
                               F->B.as<double>(), F->V0.as<double>(), F->per_tet ? F->mat.as<double>() : nullptr,
                               V0d.as<double>(), bad.as<unsigned long long>());
        HIPCHK(hipGetLastError());
    }
    if (nv > 0) {
        hipLaunchKernelGGL(k_lumped_mass, dim3(grid_n(nv, 256, 16384)), dim3(256), 0, s, (const double *)V0d.get(),
                           F->group->row_ptr.as<int64_t>(), F->group->inc.as<int32_t>(), nv, F->rho,
                           F->mass.as<double>());
        HIPCHK(hipGetLastError());
    }
    unsigned long long hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, bad.get(), sizeof hb, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return (int64_t)hb;
}

HaloView elem_halo_view(const ebbx_fem_s *F) {
    HaloView h{};
    const bool block = F->strategy == EBBX_STRAT_BLOCK || F->strategy == EBBX_STRAT_BLOCK_LDS ||
                       F->strategy == EBBX_STRAT_PIPE || F->strategy == EBBX_STRAT_LANES;
    if (!block || F->sh_n == 0 || F->nt == 0) return h;
    h.row = F->sh_row.as<int32_t>();
    h.tab = F->sh_tab.as<int4>();
    h.ptr = F->sh_ptr.as<int32_t>();
    h.pos = F->sh_pos.as<int32_t>();
    h.halo = F->halo.as<double>();
    h.nc = F->sh_nc;
    return h;
}

bool elem_pre_ok(const ebbx_fem_s *F) {
    return F->strategy == EBBX_STRAT_BLOCK && F->blk_red == 0 && F->blk_tpt == 1 && F->halo_level == 0 &&
           F->nt > 0 && F->nv > 0;
}

void elem_pre_prepare(ebbx_fem_s *F, hipStream_t s) {
    const size_t bytes = std::max<size_t>((size_t)F->halo_n * 9 * sizeof(double), 8);
    if (F->halo9.bytes() != bytes) F->halo9.reset(bytes, s);
}

HaloView elem_pre_halo(const ebbx_fem_s *F) {
    HaloView h = elem_halo_view(F);
    if (h.row) h.halo = F->halo9.as<double>();
    return h;
}

void elem_launch_pre(ebbx_fem_s *F, const double *d, const double *u, double *f, double *y, double *diag,
                     hipStream_t s) {
    if (!elem_pre_ok(F)) fail(EBBX_E_STATE, "the fused step preamble needs the block strategy (one tet per thread)");
    const size_t need = (size_t)F->halo_n * 9 * sizeof(double);
    if (F->halo9.bytes() < std::max<size_t>(need, 8)) fail(EBBX_E_STATE, "the fused step preamble's halo is not allocated");
    const int64_t nv = F->nv;
    ElemArgs a = base_args(F);
    set_vec(a.d, d, (uint32_t)nv);
    set_vec(a.u, u, (uint32_t)nv);
    double *outs[3] = {f, y, diag};
    for (int ph = 0; ph < 3; ++ph)
        for (int k = 0; k < 3; ++k) a.pre_out[ph][k] = outs[ph] + (size_t)k * nv;
    a.halo9 = F->halo9.as<double>();
    const size_t shmem = block_shmem(F, OP_KMUL);   // d and u staged, one row set
    if (shmem > lds_limit())
        fail(EBBX_E_STATE, "block strategy needs %zu bytes of LDS per block (%d vertices); reorder the mesh "
             "(Morton) or use smaller blocks", shmem, F->blk_maxv);
    const int threads = F->blk_tets;
    if (threads > 512) fail(EBBX_E_ARG, "block strategy: at most 512 tets per block with one tet per thread");
    const dim3 g((unsigned)F->nblk), b((unsigned)threads);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, shmem, s, a); };
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) {
            if (F->blk_w == 1) go(k_block_pre<float, EBBX_STVK, 1>);
            else go(k_block_pre<float, EBBX_STVK, 2>);
        } else {
            if (F->blk_w == 1) go(k_block_pre<float, EBBX_NH, 1>);
            else go(k_block_pre<float, EBBX_NH, 2>);
        }
    } else {
        if (F->model == EBBX_STVK) {
            if (F->blk_w == 1) go(k_block_pre<double, EBBX_STVK, 1>);
            else go(k_block_pre<double, EBBX_STVK, 2>);
        } else {
            if (F->blk_w == 1) go(k_block_pre<double, EBBX_NH, 1>);
            else go(k_block_pre<double, EBBX_NH, 2>);
        }
    }
    HIPCHK(hipGetLastError());
}

// ---- block tables -----------------------------------------------------------------------

// Tets are cut into blocks of bt consecutive rows.  Per block: the sorted set of
// vertices it touches, each corner's slot in that set, the block's incidences
// ordered by (vertex, local tet, corner) with each corner's row in that order
// and each vertex's run of rows, and whether the block holds every incident tet
// of the vertex.
HostBlocks host_blocks(const std::vector<int32_t> &keys, const std::vector<int64_t> &rp, int64_t nt, int32_t bt) {
    HostBlocks hb;
    const int64_t nblk = (nt + bt - 1) / bt;
    hb.bt = bt;
    hb.nblk = nblk;
    hb.vptr.assign((size_t)nblk + 1, 0);
    hb.lptr.assign(1, 0);
    std::vector<uint16_t> local((size_t)(4 * nt)), rowpos((size_t)(4 * nt));
    int64_t list_n = 0;   // incidence rows so far (all blocks)
    hb.verts.reserve((size_t)(nt + 16));
    hb.own.reserve((size_t)(nt + 16));
    hb.lptr.reserve((size_t)(nt + 16));
    std::vector<std::pair<int32_t, int32_t>> buf;   // (vertex, local tet * 4 + corner)
    int32_t maxv = 1;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t t0 = b * bt, t1 = std::min<int64_t>(nt, t0 + bt);
        const int64_t list_b0 = list_n;
        buf.clear();
        for (int64_t t = t0; t < t1; ++t)
            for (int c = 0; c < 4; ++c) buf.push_back({keys[(size_t)(c * nt + t)], (int32_t)(4 * (t - t0) + c)});
        std::sort(buf.begin(), buf.end());
        int32_t nb = 0;
        size_t i = 0;
        while (i < buf.size()) {
            size_t j = i;
            while (j < buf.size() && buf[j].first == buf[i].first) ++j;
            const int32_t v = buf[i].first;
            for (size_t k = i; k < j; ++k) {
                const int32_t tl = buf[k].second >> 2, c = buf[k].second & 3;
                local[(size_t)(c * nt + t0 + tl)] = (uint16_t)nb;
                rowpos[(size_t)(c * nt + t0 + tl)] = (uint16_t)(list_n - list_b0);   // row in the block
                ++list_n;
            }
            hb.verts.push_back(v);
            hb.lptr.push_back((int32_t)list_n);
            hb.own.push_back((int64_t)(j - i) == rp[(size_t)v + 1] - rp[(size_t)v] ? 1 : 0);
            ++nb;
            i = j;
        }
        maxv = std::max(maxv, nb);
        hb.vptr[(size_t)b + 1] = (int32_t)hb.verts.size();
        if (hb.verts.size() >= (size_t)(1u << 31)) fail(EBBX_E_ARG, "block tables exceed int32");
    }
    if (maxv > 65535) fail(EBBX_E_ARG, "a block touches %d vertices (limit 65535)", maxv);
    if (list_n >= (int64_t(1) << 31)) fail(EBBX_E_ARG, "block tables exceed int32");
    hb.maxv = maxv;
    // per tet: the rows of its four corners in its block's incidence order
    hb.pos.assign((size_t)(2 * std::max<int64_t>(nt, 1)), 0u);
    for (int64_t t = 0; t < nt; ++t) {
        hb.pos[(size_t)t] = (uint32_t)rowpos[(size_t)t] | ((uint32_t)rowpos[(size_t)(nt + t)] << 16);
        hb.pos[(size_t)(nt + t)] =
            (uint32_t)rowpos[(size_t)(2 * nt + t)] | ((uint32_t)rowpos[(size_t)(3 * nt + t)] << 16);
    }
    // packed slots: 4 x 8 bits per word if every block has <= 256 vertices
    const int w = maxv <= 256 ? 1 : 2;
    hb.w = w;
    hb.packed.assign((size_t)(w * std::max<int64_t>(nt, 1)), 0u);
    for (int64_t t = 0; t < nt; ++t) {
        const uint32_t s0 = local[(size_t)t], s1 = local[(size_t)(nt + t)], s2 = local[(size_t)(2 * nt + t)],
                       s3 = local[(size_t)(3 * nt + t)];
        if (w == 1) {
            hb.packed[(size_t)t] = s0 | (s1 << 8) | (s2 << 16) | (s3 << 24);
        } else {
            hb.packed[(size_t)t] = s0 | (s1 << 16);
            hb.packed[(size_t)(nt + t)] = s2 | (s3 << 16);
        }
    }
    return hb;
}

void upload(DevBuf &dst, const void *src, size_t bytes, hipStream_t s) {
    dst.reset(std::max<size_t>(bytes, 16), s);
    if (bytes) HIPCHK(hipMemcpy(dst.get(), src, bytes, hipMemcpyHostToDevice));
}

// Halo entries are unit-major (each unit writes one contiguous run); every
// shared (or untouched) vertex lists its entries, which ascend in unit order,
// and vertices that no tet touches get an empty run, so the halo pass zeroes
// them.  verts/own: the vertex lists of the units (blocks or super-blocks) in
// unit order; hpos receives each list entry's halo position or -1.
void build_halo(ebbx_fem_s *F, const std::vector<int32_t> &verts, const std::vector<uint8_t> &own,
                const std::vector<int64_t> &rp, std::vector<int32_t> &hpos, hipStream_t s) {
    const int64_t nv = F->nv;
    hpos.assign(verts.size(), -1);
    int32_t nh = 0;
    for (size_t p = 0; p < verts.size(); ++p)
        if (!own[p]) hpos[p] = nh++;
    std::vector<int32_t> count((size_t)nv, 0);
    for (size_t p = 0; p < verts.size(); ++p)
        if (!own[p]) ++count[(size_t)verts[p]];
    std::vector<int32_t> sh_vert, sh_ptr(1, 0), row((size_t)nv, -1);
    for (int64_t v = 0; v < nv; ++v) {
        const bool isolated = rp[(size_t)v + 1] == rp[(size_t)v];
        if (count[(size_t)v] > 0 || isolated) {
            row[(size_t)v] = (int32_t)sh_vert.size();
            sh_vert.push_back((int32_t)v);
            sh_ptr.push_back(sh_ptr.back() + count[(size_t)v]);
        }
    }
    std::vector<int32_t> sh_pos((size_t)nh), fillc(sh_vert.size(), 0);
    for (size_t p = 0; p < verts.size(); ++p)
        if (!own[p]) {
            const int32_t r = row[(size_t)verts[p]];
            sh_pos[(size_t)(sh_ptr[(size_t)r] + fillc[(size_t)r]++)] = hpos[p];
        }
    F->sh_n = (int64_t)sh_vert.size();
    F->halo_n = (int64_t)nh;
    upload(F->sh_vert, sh_vert.data(), sh_vert.size() * sizeof(int32_t), s);
    upload(F->sh_ptr, sh_ptr.data(), sh_ptr.size() * sizeof(int32_t), s);
    upload(F->sh_pos, sh_pos.data(), sh_pos.size() * sizeof(int32_t), s);
    // per vertex: its row in the shared-vertex table, or -1 (a unit stores it)
    std::vector<int32_t> shrow((size_t)std::max<int64_t>(nv, 1), -1);
    for (size_t r = 0; r < sh_vert.size(); ++r) shrow[(size_t)sh_vert[r]] = (int32_t)r;
    upload(F->sh_row, shrow.data(), shrow.size() * sizeof(int32_t), s);
    // fixed-width rows of halo positions when no vertex has more than 16 entries
    int32_t maxm = 0;
    for (size_t r = 0; r + 1 < sh_ptr.size(); ++r) maxm = std::max(maxm, sh_ptr[r + 1] - sh_ptr[r]);
    F->sh_nc = maxm <= 16 ? std::max(1, (maxm + 3) / 4) : 0;
    if (F->sh_nc > 0) {
        const size_t w = (size_t)4 * F->sh_nc;
        std::vector<int32_t> tab(std::max<size_t>(sh_vert.size() * w, 4), -1);
        for (size_t r = 0; r < sh_vert.size(); ++r)
            for (int32_t j = sh_ptr[r]; j < sh_ptr[r + 1]; ++j) tab[r * w + (size_t)(j - sh_ptr[r])] = sh_pos[(size_t)j];
        upload(F->sh_tab, tab.data(), tab.size() * sizeof(int32_t), s);
    }
    F->halo.reset(std::max<size_t>((size_t)F->halo_n * 3 * sizeof(double), 8), s);
}

// Upload the block tables (without the halo): fixed-stride copies, block b's
// vertices at [b*maxv, (b+1)*maxv) padded with -1 (halo positions hpos alike) and
// its block-relative row starts at [b*(maxv+1), (b+1)*(maxv+1)); per tet the corner
// rows and the packed slots.
// Block-local FP32 rest positions: entry (b, i) holds X of block b's i-th vertex minus X of its
// first vertex, rounded to FP32 (three columns of nblk * S entries; padding 0).
__global__ void k_block_xf(const double *X, int64_t nv, const int32_t *bverts, int64_t n, uint32_t S, float *xf) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = bverts[e], v0 = bverts[(e / S) * S];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            xf[(int64_t)k * n + e] = v >= 0 ? (float)(X[(int64_t)k * nv + v] - X[(int64_t)k * nv + v0]) : 0.0f;
    }
}

void upload_block_tables(ebbx_fem_s *F, const HostBlocks &hb, const std::vector<int32_t> &hpos, hipStream_t s) {
    const int64_t nblk = hb.nblk;
    const size_t S = (size_t)hb.maxv;
    std::vector<int32_t> pverts((size_t)nblk * S, -1), phpos((size_t)nblk * S, -1);
    std::vector<uint16_t> prow((size_t)nblk * (S + 1), 0);
    for (int64_t b = 0; b < nblk; ++b) {
        const int32_t a0 = hb.vptr[(size_t)b], a1 = hb.vptr[(size_t)b + 1];
        const int32_t base = hb.lptr[(size_t)a0], tot = hb.lptr[(size_t)a1] - base;
        for (size_t i = 0; i <= S; ++i) {
            const int32_t k = a0 + (int32_t)i;
            if (k < a1) {
                pverts[(size_t)b * S + i] = hb.verts[(size_t)k];
                if (!hpos.empty()) phpos[(size_t)b * S + i] = hpos[(size_t)k];
                prow[(size_t)b * (S + 1) + i] = (uint16_t)(hb.lptr[(size_t)k] - base);
            } else {
                prow[(size_t)b * (S + 1) + i] = (uint16_t)tot;
            }
        }
    }
    upload(F->blk_vptr, hb.vptr.data(), hb.vptr.size() * sizeof(int32_t), s);
    upload(F->blk_verts, pverts.data(), pverts.size() * sizeof(int32_t), s);
    upload(F->blk_lptr, prow.data(), prow.size() * sizeof(uint16_t), s);
    upload(F->blk_pos, hb.pos.data(), hb.pos.size() * sizeof(uint32_t), s);
    upload(F->blk_hpos, phpos.data(), phpos.size() * sizeof(int32_t), s);
    upload(F->blk_local, hb.packed.data(), hb.packed.size() * sizeof(uint32_t), s);
    F->blk_tets = hb.bt;
    F->nblk = nblk;
    F->blk_maxv = hb.maxv;
    F->blk_w = hb.w;
    F->blk_nverts = (int64_t)hb.verts.size();
    // FP32 elements on blocks of at most 256 vertices read block-local FP32 rest positions
    if (F->prec == EBBX_F32 && hb.w == 1 && nblk > 0) {
        const int64_t n = nblk * (int64_t)S;
        F->blk_xf.reset((size_t)n * 3 * sizeof(float), s);
        hipLaunchKernelGGL(k_block_xf, dim3(grid_n(n, 256, 16384)), dim3(256), 0, s, F->Xc.as<double>(), F->nv,
                           F->blk_verts.as<int32_t>(), n, (uint32_t)S, F->blk_xf.as<float>());
        HIPCHK(hipGetLastError());
    } else {
        F->blk_xf.release();
    }
}

void download_keys(const ebbx_fem_s *F, std::vector<int32_t> &keys, std::vector<int64_t> &rp) {
    keys.resize((size_t)(4 * F->nt));
    if (F->nt > 0) HIPCHK(hipMemcpy(keys.data(), F->keys, keys.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    rp.resize((size_t)(F->nv + 1));
    HIPCHK(hipMemcpy(rp.data(), F->group->row_ptr.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
}

// The BLOCK tables with a halo of the blocks' shared vertices.
void build_blocks(ebbx_fem_s *F, int32_t bt, hipStream_t s) {
    if (bt < 64 || bt > 1024 || bt % 64)
        fail(EBBX_E_ARG, "block strategy: tets per block must be a multiple of 64 from 64 to 1024 (got %d)", bt);
    std::vector<int32_t> keys;
    std::vector<int64_t> rp;
    download_keys(F, keys, rp);
    const HostBlocks hb = host_blocks(keys, rp, F->nt, bt);
    std::vector<int32_t> hpos;
    build_halo(F, hb.verts, hb.own, rp, hpos, s);
    upload_block_tables(F, hb, hpos, s);
    F->halo_level = 0;
    F->blocks_built = true;
}

// OWNER tables.  Block b owns vertices [b*vb, min(nv, (b+1)*vb)).  Its tets are
// every tet incident to an owned vertex (ascending ids); its staged vertices
// are the owned ones (local ids 0..nown-1) then the other vertices of its
// tets (ascending).  The owned incidences, in the grouping's order (vertex,
// then tet, then corner), give each owned corner of a listed tet its row in
// the block's sum buffer; the kernel needs no other reduction metadata.
void build_owner(ebbx_fem_s *F, int32_t vb, hipStream_t s) {
    const int64_t nt = F->nt, nv = F->nv;
    if (vb != 64 && vb != 128 && vb != 256)
        fail(EBBX_E_ARG, "owner strategy: owned vertices per block must be 64, 128 or 256 (got %d)", vb);
    const int64_t nblk = std::max<int64_t>(1, (nv + vb - 1) / vb);
    std::vector<int32_t> keys((size_t)(4 * nt));
    if (nt > 0) HIPCHK(hipMemcpy(keys.data(), F->keys, keys.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> rp((size_t)(nv + 1));
    HIPCHK(hipMemcpy(rp.data(), F->group->row_ptr.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> inc((size_t)(4 * nt));
    if (nt > 0) HIPCHK(hipMemcpy(inc.data(), F->group->inc.get(), inc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> tptr((size_t)nblk + 1, 0), gptr((size_t)nblk + 1, 0), ghost;
    std::vector<uint32_t> meta;   // 4 words per (block, tet)
    std::vector<int32_t> tl, gl;
    std::vector<uint32_t> pos;
    int32_t maxv = 1, maxinc = 1;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t v0 = std::min<int64_t>(nv, b * vb), v1 = std::min<int64_t>(nv, v0 + vb);
        const int64_t r0 = rp[(size_t)v0], r1 = rp[(size_t)v1];
        tl.clear();
        for (int64_t e = r0; e < r1; ++e) tl.push_back(inc[(size_t)e] >> 2);
        std::sort(tl.begin(), tl.end());
        tl.erase(std::unique(tl.begin(), tl.end()), tl.end());
        gl.clear();
        for (int32_t t : tl)
            for (int c = 0; c < 4; ++c) {
                const int32_t v = keys[(size_t)(c * nt + t)];
                if (v < v0 || v >= v1) gl.push_back(v);
            }
        std::sort(gl.begin(), gl.end());
        gl.erase(std::unique(gl.begin(), gl.end()), gl.end());
        const int64_t nvb = (v1 - v0) + (int64_t)gl.size(), ninc = r1 - r0;
        if (nvb > 2047) fail(EBBX_E_ARG, "owner block %lld stages %lld vertices (limit 2047); use fewer per block",
                             (long long)b, (long long)nvb);
        if (ninc > 8190) fail(EBBX_E_ARG, "owner block %lld has %lld owned incidences (limit 8190)", (long long)b,
                              (long long)ninc);
        maxv = std::max<int32_t>(maxv, (int32_t)nvb);
        maxinc = std::max<int32_t>(maxinc, (int32_t)ninc);
        pos.assign(4 * tl.size(), 0x1fffu);
        for (int64_t e = r0; e < r1; ++e) {
            const int32_t t = inc[(size_t)e] >> 2, c = inc[(size_t)e] & 3;
            const size_t j = (size_t)(std::lower_bound(tl.begin(), tl.end(), t) - tl.begin());
            pos[4 * j + c] = (uint32_t)(e - r0);
        }
        for (size_t j = 0; j < tl.size(); ++j) {
            const int32_t t = tl[j];
            uint32_t cw[4];
            for (int c = 0; c < 4; ++c) {
                const int32_t v = keys[(size_t)(c * nt + t)];
                const uint32_t sl = (v >= v0 && v < v1)
                                        ? (uint32_t)(v - v0)
                                        : (uint32_t)((v1 - v0) + (std::lower_bound(gl.begin(), gl.end(), v) - gl.begin()));
                cw[c] = sl | (pos[4 * j + c] << 11);
            }
            const uint64_t lo = (uint64_t)cw[0] | ((uint64_t)cw[1] << 24) | ((uint64_t)(cw[2] & 0xffffu) << 48);
            meta.push_back((uint32_t)t);
            meta.push_back((uint32_t)lo);
            meta.push_back((uint32_t)(lo >> 32));
            meta.push_back((cw[2] >> 16) | (cw[3] << 8));
        }
        ghost.insert(ghost.end(), gl.begin(), gl.end());
        if (meta.size() / 4 >= (size_t)(1u << 31) || ghost.size() >= (size_t)(1u << 31))
            fail(EBBX_E_ARG, "owner tables exceed int32");
        tptr[(size_t)b + 1] = (int32_t)(meta.size() / 4);
        gptr[(size_t)b + 1] = (int32_t)ghost.size();
    }
    F->own_vb = vb;
    F->own_nblk = nblk;
    F->own_maxv = maxv;
    F->own_maxinc = maxinc;
    F->own_ntb = (int64_t)(meta.size() / 4);
    auto up = [&](DevBuf &dst, const void *src, size_t bytes) {
        dst.reset(std::max<size_t>(bytes, 16), s);
        if (bytes) HIPCHK(hipMemcpy(dst.get(), src, bytes, hipMemcpyHostToDevice));
    };
    up(F->own_tptr, tptr.data(), tptr.size() * sizeof(int32_t));
    up(F->own_meta, meta.data(), meta.size() * sizeof(uint32_t));
    up(F->own_gptr, gptr.data(), gptr.size() * sizeof(int32_t));
    up(F->own_ghost, ghost.data(), ghost.size() * sizeof(int32_t));
}

}  // namespace ebbx
