// lanes.hip -- the stiffness product with several lanes per tet (the LANES strategy).
//
// The paper's discussion of its GPU code generation notes that per-element matrix work is
// register-heavy and that splitting one element's work over several threads is a way to
// relieve it.  Here a quad of four consecutive lanes evaluates one tet of the stiffness
// product K u: lane r (0, 1, 2) owns row r (spatial component r) of every 3x3 quantity -- it
// gathers component r of d and u at the four corners from the block's staged fields, forms
// row r of G and of dF, and writes component r of the four corner results -- and the sums
// over rows that the material laws need (F^T F and sym(F^T dF) for StVK; dF^T N and N : dF
// for neo-Hookean) are reduced across the quad with DPP quad permutations, so every lane
// holds the same sums bit for bit.  Lane 3 repeats row 2's work and writes nothing.  The
// block tables, staging, incidence-order rows, run sums and halo are those of the BLOCK
// strategy (blocks of bt tets on 4 bt threads); the other element maps of a LANES domain
// use the BLOCK kernels.
#include <algorithm>

#include "fem.h"
#include "tetmath.h"

namespace ebbx {

namespace {

// DPP quad permutation: lane i of each group of four reads lane sel_i (CTRL = sel_0 |
// sel_1 << 2 | sel_2 << 4 | sel_3 << 6).
template <int CTRL> __device__ __forceinline__ float qperm(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double qperm(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int Q_XOR1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);   // [1, 0, 3, 2]
constexpr int Q_XOR2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);   // [2, 3, 0, 1]
// the next rows of the row each lane owns (lane 3 owns row 2): rows (r+1) mod 3 and (r+2) mod 3
constexpr int Q_NEXT1 = 1 | (2 << 2) | (0 << 4) | (0 << 6);   // [1, 2, 0, 0]
constexpr int Q_NEXT2 = 2 | (0 << 2) | (1 << 4) | (1 << 6);   // [2, 0, 1, 1]

// Sum over rows 0..2 of the quad (lane 3's copy of row 2 excluded), the same in all lanes:
// (x0 + x1) + (x2 + 0), added in the same pairs in every lane.
template <class T> __device__ __forceinline__ T quad_rows_sum(T x, bool mirror) {
    const T own = mirror ? T(0) : x;
    const T s = own + qperm<Q_XOR1>(own);
    return s + qperm<Q_XOR2>(s);
}

// Row r of -V0 dP B^T for the stiffness product, with every lane of the quad holding row r of
// G and dF (Gr, dFr); returns false for an inverted neo-Hookean element.  H[c] is component r
// of corner c + 1's result; corner 0 gets minus their sum.
template <class T, int MODEL>
__device__ __forceinline__ bool kmul_row(T mu, T lam, T V0, const T *b, const T *Gr, const T *dFr, int r,
                                         bool mirror, T *H) {
    // (register arrays are indexed by compile-time positions only, selecting on r)
    const T Fr[3] = {Gr[0] + (r == 0 ? T(1) : T(0)), Gr[1] + (r == 1 ? T(1) : T(0)), Gr[2] + (r == 2 ? T(1) : T(0))};
    T dPr[3];
    bool ok = true;
    if (MODEL == EBBX_STVK) {
        // 2E = G + G^T + G^T G and Y = F^T dF + dF^T F (symmetric, six entries each) summed
        // over rows; row r adds G_r[b] to entry (r, b) and G_r[a] to (a, r) of G + G^T, so E
        // keeps the displacement-gradient form (no F^T F - I cancellation)
        const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
        T E2[6], Y[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const T lin = (r == ia[k] ? Gr[ib[k]] : T(0)) + (r == ib[k] ? Gr[ia[k]] : T(0));
            E2[k] = quad_rows_sum(lin + Gr[ia[k]] * Gr[ib[k]], mirror);
            Y[k] = quad_rows_sum(Fr[ia[k]] * dFr[ib[k]] + Fr[ib[k]] * dFr[ia[k]], mirror);
        }
        // S = 2 mu E + lam tr(E) I;  dS = mu Y + lam/2 tr(Y) I
        const T trE = T(0.5) * (E2[0] + E2[1] + E2[2]);
        const T trY = Y[0] + Y[1] + Y[2];
        T S[9], dS[9];
        S[0] = mu * E2[0] + lam * trE;
        S[4] = mu * E2[1] + lam * trE;
        S[8] = mu * E2[2] + lam * trE;
        S[1] = S[3] = mu * E2[3];
        S[2] = S[6] = mu * E2[4];
        S[5] = S[7] = mu * E2[5];
        dS[0] = mu * Y[0] + T(0.5) * lam * trY;
        dS[4] = mu * Y[1] + T(0.5) * lam * trY;
        dS[8] = mu * Y[2] + T(0.5) * lam * trY;
        dS[1] = dS[3] = mu * Y[3];
        dS[2] = dS[6] = mu * Y[4];
        dS[5] = dS[7] = mu * Y[5];
        // row r of dF S + F dS
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dPr[j] = dFr[0] * S[j] + dFr[1] * S[3 + j] + dFr[2] * S[6 + j] + Fr[0] * dS[j] + Fr[1] * dS[3 + j] +
                     Fr[2] * dS[6 + j];
    } else {
        // every lane takes the other two rows of G: J - 1 from the whole G (free of
        // cancellation), row r of cof(F) = F_{r+1} x F_{r+2}
        T G1[3], G2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            G1[k] = qperm<Q_NEXT1>(Gr[k]);
            G2[k] = qperm<Q_NEXT2>(Gr[k]);
        }
        const int r1 = r == 2 ? 0 : r + 1, r2 = r == 0 ? 2 : r - 1;
        T G[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) G[3 * i + k] = r == i ? Gr[k] : (r1 == i ? G1[k] : G2[k]);
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T iJ = t_rcp(J);
        const T lnJ = t_log1p(jm1);
        T F1[3], F2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            F1[k] = G1[k] + (r1 == k ? T(1) : T(0));
            F2[k] = G2[k] + (r2 == k ? T(1) : T(0));
        }
        // N = F^-T = cof(F) / J, row r
        const T Nr[3] = {(F1[1] * F2[2] - F1[2] * F2[1]) * iJ, (F1[2] * F2[0] - F1[0] * F2[2]) * iJ,
                         (F1[0] * F2[1] - F1[1] * F2[0]) * iJ};
        // M = dF^T N and N : dF, summed over rows
        T M[9];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[3 * k + j] = quad_rows_sum(dFr[k] * Nr[j], mirror);
        const T NdF = quad_rows_sum(Nr[0] * dFr[0] + Nr[1] * dFr[1] + Nr[2] * dFr[2], mirror);
        // row r of mu dF + (mu - lam ln J) N dF^T N + lam (N : dF) N
        const T c1 = mu - lam * lnJ, c2 = lam * NdF;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dPr[j] = mu * dFr[j] + c1 * (Nr[0] * M[j] + Nr[1] * M[3 + j] + Nr[2] * M[6 + j]) + c2 * Nr[j];
        ok = J > T(0);
    }
    // row r of -V0 dP B^T
#pragma unroll
    for (int c = 0; c < 3; ++c) H[c] = -V0 * (dPr[0] * b[3 * c] + dPr[1] * b[3 * c + 1] + dPr[2] * b[3 * c + 2]);
    return ok;
}

template <class T, int MODEL, int W>
__global__ __launch_bounds__(1024) void k_lanes(ElemArgs a) {
    extern __shared__ uint4 s_dyn4[];
    if (a.skip && *a.skip) return;   // uniform over the grid
    const uint32_t nt = a.nt;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x, BT = nthr >> 2;
    const uint32_t LB = 4 * BT;   // rows of one component column
    const uint32_t blk = xcd_block(blockIdx.x, a.nblk, a.xcd_run_log2);
    const uint32_t S = a.blk_stride;
    const int32_t *bverts = a.blk_verts + (size_t)blk * S;
    const int32_t *bhpos = a.blk_hpos + (size_t)blk * S;
    const uint16_t *brow = a.blk_row + (size_t)blk * (S + 1);
    const uint32_t t0 = blk * BT;
    if (a.mdone) {   // a batch: skip the block once every mesh it touches has finished (uniform)
        const int32_t m0 = a.tmesh[t0], m1 = a.tmesh[min(t0 + BT, nt) - 1];
        bool all = true;
        for (int32_t m = m0; m <= m1; ++m) all = all && a.mdone[m] != 0;
        if (all) return;
    }
    constexpr bool XB = W == 1;   // rest positions staged, B recomputed (blocks of <= 256 vertices)
    double *s_d = (double *)s_dyn4;
    double *s_u = s_d + 3 * S;
    double *s_x = s_u + 3 * S;
    T *s_h = (T *)(s_x + (XB ? 3 * S : 0));
    // this quad's tet and the lane's row
    const uint32_t tl = tid >> 2, t = t0 + tl;
    const int lane = (int)(tid & 3u), r = lane == 3 ? 2 : lane;
    const bool mirror = lane == 3;
    uint32_t sl[4] = {0, 0, 0, 0}, pw0 = 0, pw1 = 0;
    T b[9], V0 = T(0), mu = (T)a.mu, lam = (T)a.lam;
    if (t < nt) {
        if (W == 1) {
            const uint32_t w = ldc<uint32_t>(a.slot[0], t);
            sl[0] = w & 255u;
            sl[1] = (w >> 8) & 255u;
            sl[2] = (w >> 16) & 255u;
            sl[3] = w >> 24;
        } else {
            const uint32_t w0 = ldc<uint32_t>(a.slot[0], t), w1 = ldc<uint32_t>(a.slot[1], t);
            sl[0] = w0 & 65535u;
            sl[1] = w0 >> 16;
            sl[2] = w1 & 65535u;
            sl[3] = w1 >> 16;
        }
        pw0 = ldc<uint32_t>(a.blk_pos[0], t);
        pw1 = ldc<uint32_t>(a.blk_pos[1], t);
        if (!XB) {
#pragma unroll
            for (int k = 0; k < 9; ++k) b[k] = ldc<T>(a.B[k], t);
            V0 = tet_V0(b);
        }
        if (a.mu_t) {
            mu = ldc<T>(a.mu_t, t);
            lam = ldc<T>(a.lam_t, t);
        }
    }
    for (uint32_t i = tid; i < S; i += nthr) {
        const int32_t gvs = bverts[i];
        if (gvs < 0) continue;
        const uint32_t gv = (uint32_t)gvs;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_d[k * S + i] = ldc<double>(a.d[k], gv);
            s_u[k * S + i] = ldc<double>(a.u[k], gv);
            if (XB) s_x[k * S + i] = ldc<double>(a.X[k], gv);
        }
    }
    __syncthreads();
    if (t < nt) {   // uniform over the quad
        if (XB) rest_B(s_x, S, sl, b, V0);
        // row r of dD and dU from FP64 differences, then row r of G = dD B and dF = dU B
        T dd[3], du[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dd[c] = (T)(s_d[r * S + sl[c + 1]] - s_d[r * S + sl[0]]);
            du[c] = (T)(s_u[r * S + sl[c + 1]] - s_u[r * S + sl[0]]);
        }
        T Gr[3], dFr[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Gr[j] = dd[0] * b[j] + dd[1] * b[3 + j] + dd[2] * b[6 + j];
            dFr[j] = du[0] * b[j] + du[1] * b[3 + j] + du[2] * b[6 + j];
        }
        T H[3];
        kmul_row<T, MODEL>(mu, lam, V0, b, Gr, dFr, r, mirror, H);
        if (!mirror) {
            const uint32_t p[4] = {pw0 & 0xffffu, pw0 >> 16, pw1 & 0xffffu, pw1 >> 16};
            s_h[r * LB + p[1]] = H[0];
            s_h[r * LB + p[2]] = H[1];
            s_h[r * LB + p[3]] = H[2];
            s_h[r * LB + p[0]] = -(H[0] + H[1] + H[2]);
        }
    }
    __syncthreads();
    // each block vertex sums its run of rows (fixed order, FP64): stored if the block owns it,
    // else written to the halo
    for (uint32_t i = tid; i < S; i += nthr) {
        const int32_t gvs = bverts[i];
        if (gvs < 0) continue;
        const uint32_t gv = (uint32_t)gvs;
        const int32_t j0 = brow[i], j1 = brow[i + 1], hp = bhpos[i];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int32_t j = j0; j < j1; ++j) {
            a0 += (double)s_h[j];
            a1 += (double)s_h[LB + j];
            a2 += (double)s_h[2 * LB + j];
        }
        if (hp < 0) {
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
}

template <class T, int MODEL>
void launch_model(int w, const ElemArgs &a, unsigned grid, unsigned threads, size_t shmem, hipStream_t s) {
    if (w == 1) hipLaunchKernelGGL((k_lanes<T, MODEL, 1>), dim3(grid), dim3(threads), shmem, s, a);
    else hipLaunchKernelGGL((k_lanes<T, MODEL, 2>), dim3(grid), dim3(threads), shmem, s, a);
    HIPCHK(hipGetLastError());
}

}  // namespace

size_t lanes_shmem(const ebbx_fem_s *F) {
    const int nx = F->blk_w == 1 ? 1 : 0;
    return (size_t)3 * (2 + nx) * F->blk_maxv * sizeof(double) + (size_t)12 * F->blk_tets * F->esize;
}

void launch_lanes(ebbx_fem_s *F, const ElemArgs &a, hipStream_t s) {
    const unsigned threads = 4u * (unsigned)F->blk_tets, grid = (unsigned)F->nblk;
    const size_t shmem = lanes_shmem(F);
    if (F->prec == EBBX_F32) {
        if (F->model == EBBX_STVK) launch_model<float, EBBX_STVK>(F->blk_w, a, grid, threads, shmem, s);
        else launch_model<float, EBBX_NH>(F->blk_w, a, grid, threads, shmem, s);
    } else {
        if (F->model == EBBX_STVK) launch_model<double, EBBX_STVK>(F->blk_w, a, grid, threads, shmem, s);
        else launch_model<double, EBBX_NH>(F->blk_w, a, grid, threads, shmem, s);
    }
}

}  // namespace ebbx
