// solve.hip -- the implicit-Euler step, its adjoint, and batches of meshes.
//
// The step is the linearised backward-Euler step of the paper's Vega
// workload (Performance Evaluation, Vega: an implicit integrator that builds
// a linear system from the force and stiffness evaluations and solves it with
// a Jacobi-preconditioned conjugate gradient), written as data-parallel
// kernels over the vertex DOFs.
//
// Every solve is segmented by mesh: the DOFs of a domain are split into
// chunks of at most VT vertices that never straddle two meshes, and each
// mesh carries its own CG scalars on the device.  A plain domain is one
// mesh; a batch is the union of many meshes whose solves run side by side in
// the same kernels, each stopping on its own tolerance.  Dot products are
// two-pass reductions: the first pass is fused into the vector kernels
// (per-chunk partial sums, wavefront shuffles then LDS; Runtime
// Implementation, "Reductions"), the second sums a mesh's chunk partials in
// a fixed order, so results are reproducible run to run.  The iterations are
// captured once into HIP graphs and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

#include "fem.h"

namespace ebbx {

// CG state of one mesh, kept on the device.
struct CGState {
    double rz, rr, pq, alpha, beta, bnorm;
    int iters, status, done, converged;
    unsigned long long n_inv;
};

// Solve-wide flags: meshes still iterating; all_done = 1 once none is.  The
// per-mesh finished flags (nm ints) follow the struct in memory.
struct SolveCtl {
    int n_active, all_done;
};

__device__ __forceinline__ int *mesh_done(SolveCtl *c) { return (int *)(c + 1); }

constexpr int VT = 256;   // threads of the vertex kernels = vertices per chunk

// Chunks of the vertex range: chunk c covers vertices [lo[c], hi[c]) of mesh
// mesh[c]; the chunks of mesh m are [cptr[m], cptr[m+1]).
struct Chunks {
    const int32_t *lo, *hi, *mesh, *cptr;
    int xcd;   // 1: chunks dealt to the XCDs in contiguous ranges (one mesh), as its tet blocks are
};

// The chunk of this workgroup.  With one mesh, XCD x takes one contiguous eighth of the
// chunks, the vertices of its eighth of the (Morton-ordered) tet blocks, so that a chunk's
// vectors and its shared vertices' halo entries stay under one L2 from kernel to kernel.
__device__ __forceinline__ int chunk_of(const Chunks &ch) {
    return ch.xcd ? (int)xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
}

// This workgroup's chunk c, its mesh m, its vertices [lo, hi) and its mesh's chunks [c0, c1).
// ONE: a single mesh, launched one workgroup per chunk, whose chunk c holds vertices
// [c VT, min((c + 1) VT, nv)): every field follows from blockIdx without a table read, so the
// first vector loads do not wait behind a chain of dependent table loads.
struct ChunkAt {
    int c, m, c0, c1;
    int64_t lo, hi;
};
template <bool ONE>
__device__ __forceinline__ ChunkAt chunk_at(const Chunks &ch, int64_t nv) {
    if (ONE) {
        const int c = (int)xcd_block(blockIdx.x, gridDim.x);
        const int64_t lo = (int64_t)c * VT;
        return ChunkAt{c, 0, 0, (int)gridDim.x, lo, lo + VT < nv ? lo + VT : nv};
    }
    const int c = chunk_of(ch), m = ch.mesh[c];
    return ChunkAt{c, m, ch.cptr[m], ch.cptr[m + 1], ch.lo[c], ch.hi[c]};
}

static unsigned grid_one(int nch, int cpw) { return (unsigned)((nch + cpw - 1) / cpw); }

static unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + VT - 1) / VT)); }

// Sum of one double over a 256-thread block (fixed order).
__device__ __forceinline__ double block_sum(double x, double *s4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = x;
    __syncthreads();
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// N block sums at once (s: 4 N doubles), each combined exactly as block_sum combines one.
template <int N>
__device__ __forceinline__ void block_sums(double (&x)[N], double *s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] += __shfl_xor(x[i], o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) s[4 * i + (threadIdx.x >> 6)] = x[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (s[4 * i] + s[4 * i + 1]) + (s[4 * i + 2] + s[4 * i + 3]);
}

// Chunk partials, 4 doubles per chunk: [0] p.q, [1] r.r, [2 + parity] r.z of the
// iterations of that parity (the initial residual counts as parity 1).
constexpr int PQ = 0, RR = 1, RZ = 2;

// Each thread's share of a fixed-order sum over chunks [c0, c1): acc[s] += the partials at
// offset o[s] of chunks c0 + t, c0 + t + VT, c0 + t + 2 VT, ... in that order.  The loads of
// PART_BATCH strided chunks are issued before any of them is added, so a workgroup waits for
// one round trip per batch rather than one per chunk; the order of the additions is unchanged.
constexpr int PART_BATCH = 8;
template <int NS>
__device__ __forceinline__ void part_acc(const double *part, int c0, int c1, const int (&o)[NS], double (&acc)[NS]) {
    for (int cb = c0 + (int)threadIdx.x; cb < c1; cb += PART_BATCH * VT) {
        double l[PART_BATCH][NS];
#pragma unroll
        for (int j = 0; j < PART_BATCH; ++j) {
            const int c = cb + j * VT;
#pragma unroll
            for (int s = 0; s < NS; ++s) l[j][s] = c < c1 ? part[4 * c + o[s]] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PART_BATCH; ++j)
            if (cb + j * VT < c1)
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[s] += l[j][s];
    }
}

// Fixed-order sum of the partials at offset o of chunks [c0, c1).
__device__ __forceinline__ double sum_parts(const double *part, int c0, int c1, int o, double *s4) {
    double acc[1] = {0.0};
    part_acc<1>(part, c0, c1, {o}, acc);
    return block_sum(acc[0], s4);
}

// Three fixed-order sums at once (offsets o0, o1, o2), each with exactly the
// operation order of sum_parts, sharing the barriers.
__device__ __forceinline__ void sum_parts3(const double *part, int c0, int c1, int o0, int o1, int o2, double *s12,
                                           double &r0, double &r1, double &r2) {
    double acc[3] = {0.0, 0.0, 0.0};
    part_acc<3>(part, c0, c1, {o0, o1, o2}, acc);
    double a0 = acc[0], a1 = acc[1], a2 = acc[2];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s12[threadIdx.x >> 6] = a0;
        s12[4 + (threadIdx.x >> 6)] = a1;
        s12[8 + (threadIdx.x >> 6)] = a2;
    }
    __syncthreads();
    r0 = (s12[0] + s12[1]) + (s12[2] + s12[3]);
    r1 = (s12[4] + s12[5]) + (s12[6] + s12[7]);
    r2 = (s12[8] + s12[9]) + (s12[10] + s12[11]);
}

// Two fixed-order sums at once (offsets o0, o1), as sum_parts3.
__device__ __forceinline__ void sum_parts2(const double *part, int c0, int c1, int o0, int o1, double *s12, double &r0,
                                           double &r1) {
    double acc[2] = {0.0, 0.0};
    part_acc<2>(part, c0, c1, {o0, o1}, acc);
    double a0 = acc[0], a1 = acc[1];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s12[threadIdx.x >> 6] = a0;
        s12[4 + (threadIdx.x >> 6)] = a1;
    }
    __syncthreads();
    r0 = (s12[0] + s12[1]) + (s12[2] + s12[3]);
    r1 = (s12[4] + s12[5]) + (s12[6] + s12[7]);
}

// One thread of the mesh's block marks mesh m finished.
__device__ __forceinline__ void mark_done(CGState &st, SolveCtl *ctl, int m) {
    st.done = 1;
    mesh_done(ctl)[m] = 1;
    if (atomicSub(&ctl->n_active, 1) == 1) ctl->all_done = 1;
}

// Rebuild the active list (ActList) of a batched solve from the meshes' finished flags, at the
// start of a CG iteration; one workgroup.  Mesh m's tets are [tptr[m], tptr[m+1]), its blocks
// of bt tets those holding them; its first block is left to an earlier unfinished mesh with
// tets in that block, if there is one (small meshes can share a block with several others).
// Scans are in mesh order, so the list is the same on every run.
__global__ __launch_bounds__(VT) void k_active(const SolveCtl *ctl, const int64_t *tptr, const int32_t *tmesh,
                                               int32_t nm, int32_t bt, int32_t *act) {
    __shared__ int32_t s_x[2][VT];
    const int *done = (const int *)(ctl + 1);
    int32_t *hdr = act, *bpfx = act + 4, *bstart = bpfx + (nm + 1);
    int32_t cn = 0, cb = 0;   // carried over the tiles: meshes, blocks
    const int tid = threadIdx.x;
    for (int32_t base = 0; base < nm; base += VT) {
        const int32_t m = base + tid;
        const bool on = m < nm && !done[m];
        int32_t nb = 0, bs = 0;
        if (on) {
            const int64_t t0 = tptr[m], t1 = tptr[m + 1];
            if (t1 > t0) {
                const int64_t b0 = t0 / bt, b1 = (t1 - 1) / bt + 1;
                bool taken = false;
                for (int32_t mm = tmesh[b0 * bt]; mm < m && !taken; ++mm) taken = !done[mm];
                bs = (int32_t)(b0 + (taken ? 1 : 0));
                nb = (int32_t)(b1 - bs);
            }
        }
        // inclusive scans of (on, nb) over the tile (Hillis-Steele in LDS)
        int32_t v0 = on ? 1 : 0, v1 = nb;
        s_x[0][tid] = v0;
        s_x[1][tid] = v1;
        __syncthreads();
        for (int o = 1; o < VT; o <<= 1) {
            const int32_t a0 = tid >= o ? s_x[0][tid - o] : 0, a1 = tid >= o ? s_x[1][tid - o] : 0;
            __syncthreads();
            v0 += a0;
            v1 += a1;
            s_x[0][tid] = v0;
            s_x[1][tid] = v1;
            __syncthreads();
        }
        if (on) {
            const int32_t k = cn + v0 - 1;
            bpfx[k] = cb + v1 - nb;
            bstart[k] = bs;
        }
        cn += s_x[0][VT - 1];
        cb += s_x[1][VT - 1];
        __syncthreads();
    }
    if (tid == 0) {
        bpfx[cn] = cb;
        hdr[0] = cb;
        hdr[1] = 0;
        hdr[2] = cn;
        hdr[3] = 0;
    }
}

struct StepVec {
    double *dn, *vn, *f, *y, *r, *z, *p, *q, *x, *diag;
};

__global__ void k_step_begin(CGState *st, int nm, SolveCtl *ctl, unsigned long long *n_inv) {
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nm; m += gridDim.x * blockDim.x) {
        CGState &s = st[m];
        s.rz = s.rr = s.pq = s.alpha = s.beta = s.bnorm = 0.0;
        s.iters = 0;
        s.status = EBBX_OK;
        s.done = 0;
        s.converged = 0;
        s.n_inv = 0;
        n_inv[m] = 0ull;
        mesh_done(ctl)[m] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->n_active = nm;
        ctl->all_done = nm == 0;
    }
}

// diag = cm M - ck Kdiag (1 on pinned rows); r = Pi b; z = D^-1 r; p = z; x = 0;
// chunk partials (r.z, r.r), where A = cm M - ck K with cm = 1 + dt alpha and
// ck = dt^2 + dt beta (Rayleigh damping D = alpha M - beta K)
// mode 0 (step): b = dt (f + M g - alpha M v_n + (dt + beta) y), with f = f(d_n)
// and y = K(d_n) v_n;
// mode 1 (adjoint solve): b = f, the right-hand side placed in f beforehand.
// f, K v and the stiffness diagonal of vertex v as the fused step preamble left them: a shared
// vertex sums its 9-wide halo entries in unit order, as the halo pass of each map would.
__device__ __forceinline__ void finished_pre(const HaloView &h, const StepVec &w, int64_t nv, int64_t v,
                                             double (&o)[9]) {
    const int32_t r = h.row ? h.row[v] : -1;
    if (r < 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = w.f[k * nv + v];
            o[3 + k] = w.y[k * nv + v];
            o[6 + k] = w.diag[k * nv + v];
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) o[j] = 0.0;
    auto add = [&](int32_t pos) {
        const double *hq = h.halo + 9 * (size_t)pos;
#pragma unroll
        for (int j = 0; j < 9; ++j) o[j] += hq[j];
    };
    if (h.nc > 0) {
        for (int c = 0; c < h.nc; ++c) {
            const int4 q = h.tab[(size_t)r * h.nc + c];
            const int32_t p4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (p4[k] >= 0) add(p4[k]);
        }
    } else {
        for (int32_t j = h.ptr[r]; j < h.ptr[r + 1]; ++j) add(h.pos[j]);
    }
}

// pre (nullable row): the step's f, K v and diagonal come from the fused preamble and its halo
__global__ __launch_bounds__(VT) void k_step_rhs(StepVec w, const double *mass, const uint8_t *pinned, int64_t nv,
                                                 double dt, double gx, double gy, double gz, double alpha, double beta,
                                                 int precond, int mode, Chunks ch, double *part, HaloView pre) {
    const double cm = 1.0 + dt * alpha, ck = dt * dt + dt * beta;
    __shared__ double s4[4];
    const int c = chunk_of(ch);
    const int64_t v = (int64_t)ch.lo[c] + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (v < ch.hi[c]) {
        const double m = mass[v];
        const bool pin = pinned[v] != 0;
        const double g[3] = {gx, gy, gz};
        double fyd[9];
        if (pre.row) finished_pre(pre, w, nv, v, fyd);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            const double fk = pre.row ? fyd[k] : w.f[i], yk = pre.row ? fyd[3 + k] : w.y[i];
            const double b = mode ? w.f[i] : dt * (fk + m * g[k] - alpha * m * w.vn[i] + (dt + beta) * yk);
            const double dg = pin ? 1.0 : (precond ? cm * m - ck * (pre.row ? fyd[6 + k] : w.diag[i]) : 1.0);
            const double r = pin ? 0.0 : b;
            const double z = r / dg;
            w.diag[i] = dg;
            w.r[i] = r;
            w.z[i] = z;
            w.p[i] = z;
            w.x[i] = 0.0;
            rz += r * z;
            rr += r * r;
        }
    }
    rz = block_sum(rz, s4);
    rr = block_sum(rr, s4);
    if (threadIdx.x == 0) {
        part[4 * c + RZ + 1] = rz;
        part[4 * c + RR] = rr;
    }
}

// per mesh: initial r.z and |b|; inverted elements or b = 0 finish the mesh at once
__global__ __launch_bounds__(VT) void k_step_init(CGState *st, const double *part, Chunks ch,
                                                  const unsigned long long *n_inv, SolveCtl *ctl) {
    __shared__ double s4[4];
    const int m = blockIdx.x;
    const double rz = sum_parts(part, ch.cptr[m], ch.cptr[m + 1], RZ + 1, s4);
    const double rr = sum_parts(part, ch.cptr[m], ch.cptr[m + 1], RR, s4);
    if (threadIdx.x == 0) {
        CGState &s = st[m];
        s.rz = rz;
        s.rr = rr;
        s.bnorm = sqrt(rr);
        s.n_inv = n_inv[m];
        if (s.n_inv > 0) {
            s.status = EBBX_E_INVERTED;
            mark_done(s, ctl, m);
        } else if (rr == 0.0) {
            s.converged = 1;
            mark_done(s, ctl, m);
        }
    }
}

// Vertex v's value of an element-map output that may still have its shared
// vertices' sums in the halo (same summation order as the halo pass).
__device__ __forceinline__ void finished(const HaloView &h, const double *y, int64_t nv, int64_t v, double *o) {
    const int32_t r = h.row ? h.row[v] : -1;
    if (r < 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) o[k] = y[k * nv + v];
        return;
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (h.nc > 0) {
        for (int c = 0; c < h.nc; ++c) {
            const int4 q = h.tab[(size_t)r * h.nc + c];
            const int32_t p4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (p4[k] >= 0) {
                    const double *hq = h.halo + 3 * (size_t)p4[k];
                    a0 += hq[0];
                    a1 += hq[1];
                    a2 += hq[2];
                }
        }
    } else {
        for (int32_t j = h.ptr[r]; j < h.ptr[r + 1]; ++j) {
            const double *hq = h.halo + 3 * (size_t)h.pos[j];
            a0 += hq[0];
            a1 += hq[1];
            a2 += hq[2];
        }
    }
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
}

// q = Pi (cm M p - ck y); chunk partial p.q (y finished here if the element map left it in the halo)
template <bool ONE>
__global__ __launch_bounds__(VT) void k_cg_Ap(StepVec w, const double *mass, const uint8_t *pinned, int64_t nv,
                                              double cm, double ck, const CGState *st, Chunks ch, HaloView hv,
                                              double *part) {
    __shared__ double s4[4];
    const ChunkAt a = chunk_at<ONE>(ch, nv);
    const int c = a.c;
    if (st[a.m].done) return;   // uniform over the block
    const int64_t v = a.lo + threadIdx.x;
    double pq = 0.0;
    if (v < a.hi) {
        const double m = mass[v];
        const bool pin = pinned[v] != 0;
        double y[3];
        finished(hv, w.y, nv, v, y);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            const double p = w.p[i];
            const double q = pin ? 0.0 : cm * m * p - ck * y[k];
            w.q[i] = q;
            pq += p * q;
        }
    }
    pq = block_sum(pq, s4);
    if (threadIdx.x == 0) part[4 * c + PQ] = pq;
}

__global__ __launch_bounds__(VT) void k_cg_alpha(CGState *st, const double *part, Chunks ch, SolveCtl *ctl) {
    __shared__ double s4[4];
    const int m = blockIdx.x;
    if (st[m].done) return;
    const double pq = sum_parts(part, ch.cptr[m], ch.cptr[m + 1], PQ, s4);
    if (threadIdx.x == 0) {
        CGState &s = st[m];
        s.pq = pq;
        if (!(pq > 0.0)) {
            s.status = EBBX_E_NOT_SPD;
            mark_done(s, ctl, m);
        } else {
            s.alpha = s.rz / pq;
        }
    }
}

// x += alpha p; r -= alpha q; z = D^-1 r; chunk partials (r.z, r.r)
template <bool ONE>
__global__ __launch_bounds__(VT) void k_cg_update(StepVec w, int64_t nv, const CGState *st, Chunks ch, double *part) {
    __shared__ double s4[4];
    const ChunkAt a = chunk_at<ONE>(ch, nv);
    const int c = a.c;
    const CGState &s = st[a.m];
    if (s.done) return;
    const double alpha = s.alpha;
    const int64_t v = a.lo + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (v < a.hi) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            w.x[i] += alpha * w.p[i];
            const double r = w.r[i] - alpha * w.q[i];
            const double z = r / w.diag[i];
            w.r[i] = r;
            w.z[i] = z;
            rz += r * z;
            rr += r * r;
        }
    }
    rz = block_sum(rz, s4);
    rr = block_sum(rr, s4);
    if (threadIdx.x == 0) {
        part[4 * c + RZ] = rz;
        part[4 * c + RR] = rr;
    }
}

__global__ __launch_bounds__(VT) void k_cg_beta(CGState *st, const double *part, Chunks ch, double tol, int maxit,
                                                SolveCtl *ctl) {
    __shared__ double s4[4];
    const int m = blockIdx.x;
    if (st[m].done) return;
    const double rz = sum_parts(part, ch.cptr[m], ch.cptr[m + 1], RZ, s4);
    const double rr = sum_parts(part, ch.cptr[m], ch.cptr[m + 1], RR, s4);
    if (threadIdx.x == 0) {
        CGState &s = st[m];
        s.iters += 1;
        s.rr = rr;
        if (sqrt(rr) <= tol * s.bnorm || rz == 0.0) {
            s.converged = 1;
            mark_done(s, ctl, m);
        } else {
            s.beta = rz / s.rz;
            s.rz = rz;
            if (s.iters >= maxit) mark_done(s, ctl, m);
        }
    }
}

// p = z + beta p
template <bool ONE>
__global__ __launch_bounds__(VT) void k_cg_p(StepVec w, int64_t nv, const CGState *st, Chunks ch) {
    const ChunkAt a = chunk_at<ONE>(ch, nv);
    const CGState &s = st[a.m];
    if (s.done) return;
    const double beta = s.beta;
    const int64_t v = a.lo + threadIdx.x;
    if (v < a.hi)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            w.p[i] = w.z[i] + beta * w.p[i];
        }
}

// Fused forms for meshes of at most FUSE_CHUNKS chunks: every workgroup of a
// mesh sums the mesh's chunk partials itself (the same fixed order in every
// workgroup, so all of them see the same scalar) instead of a separate
// one-workgroup-per-mesh kernel; the mesh's first chunk records the state.
// r.z ping-pongs between two partial slots by iteration parity, so a
// workgroup can still read the previous iteration's value.
constexpr int FUSE_CHUNKS = 2048;

// alpha = (r.z)_prev / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials (r.z, r.r).
// The vector loads are issued before the partial sums, so they overlap them.
__global__ __launch_bounds__(VT) void k_cg_update_f(StepVec w, int64_t nv, CGState *st, Chunks ch, double *part,
                                                    int par, SolveCtl *ctl) {
    __shared__ double s12[12];
    const ChunkAt a = chunk_at<false>(ch, nv);
    const int c = a.c, m = a.m;
    if (st[m].done) return;   // uniform over the block
    const int64_t v = a.lo + threadIdx.x;
    const bool in = v < a.hi;
    double x[3] = {0, 0, 0}, p[3] = {0, 0, 0}, r[3] = {0, 0, 0}, q[3] = {0, 0, 0}, dg[3] = {1, 1, 1};
    if (in)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            x[k] = w.x[i];
            p[k] = w.p[i];
            r[k] = w.r[i];
            q[k] = w.q[i];
            dg[k] = w.diag[i];
        }
    double pq, rz0;
    sum_parts2(part, a.c0, a.c1, PQ, RZ + (par ^ 1), s12, pq, rz0);
    const bool first = c == a.c0 && threadIdx.x == 0;
    if (!(pq > 0.0)) {   // breakdown: every workgroup of the mesh sees it and leaves x, r alone
        if (first) {
            st[m].pq = pq;
            st[m].status = EBBX_E_NOT_SPD;
            mark_done(st[m], ctl, m);
        }
        return;
    }
    const double alpha = rz0 / pq;
    if (first) {
        st[m].pq = pq;
        st[m].alpha = alpha;
    }
    double rz = 0.0, rr = 0.0;
    if (in) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            w.x[i] = x[k] + alpha * p[k];
            const double rn = r[k] - alpha * q[k];
            const double z = rn / dg[k];
            w.r[i] = rn;
            w.z[i] = z;
            rz += rn * z;
            rr += rn * rn;
        }
    }
    rz = block_sum(rz, s12);
    rr = block_sum(rr, s12);
    if (threadIdx.x == 0) {
        part[4 * c + RZ + par] = rz;
        part[4 * c + RR] = rr;
    }
}

// stopping test; beta = (r.z)_new / (r.z)_prev; p = z + beta p
__global__ __launch_bounds__(VT) void k_cg_p_f(StepVec w, int64_t nv, CGState *st, Chunks ch, const double *part,
                                               int par, double tol, int maxit, SolveCtl *ctl) {
    __shared__ double s12[12];
    const ChunkAt a = chunk_at<false>(ch, nv);
    const int c = a.c, m = a.m;
    if (st[m].done) return;   // uniform; a mesh marked done by its first chunk needs no new p
    const int64_t v = a.lo + threadIdx.x;
    const bool in = v < a.hi;
    double z[3] = {0, 0, 0}, p[3] = {0, 0, 0};
    if (in)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            z[k] = w.z[k * nv + v];
            p[k] = w.p[k * nv + v];
        }
    double rz, rr, rz0;
    sum_parts3(part, a.c0, a.c1, RZ + par, RR, RZ + (par ^ 1), s12, rz, rr, rz0);
    const bool conv = sqrt(rr) <= tol * st[m].bnorm || rz == 0.0;
    const double beta = rz / rz0;
    if (c == a.c0 && threadIdx.x == 0) {
        CGState &s = st[m];
        const int it = s.iters + 1;
        s.iters = it;
        s.rr = rr;
        if (conv) {
            s.converged = 1;
            mark_done(s, ctl, m);
        } else {
            s.beta = beta;
            s.rz = rz;
            if (it >= maxit) mark_done(s, ctl, m);
        }
    }
    if (conv || !in) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) w.p[k * nv + v] = z[k] + beta * p[k];
}

// The fused iteration's vector kernels for one mesh, CPW chunks per workgroup: workgroup g
// (dealt to the XCDs in contiguous ranges) takes chunks [g CPW, (g + 1) CPW), thread t vertex
// g CPW VT + j VT + t of its chunk j.  These kernels move little data each, so much of their
// time is fixed cost (dispatch, the partial sums every workgroup forms), which fewer
// workgroups pay fewer times.  Formulas, chunk partials and sums are those of k_cg_Ap,
// k_cg_update_f and k_cg_p_f, bit for bit.  Measured (64^3 step, 100 iterations): two chunks
// per workgroup help the p kernel (about 0.5 us per iteration) and slow the other two (the
// update with two: +0.6 us, both with two: +3.5 us), whose loads already keep HBM busy.
constexpr int AP_CPW = 1, UP_CPW = 1, P_CPW = 2;

template <int CPW>
__global__ __launch_bounds__(VT) void k_cg_Ap_one(StepVec w, const double *mass, const uint8_t *pinned, int64_t nv,
                                                  int nch, double cm, double ck, const CGState *st, HaloView hv,
                                                  double *part) {
    __shared__ double s[4 * CPW];
    if (st[0].done) return;   // uniform
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int64_t v0 = (int64_t)g * CPW * VT + threadIdx.x;
    double pq[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        pq[j] = 0.0;
        const int64_t v = v0 + j * VT;
        if (v < nv) {
            const double m = mass[v];
            const bool pin = pinned[v] != 0;
            double y[3];
            finished(hv, w.y, nv, v, y);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t i = k * nv + v;
                const double p = w.p[i];
                const double q = pin ? 0.0 : cm * m * p - ck * y[k];
                w.q[i] = q;
                pq[j] += p * q;
            }
        }
    }
    block_sums<CPW>(pq, s);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < CPW; ++j)
            if (g * CPW + j < nch) part[4 * (g * CPW + j) + PQ] = pq[j];
}

template <int CPW>
__global__ __launch_bounds__(VT) void k_cg_update_one(StepVec w, int64_t nv, int nch, CGState *st, double *part,
                                                      int par, SolveCtl *ctl) {
    __shared__ double s[8 * CPW > 12 ? 8 * CPW : 12];
    if (st[0].done) return;   // uniform
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int64_t v0 = (int64_t)g * CPW * VT + threadIdx.x;
    double x[CPW][3], p[CPW][3], r[CPW][3], q[CPW][3], dg[CPW][3];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int64_t v = v0 + j * VT;
        const bool in = v < nv;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            x[j][k] = in ? w.x[i] : 0.0;
            p[j][k] = in ? w.p[i] : 0.0;
            r[j][k] = in ? w.r[i] : 0.0;
            q[j][k] = in ? w.q[i] : 0.0;
            dg[j][k] = in ? w.diag[i] : 1.0;
        }
    }
    double pq, rz0;
    sum_parts2(part, 0, nch, PQ, RZ + (par ^ 1), s, pq, rz0);
    const bool first = g == 0 && threadIdx.x == 0;
    if (!(pq > 0.0)) {   // breakdown: every workgroup sees it and leaves x, r alone
        if (first) {
            st[0].pq = pq;
            st[0].status = EBBX_E_NOT_SPD;
            mark_done(st[0], ctl, 0);
        }
        return;
    }
    const double alpha = rz0 / pq;
    if (first) {
        st[0].pq = pq;
        st[0].alpha = alpha;
    }
    double red[2 * CPW];   // (r.z, r.r) of chunk j at 2 j, 2 j + 1
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        double rz = 0.0, rr = 0.0;
        const int64_t v = v0 + j * VT;
        if (v < nv)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t i = k * nv + v;
                w.x[i] = x[j][k] + alpha * p[j][k];
                const double rn = r[j][k] - alpha * q[j][k];
                const double z = rn / dg[j][k];
                w.r[i] = rn;
                w.z[i] = z;
                rz += rn * z;
                rr += rn * rn;
            }
        red[2 * j] = rz;
        red[2 * j + 1] = rr;
    }
    block_sums<2 * CPW>(red, s);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < CPW; ++j)
            if (g * CPW + j < nch) {
                part[4 * (g * CPW + j) + RZ + par] = red[2 * j];
                part[4 * (g * CPW + j) + RR] = red[2 * j + 1];
            }
}

template <int CPW>
__global__ __launch_bounds__(VT) void k_cg_p_one(StepVec w, int64_t nv, int nch, CGState *st, const double *part,
                                                 int par, double tol, int maxit, SolveCtl *ctl) {
    __shared__ double s12[12];
    if (st[0].done) return;   // uniform
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int64_t v0 = (int64_t)g * CPW * VT + threadIdx.x;
    double z[CPW][3], p[CPW][3];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int64_t v = v0 + j * VT;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            z[j][k] = v < nv ? w.z[k * nv + v] : 0.0;
            p[j][k] = v < nv ? w.p[k * nv + v] : 0.0;
        }
    }
    double rz, rr, rz0;
    sum_parts3(part, 0, nch, RZ + par, RR, RZ + (par ^ 1), s12, rz, rr, rz0);
    const bool conv = sqrt(rr) <= tol * st[0].bnorm || rz == 0.0;
    const double beta = rz / rz0;
    if (g == 0 && threadIdx.x == 0) {
        CGState &s = st[0];
        const int it = s.iters + 1;
        s.iters = it;
        s.rr = rr;
        if (conv) {
            s.converged = 1;
            mark_done(s, ctl, 0);
        } else {
            s.beta = beta;
            s.rz = rz;
            if (it >= maxit) mark_done(s, ctl, 0);
        }
    }
    if (conv) return;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int64_t v = v0 + j * VT;
        if (v < nv)
#pragma unroll
            for (int k = 0; k < 3; ++k) w.p[k * nv + v] = z[j][k] + beta * p[j][k];
    }
}

// One CG iteration after K p for a single mesh of at most SMALL_NV vertices, in one workgroup:
// the passes of k_cg_Ap, k_cg_update_f and k_cg_p_f with workgroup barriers where the large
// solve needs a launch (each dot product is one fixed-order workgroup sum).  The CG scalars live
// in the mesh's state (r.z carried there from one iteration to the next).  A small mesh's
// iteration is launch-bound, so two launches instead of four halve it.
constexpr int SMALL_T = 1024;
constexpr int64_t SMALL_NV = 4096;

__device__ __forceinline__ double block_sum_small(double x, double *s16) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s16[threadIdx.x >> 6] = x;
    __syncthreads();
    // the first four waves combine as block_sum does, so a mesh of at most VT vertices (one
    // chunk, the other waves' sums zero) gets the sums of the multi-workgroup path bit for bit
    const double a = (s16[0] + s16[1]) + (s16[2] + s16[3]);
    double b = 0.0;
#pragma unroll
    for (int g = 1; g < SMALL_T / 256; ++g) b += (s16[4 * g] + s16[4 * g + 1]) + (s16[4 * g + 2] + s16[4 * g + 3]);
    return a + b;
}

__global__ __launch_bounds__(SMALL_T) void k_cg_iter_small(StepVec w, const double *mass, const uint8_t *pinned,
                                                           int64_t nv, double cm, double ck, CGState *st, HaloView hv,
                                                           double tol, int maxit, SolveCtl *ctl) {
    __shared__ double s16[SMALL_T / 64];
    CGState &s = st[0];
    if (s.done) return;   // uniform
    // q = Pi (cm M p - ck K p) and p.q
    double pq = 0.0;
    for (int64_t v = threadIdx.x; v < nv; v += SMALL_T) {
        const double m = mass[v];
        const bool pin = pinned[v] != 0;
        double y[3];
        finished(hv, w.y, nv, v, y);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            const double p = w.p[i];
            const double q = pin ? 0.0 : cm * m * p - ck * y[k];
            w.q[i] = q;
            pq += p * q;
        }
    }
    pq = block_sum_small(pq, s16);
    const double rz0 = s.rz;
    if (!(pq > 0.0)) {   // breakdown: x and r are left alone
        __syncthreads();
        if (threadIdx.x == 0) {
            s.pq = pq;
            s.status = EBBX_E_NOT_SPD;
            mark_done(s, ctl, 0);
        }
        return;
    }
    const double alpha = rz0 / pq;
    // x += alpha p; r -= alpha q; z = D^-1 r (each thread rereads only what it wrote)
    double rz = 0.0, rr = 0.0;
    for (int64_t v = threadIdx.x; v < nv; v += SMALL_T) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            w.x[i] += alpha * w.p[i];
            const double rn = w.r[i] - alpha * w.q[i];
            const double z = rn / w.diag[i];
            w.r[i] = rn;
            w.z[i] = z;
            rz += rn * z;
            rr += rn * rn;
        }
    }
    rz = block_sum_small(rz, s16);
    rr = block_sum_small(rr, s16);
    const bool conv = sqrt(rr) <= tol * s.bnorm || rz == 0.0;
    const double beta = rz / rz0;
    __syncthreads();   // every thread has read the state before thread 0 updates it
    if (threadIdx.x == 0) {
        s.pq = pq;
        s.alpha = alpha;
        const int it = s.iters + 1;
        s.iters = it;
        s.rr = rr;
        if (conv) {
            s.converged = 1;
            mark_done(s, ctl, 0);
        } else {
            s.beta = beta;
            s.rz = rz;
            if (it >= maxit) mark_done(s, ctl, 0);
        }
    }
    if (conv) return;
    for (int64_t v = threadIdx.x; v < nv; v += SMALL_T)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            w.p[i] = w.z[i] + beta * w.p[i];
        }
}

__global__ void k_copy_in(const double *d, const double *v, double *dn, double *vn, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        dn[i] = d[i];
        vn[i] = v[i];
    }
}

__device__ __forceinline__ void write_stats(const CGState &s, double tol, ebbx_step_stats *out) {
    int status = s.status;
    if (status == EBBX_OK && !s.converged && tol > 0.0) status = EBBX_E_NOT_CONVERGED;
    out->iters = s.iters;
    out->status = status;
    out->rel_res = s.bnorm > 0.0 ? sqrt(s.rr) / s.bnorm : 0.0;
    out->n_inverted = (int64_t)s.n_inv;
}

// per chunk: v = v_n + x, d = d_n + dt v unless the mesh's solve broke down;
// the first chunk of each mesh writes its stats record
__global__ __launch_bounds__(VT) void k_step_end(StepVec w, int64_t nv, double dt, double tol, const CGState *st,
                                                 Chunks ch, double *d, double *v, ebbx_step_stats *stats) {
    const int c = chunk_of(ch), m = ch.mesh[c];
    const CGState &s = st[m];
    const int64_t j = (int64_t)ch.lo[c] + threadIdx.x;
    if (s.status == EBBX_OK && j < ch.hi[c])
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + j;
            const double vv = w.vn[i] + w.x[i];
            v[i] = vv;
            d[i] = w.dn[i] + dt * vv;
        }
    if (stats && c == ch.cptr[m] && threadIdx.x == 0) write_stats(s, tol, stats + m);
}

// adjoint: d_n copied in, g^ = gv + dt gx into f (the solve's right-hand side)
__global__ void k_vjp_prep(const double *d, const double *gx, const double *gv, double dt, StepVec w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w.dn[i] = d[i];
        w.f[i] = gv[i] + dt * gx[i];
    }
}

// adjoint: d_bar = gx + dt K w + ck T[v', w];  v_bar = g^ + ck K w - dt alpha M w
// (K w in y, T[v', w] in q, g^ in f, w in x); stats of each mesh's adjoint solve
__global__ __launch_bounds__(VT) void k_vjp_end(StepVec w, const double *gx, const double *mass, double dt, double ck,
                                                double dt_alpha, int64_t nv, const CGState *st, Chunks ch, double tol,
                                                double *d_bar, double *v_bar, ebbx_step_stats *stats) {
    const int c = chunk_of(ch), m = ch.mesh[c];
    const int64_t j = (int64_t)ch.lo[c] + threadIdx.x;
    if (j < ch.hi[c])
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + j;
            const double kw = w.y[i];
            d_bar[i] = gx[i] + dt * kw + ck * w.q[i];
            v_bar[i] = w.f[i] + ck * kw - dt_alpha * mass[j] * w.x[i];
        }
    if (stats && c == ch.cptr[m] && threadIdx.x == 0) write_stats(st[m], tol, stats + m);
}

// ---- batches: validation and per-tet material ----------------------------------------------

// Counts layout violations: mesh ids decreasing along verts or tets, or a tet
// whose corners lie in another mesh.
__global__ void k_batch_check(const int32_t *vmesh, const int32_t *tmesh, const int32_t *keys, int64_t nv,
                              int64_t nt, unsigned long long *bad) {
    const int64_t n = std::max(nv, nt);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long e = 0;
        if (i < nv && i > 0 && vmesh[i] < vmesh[i - 1]) ++e;
        if (i < nt) {
            const int32_t m = tmesh[i];
            if (i > 0 && m < tmesh[i - 1]) ++e;
            for (int c = 0; c < 4; ++c)
                if (vmesh[keys[(int64_t)c * nt + i]] != m) ++e;
        }
        if (e) atomicAdd(bad, e);
    }
}

__global__ void k_expand_material(const int32_t *tmesh, const double *E_m, const double *nu_m, int64_t nt,
                                  double *E_t, double *nu_t, unsigned long long *bad) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = tmesh[t];
        const double E = E_m[m], nu = nu_m[m];
        if (!(E > 0.0) || !(nu > -1.0 && nu < 0.5)) atomicAdd(bad, 1ull);
        E_t[t] = E;
        nu_t[t] = nu;
    }
}

}  // namespace ebbx

using namespace ebbx;

struct ebbx_fem_s::Step {
    DevBuf vec, part, state, ctl, chunks;
    DevBuf act, tptr;   // batches: the active list and the meshes' tet offsets (nm + 1)
    StepVec w{};
    Chunks ch{};
    int nch = 0, nm = 1;
    // graphs: preambles of the step (0) and of the adjoint solve (1), and a chunk of CG iterations
    hipGraphExec_t pre[2] = {nullptr, nullptr}, chunk = nullptr;
    hipGraph_t g_pre[2] = {nullptr, nullptr}, g_chunk = nullptr;
    hipStream_t cap = nullptr;
    int first_iters = 0, chunk_iters = 0;
    bool valid = false;   // graphs match the parameters below
    bool fused = true;    // one-kernel alpha and beta (every mesh has at most FUSE_CHUNKS chunks)
    // parameters baked into the graphs
    double dt = -1, g[3] = {0, 0, 0}, tol = -1, alpha = -1, beta = -1;
    int maxit = -1, precond = -1, strategy = -1, block = -1;
    int *h_done = nullptr;   // pinned host flag for convergence checks
    void drop_graphs() {
        for (int k = 0; k < 2; ++k) {
            if (pre[k]) (void)hipGraphExecDestroy(pre[k]);
            if (g_pre[k]) (void)hipGraphDestroy(g_pre[k]);
            pre[k] = nullptr;
            g_pre[k] = nullptr;
        }
        if (chunk) (void)hipGraphExecDestroy(chunk);
        if (g_chunk) (void)hipGraphDestroy(g_chunk);
        chunk = nullptr;
        g_chunk = nullptr;
        valid = false;
    }
    ~Step() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (h_done) (void)hipHostFree(h_done);
    }
};

ebbx_fem_s::ebbx_fem_s() = default;
ebbx_fem_s::~ebbx_fem_s() = default;

namespace ebbx {
void step_drop_graphs(ebbx_fem_s *F) {
    if (F->step) F->step->drop_graphs();
}
}  // namespace ebbx

namespace {

void capture_begin(hipStream_t cap) { HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)); }

hipGraphExec_t capture_end(hipStream_t cap, hipGraph_t *g) {
    HIPCHK(hipStreamEndCapture(cap, g));
    hipGraphExec_t ex = nullptr;
    HIPCHK(hipGraphInstantiate(&ex, *g, nullptr, nullptr, 0));
    return ex;
}

// The buffers one solve runs on: the CG vectors, the chunk table of the mesh
// segmentation, the chunk partials and the per-mesh state.
struct SolveBufs {
    StepVec w;
    Chunks ch;
    CGState *st;
    SolveCtl *ctl;
    double *part;
    int nch, nm;
    bool fused;
    int32_t *act;           // batches: the active list (NULL: every kernel covers every mesh)
    const int64_t *tptr;    // batches: the meshes' tet offsets
};

// Whether the step preamble of `mode` runs the fused element pass (the step, with the Jacobi
// preconditioner, under the block strategy).
bool pre_fused(const ebbx_fem_s *F, const ebbx_step_params &p, int mode) {
    return mode == 0 && p.precond == EBBX_PRECOND_JACOBI && elem_pre_ok(F);
}

// The preamble of `mode` (0: step, 1: adjoint solve) onto stream cs: state reset, (step)
// forces and K v, the Jacobi diagonal, the right-hand side and the initial residual.
void launch_preamble(ebbx_fem_s *F, const ebbx_step_params &p, int mode, const SolveBufs &b, hipStream_t cs) {
    const int64_t nv = F->nv;
    unsigned long long *n_inv = F->status.as<unsigned long long>();
    hipLaunchKernelGGL(k_step_begin, dim3((b.nm + VT - 1) / VT), dim3(VT), 0, cs, b.st, b.nm, b.ctl, n_inv);
    // the block strategy evaluates the step's force, K v and diagonal in one fused pass whose
    // shared vertices k_step_rhs finishes; other strategies run the three maps
    const bool fused = pre_fused(F, p, mode);
    HaloView pre{};
    if (fused) {
        elem_launch_pre(F, b.w.dn, b.w.vn, b.w.f, b.w.y, b.w.diag, cs);
        pre = elem_pre_halo(F);
    } else {
        if (mode == 0) {
            elem_launch(F, OP_FORCE, b.w.dn, nullptr, b.w.f, 0, cs);
            elem_launch(F, OP_KMUL, b.w.dn, b.w.vn, b.w.y, 0, cs);
        }
        if (p.precond == EBBX_PRECOND_JACOBI) elem_launch(F, OP_DIAG, b.w.dn, nullptr, b.w.diag, 0, cs);
    }
    hipLaunchKernelGGL(k_step_rhs, dim3(b.nch), dim3(VT), 0, cs, b.w, F->mass.as<double>(), F->pinned.as<uint8_t>(),
                       nv, p.dt, p.g[0], p.g[1], p.g[2], p.alpha, p.beta, p.precond, mode, b.ch, b.part, pre);
    hipLaunchKernelGGL(k_step_init, dim3(b.nm), dim3(VT), 0, cs, b.st, (const double *)b.part, b.ch,
                       (const unsigned long long *)n_inv, b.ctl);
    HIPCHK(hipGetLastError());
}

// `count` CG iterations (at most maxit) onto stream cs, starting at an even iteration (the
// fused kernels pick r.z slots by iteration parity).  Every kernel is predicated on its
// mesh's done flag, the element map on the solve-wide all_done flag.
void launch_iterations(ebbx_fem_s *F, const ebbx_step_params &p, const SolveBufs &b, int count, hipStream_t cs) {
    const int64_t nv = F->nv;
    // K p: a block-strategy element map leaves its shared vertices in the halo and
    // k_cg_Ap finishes them as it reads y (one launch and one y round trip fewer)
    const HaloView hv = elem_halo_view(F);
    const double cm = 1.0 + p.dt * p.alpha, ck = p.dt * p.dt + p.dt * p.beta;
    CGState *st = b.st;
    SolveCtl *ctl = b.ctl;
    double *part = b.part;
    // a batch in the block strategy evaluates K p over a list of the blocks of its unfinished
    // meshes, rebuilt at the start of every iteration, so finished meshes cost no workgroups
    const bool list = b.act && elem_list_ok(F, OP_KMUL);
    const int32_t *act = list ? b.act : nullptr;
    if (b.nm == 1 && b.fused && nv <= SMALL_NV) {
        // a small mesh: K p, then one single-workgroup kernel for the rest of the iteration
        for (int it = 0; it < count && it < p.maxit; ++it) {
            elem_launch(F, OP_KMUL, b.w.dn, b.w.p, b.w.y, 0, cs, &ctl->all_done, nullptr, nullptr, hv.row == nullptr);
            hipLaunchKernelGGL(k_cg_iter_small, dim3(1), dim3(SMALL_T), 0, cs, b.w, F->mass.as<double>(),
                               F->pinned.as<uint8_t>(), nv, cm, ck, st, hv, p.tol, p.maxit, ctl);
        }
        HIPCHK(hipGetLastError());
        return;
    }
    // one mesh: the vector kernels take their chunk from blockIdx alone
    const bool one = b.nm == 1;
    for (int it = 0; it < count && it < p.maxit; ++it) {
        if (list) {
            hipLaunchKernelGGL(k_active, dim3(1), dim3(VT), 0, cs, (const SolveCtl *)ctl, b.tptr, F->tmesh,
                               (int32_t)b.nm, (int32_t)F->blk_tets, b.act);
        }
        elem_launch(F, OP_KMUL, b.w.dn, b.w.p, b.w.y, 0, cs, &ctl->all_done, nullptr,
                    b.nm > 1 ? (const int *)(ctl + 1) : nullptr, hv.row == nullptr, nullptr, act);
        if (one && b.fused) {
            // one mesh: the fused iteration's vector kernels with several chunks per workgroup
            const int par = it & 1;
            hipLaunchKernelGGL(k_cg_Ap_one<AP_CPW>, dim3(grid_one(b.nch, AP_CPW)), dim3(VT), 0, cs, b.w,
                               F->mass.as<double>(), F->pinned.as<uint8_t>(), nv, b.nch, cm, ck, (const CGState *)st,
                               hv, part);
            hipLaunchKernelGGL(k_cg_update_one<UP_CPW>, dim3(grid_one(b.nch, UP_CPW)), dim3(VT), 0, cs, b.w, nv,
                               b.nch, st, part, par, ctl);
            hipLaunchKernelGGL(k_cg_p_one<P_CPW>, dim3(grid_one(b.nch, P_CPW)), dim3(VT), 0, cs, b.w, nv, b.nch, st,
                               (const double *)part, par, p.tol, p.maxit, ctl);
            continue;
        }
        hipLaunchKernelGGL(one ? k_cg_Ap<true> : k_cg_Ap<false>, dim3(b.nch), dim3(VT), 0, cs, b.w,
                           F->mass.as<double>(), F->pinned.as<uint8_t>(), nv, cm, ck, (const CGState *)st, b.ch, hv,
                           part);
        if (b.fused) {
            const int par = it & 1;
            hipLaunchKernelGGL(k_cg_update_f, dim3(b.nch), dim3(VT), 0, cs, b.w, nv, st, b.ch, part, par,
                               ctl);
            hipLaunchKernelGGL(k_cg_p_f, dim3(b.nch), dim3(VT), 0, cs, b.w, nv, st, b.ch,
                               (const double *)part, par, p.tol, p.maxit, ctl);
        } else {
            hipLaunchKernelGGL(k_cg_alpha, dim3(b.nm), dim3(VT), 0, cs, st, (const double *)part, b.ch, ctl);
            hipLaunchKernelGGL(one ? k_cg_update<true> : k_cg_update<false>, dim3(b.nch), dim3(VT), 0, cs, b.w, nv,
                               (const CGState *)st, b.ch, part);
            hipLaunchKernelGGL(k_cg_beta, dim3(b.nm), dim3(VT), 0, cs, st, (const double *)part, b.ch, p.tol, p.maxit,
                               ctl);
            hipLaunchKernelGGL(one ? k_cg_p<true> : k_cg_p<false>, dim3(b.nch), dim3(VT), 0, cs, b.w, nv,
                               (const CGState *)st, b.ch);
        }
    }
    HIPCHK(hipGetLastError());
}

SolveBufs step_bufs(ebbx_fem_s *F) {
    auto &S = *F->step;
    return SolveBufs{S.w, S.ch, S.state.as<CGState>(), S.ctl.as<SolveCtl>(), S.part.as<double>(), S.nch, S.nm,
                     S.fused, S.nm > 1 ? S.act.as<int32_t>() : nullptr,
                     S.nm > 1 ? S.tptr.as<int64_t>() : nullptr};
}

// Capture the preamble of `mode` (0: step, 1: adjoint solve) and, if the
// parameters changed, the CG chunk shared by both.
void build_graphs(ebbx_fem_s *F, const ebbx_step_params &p, int mode) {
    auto &S = *F->step;
    const bool same = S.dt == p.dt && !std::memcmp(S.g, p.g, sizeof S.g) && S.tol == p.tol && S.maxit == p.maxit &&
                      S.alpha == p.alpha && S.beta == p.beta &&
                      S.precond == p.precond && S.strategy == F->strategy && S.block == F->block && S.valid;
    if (!same) S.drop_graphs();
    if (S.pre[mode]) return;
    const SolveBufs b = step_bufs(F);
    hipStream_t cs = S.cap;
    if (pre_fused(F, p, mode)) elem_pre_prepare(F, cs);   // its halo, allocated outside the capture
    capture_begin(cs);
    CaptureGuard guard(cs);
    launch_preamble(F, p, mode, b, cs);
    // chunks of CG iterations.  A fixed-count solve (tol = 0) runs chunks of up to 128
    // without host checks.  With a tolerance the first chunk has 32 iterations and later
    // ones 16 (8 for a batch, whose idle iterations still dispatch every block and chunk of
    // every mesh), each launched only after the host has read that some mesh is still
    // iterating: iterations past convergence cost a launch each, so the chunks stay short.
    S.first_iters = std::max(1, std::min(p.maxit, p.tol > 0.0 ? 32 : 128));
    S.chunk_iters = std::max(1, std::min(p.maxit, p.tol > 0.0 ? (b.nm > 1 ? 8 : 16) : 128));
    // the fused kernels pick r.z slots by iteration parity: later chunks must start at even iterations
    if (p.maxit > S.first_iters && ((S.first_iters | S.chunk_iters) & 1))
        fail(EBBX_E_STATE, "CG chunk sizes must be even");
    // the preamble graph also holds the first chunk, so a solve that converges
    // within it is one graph launch
    launch_iterations(F, p, b, S.first_iters, cs);
    guard.disarm();
    S.pre[mode] = capture_end(cs, &S.g_pre[mode]);
    if (!S.chunk && p.maxit > S.first_iters) {
        capture_begin(cs);
        CaptureGuard chunk_guard(cs);
        launch_iterations(F, p, b, S.chunk_iters, cs);
        chunk_guard.disarm();
        S.chunk = capture_end(cs, &S.g_chunk);
    }
    S.valid = true;
    S.dt = p.dt;
    std::memcpy(S.g, p.g, sizeof S.g);
    S.tol = p.tol;
    S.alpha = p.alpha;
    S.beta = p.beta;
    S.maxit = p.maxit;
    S.precond = p.precond;
    S.strategy = F->strategy;
    S.block = F->block;
}

void check_step_params(const ebbx_step_params *params) {
    if (!params) fail(EBBX_E_ARG, "params is NULL");
    const ebbx_step_params &p = *params;
    if (!(p.dt > 0.0)) fail(EBBX_E_ARG, "dt must be > 0");
    if (p.maxit < 0) fail(EBBX_E_ARG, "maxit must be >= 0");
    if (!(p.tol >= 0.0)) fail(EBBX_E_ARG, "tol must be >= 0");
    if (!(p.alpha >= 0.0) || !(p.beta >= 0.0) || !std::isfinite(p.alpha) || !std::isfinite(p.beta))
        fail(EBBX_E_ARG, "damping coefficients alpha and beta must be finite and >= 0");
    if (p.precond != EBBX_PRECOND_NONE && p.precond != EBBX_PRECOND_JACOBI) fail(EBBX_E_ARG, "bad precond");
}

// Solver buffers and the chunk tables of the mesh segmentation (once per domain).
void ensure_step(ebbx_fem_s *F, hipStream_t s) {
    if (F->step) return;
    const int64_t nv = F->nv, nm = F->nm;
    auto S = std::make_unique<ebbx_fem_s::Step>();
    const int64_t n3 = 3 * std::max<int64_t>(nv, 1);
    S->vec.reset((size_t)n3 * 10 * sizeof(double), s);
    double *b = S->vec.as<double>();
    S->w = StepVec{b, b + n3, b + 2 * n3, b + 3 * n3, b + 4 * n3, b + 5 * n3, b + 6 * n3, b + 7 * n3, b + 8 * n3,
                   b + 9 * n3};
    // chunks: every mesh gets at least one (possibly empty) so that it reports stats
    std::vector<int32_t> lo, hi, mesh, cptr(1, 0);
    for (int64_t m = 0; m < nm; ++m) {
        const int64_t a = F->mesh_vptr[m], e = F->mesh_vptr[m + 1];
        int64_t v = a;
        do {
            const int64_t w = std::min<int64_t>(v + VT, e);
            lo.push_back((int32_t)v);
            hi.push_back((int32_t)w);
            mesh.push_back((int32_t)m);
            v = w;
        } while (v < e);
        cptr.push_back((int32_t)lo.size());
    }
    const int64_t nch = (int64_t)lo.size();
    if (nch >= (int64_t(1) << 31)) fail(EBBX_E_ARG, "too many vertex chunks");
    S->nch = (int)nch;
    S->nm = (int)nm;
    S->chunks.reset((size_t)(3 * nch + nm + 1) * sizeof(int32_t), s);
    int32_t *cp = S->chunks.as<int32_t>();
    HIPCHK(hipMemcpyAsync(cp, lo.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cp + nch, hi.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cp + 2 * nch, mesh.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(cp + 3 * nch, cptr.data(), (nm + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    S->ch = Chunks{cp, cp + nch, cp + 2 * nch, cp + 3 * nch, nm == 1 ? 1 : 0};
    S->part.reset((size_t)nch * 4 * sizeof(double), s);
    int32_t most = 0;
    for (int64_t m = 0; m < nm; ++m) most = std::max(most, cptr[(size_t)m + 1] - cptr[(size_t)m]);
    S->fused = most <= FUSE_CHUNKS;
    if (nm > 1) {
        if ((int64_t)F->mesh_tptr.size() != nm + 1) fail(EBBX_E_STATE, "batch without per-mesh tet offsets");
        S->act.reset(act_list_ints(nm) * sizeof(int32_t), s);
        S->tptr.reset((size_t)(nm + 1) * sizeof(int64_t), s);
        HIPCHK(hipMemcpyAsync(S->tptr.get(), F->mesh_tptr.data(), (nm + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    S->state.reset((size_t)std::max<int64_t>(nm, 1) * sizeof(CGState), s);
    S->ctl.reset(sizeof(SolveCtl) + (size_t)std::max<int64_t>(nm, 1) * sizeof(int), s);
    HIPCHK(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void **)&S->h_done, sizeof(int), hipHostMallocDefault));
    HIPCHK(hipStreamSynchronize(s));
    F->step = std::move(S);
}

// Launch the preamble of `mode` and the CG chunks on s.
void run_solve(ebbx_fem_s *F, const ebbx_step_params &p, int mode, hipStream_t s) {
    build_graphs(F, p, mode);
    auto &S = *F->step;
    // preamble + first chunk, then further chunks until maxit
    HIPCHK(hipGraphLaunch(S.pre[mode], s));
    SolveCtl *ctl = S.ctl.as<SolveCtl>();
    for (int done = S.first_iters; done < p.maxit; done += S.chunk_iters) {
        // with a tolerance, stop launching once every mesh has finished
        if (p.tol > 0.0) {
            HIPCHK(hipMemcpyAsync(S.h_done, &ctl->all_done, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (*S.h_done) break;
        }
        HIPCHK(hipGraphLaunch(S.chunk, s));
    }
}

// One implicit step of every mesh of F; stats: one record per mesh (nullable).
void implicit_step(ebbx_fem_s *F, double *d, double *v, const ebbx_step_params *params, ebbx_step_stats *stats,
                   hipStream_t s) {
    check_step_params(params);
    const ebbx_step_params &p = *params;
    const int64_t nv = F->nv;
    if (nv > 0 && (!d || !v)) fail(EBBX_E_ARG, "d or v is NULL");
    if (nv > 0 && overlap(d, v, (size_t)(3 * nv) * sizeof(double))) fail(EBBX_E_PHASE, "d aliases v");
    ensure_step(F, s);
    auto &S = *F->step;
    if (nv > 0) {
        hipLaunchKernelGGL(k_copy_in, dim3(grid_for(3 * nv)), dim3(VT), 0, s, (const double *)d, (const double *)v,
                           S.w.dn, S.w.vn, 3 * nv);
        HIPCHK(hipGetLastError());
    }
    run_solve(F, p, 0, s);
    hipLaunchKernelGGL(k_step_end, dim3(S.nch), dim3(VT), 0, s, S.w, nv, p.dt, p.tol,
                       (const CGState *)S.state.as<CGState>(), S.ch, d, v, stats);
    HIPCHK(hipGetLastError());
}

}  // namespace

extern "C" ebbx_status ebbx_implicit_step(ebbx_fem fem, double *d, double *v, const ebbx_step_params *params,
                                          ebbx_step_stats *stats_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (F->nm != 1) fail(EBBX_E_STATE, "this domain is a batch of %lld meshes: use ebbx_batch_implicit_step",
                         (long long)F->nm);
    implicit_step(F, d, v, params, stats_dev, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_implicit_step_vjp(ebbx_fem fem, const double *d_n, const double *v_np1,
                                              const ebbx_step_params *params, const double *gx, const double *gv,
                                              double *d_bar, double *v_bar, double *E_bar,
                                              ebbx_step_stats *stats_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (F->nm != 1) fail(EBBX_E_STATE, "the adjoint step takes a single-mesh domain");
    check_step_params(params);
    const ebbx_step_params &p = *params;
    const int64_t nv = F->nv;
    if (nv > 0 && (!d_n || !v_np1 || !gx || !gv || !d_bar || !v_bar)) fail(EBBX_E_ARG, "a vector argument is NULL");
    const size_t bytes = (size_t)(3 * nv) * sizeof(double);
    if (nv > 0) {
        const void *ins[4] = {d_n, v_np1, gx, gv};
        for (const void *o : {(const void *)d_bar, (const void *)v_bar})
            for (const void *i : ins)
                if (overlap(o, i, bytes)) fail(EBBX_E_PHASE, "an output of the adjoint aliases an input");
        if (overlap(d_bar, v_bar, bytes)) fail(EBBX_E_PHASE, "d_bar aliases v_bar");
    }
    hipStream_t s = (hipStream_t)stream;
    ensure_step(F, s);
    auto &S = *F->step;
    if (nv > 0) {
        hipLaunchKernelGGL(k_vjp_prep, dim3(grid_for(3 * nv)), dim3(VT), 0, s, d_n, gx, gv, p.dt, S.w, 3 * nv);
        HIPCHK(hipGetLastError());
    }
    // A w = Pi (gv + dt gx), with A = (1 + dt alpha) M - (dt^2 + dt beta) K(d_n); w ends in x
    run_solve(F, p, 1, s);
    elem_launch(F, OP_KMUL, S.w.dn, S.w.x, S.w.y, 0, s);
    elem_launch(F, OP_TMUL, S.w.dn, v_np1, S.w.q, 0, s, nullptr, S.w.x);
    const double ck = p.dt * p.dt + p.dt * p.beta;
    hipLaunchKernelGGL(k_vjp_end, dim3(S.nch), dim3(VT), 0, s, S.w, gx, F->mass.as<double>(), p.dt, ck,
                       p.dt * p.alpha, nv, (const CGState *)S.state.as<CGState>(), S.ch, p.tol, d_bar, v_bar,
                       stats_dev);
    HIPCHK(hipGetLastError());
    if (E_bar) elem_egrad(F, S.w.dn, v_np1, S.w.x, p.dt, ck, E_bar, s);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_stats_fetch(const ebbx_step_stats *stats_dev, ebbx_step_stats *host, ebbx_stream stream) {
    EBBX_API_BEGIN
    if (!stats_dev || !host) fail(EBBX_E_ARG, "stats pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(host, stats_dev, sizeof(ebbx_step_stats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    EBBX_API_END
}

// ---- batches ------------------------------------------------------------------------------

struct ebbx_batch_s {
    std::unique_ptr<ebbx_fem_s> fem;   // the union domain
    ebbx_relation_s *meshes = nullptr;
    DevBuf E_t, nu_t;                  // per-tet material expanded from the meshes' fields
    ~ebbx_batch_s() {
        if (fem) fem_unregister(fem.get());
    }
};

namespace {
std::mutex g_batch_mu;
std::set<ebbx_batch_s *> g_batches;

ebbx_batch_s *check_batch(ebbx_batch b) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (!b || !g_batches.count(b)) fail(EBBX_E_ARG, "invalid batch handle");
    return b;
}

}  // namespace

namespace ebbx {
const char *batch_relation_user(const ebbx_relation_s *r) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (const ebbx_batch_s *B : g_batches)
        if (B->meshes == r) return "a batch (its meshes relation)";
    return nullptr;
}
}  // namespace ebbx

namespace {

KeyField &mesh_key(ebbx_relation_s *r, const char *name, ebbx_relation_s *meshes) {
    if (!name) fail(EBBX_E_ARG, "a mesh key-field name is NULL");
    KeyField &k = get_key(r, name);
    if (k.target != meshes) fail(EBBX_E_ARG, "key-field '%s' does not target '%s'", name, meshes->name.c_str());
    if (k.arity != 1) fail(EBBX_E_SHAPE, "key-field '%s' must have arity 1", name);
    return k;
}
}  // namespace

extern "C" {

ebbx_status ebbx_batch_create(ebbx_relation meshes, ebbx_relation tets, ebbx_relation verts,
                              const ebbx_batch_fields *fields, const ebbx_fem_params *params, ebbx_batch *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = nullptr;
    if (!fields || !params) fail(EBBX_E_ARG, "fields or params is NULL");
    if (params->E_field) fail(EBBX_E_ARG, "a batch takes its material from the meshes relation (E_field must be NULL)");
    auto *mr = check_rel(meshes);
    auto *tr = check_rel(tets);
    auto *vr = check_rel(verts);
    const int64_t nm = mr->size;
    if (nm < 1) fail(EBBX_E_ARG, "a batch needs at least one mesh");
    if (!fields->E || !fields->nu) fail(EBBX_E_ARG, "the meshes' E and nu field names are required");
    const double *E_m = (const double *)get_field(mr, fields->E, EBBX_F64, 1).ptr;
    const double *nu_m = (const double *)get_field(mr, fields->nu, EBBX_F64, 1).ptr;
    KeyField &tk = mesh_key(tr, fields->tet_mesh, mr);
    KeyField &vk = mesh_key(vr, fields->vert_mesh, mr);
    hipStream_t s = nullptr;
    auto B = std::make_unique<ebbx_batch_s>();
    B->meshes = mr;
    // the union domain, first with a placeholder uniform material
    ebbx_fem_params up = *params;
    up.E = 1.0;
    up.nu = 0.25;
    B->fem = fem_build(tr, fields->tet_verts, vr, fields->pos, fields->pinned, up, nullptr);
    ebbx_fem_s *F = B->fem.get();
    const int64_t nt = F->nt, nv = F->nv;
    // layout: verts and tets sorted by mesh, every tet inside its mesh
    DevBuf bad(2 * sizeof(unsigned long long), s);
    HIPCHK(hipMemsetAsync(bad.get(), 0, 2 * sizeof(unsigned long long), s));
    if (std::max(nt, nv) > 0) {
        hipLaunchKernelGGL(k_batch_check, dim3(grid_for(std::max(nt, nv))), dim3(VT), 0, s, vk.ptr, tk.ptr, F->keys, nv,
                           nt, bad.as<unsigned long long>());
        HIPCHK(hipGetLastError());
    }
    // per-tet material from the meshes' E and nu
    B->E_t.reset((size_t)std::max<int64_t>(nt, 1) * sizeof(double), s);
    B->nu_t.reset((size_t)std::max<int64_t>(nt, 1) * sizeof(double), s);
    if (nt > 0) {
        hipLaunchKernelGGL(k_expand_material, dim3(grid_for(nt)), dim3(VT), 0, s, tk.ptr, E_m, nu_m, nt,
                           B->E_t.as<double>(), B->nu_t.as<double>(), bad.as<unsigned long long>() + 1);
        HIPCHK(hipGetLastError());
    }
    unsigned long long hbad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hbad, bad.get(), sizeof hbad, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad[0]) fail(EBBX_E_LAYOUT, "batch layout: verts and tets must be sorted by mesh and every tet must lie in its "
                      "mesh (%llu violations)", hbad[0]);
    if (hbad[1]) fail(EBBX_E_ARG, "a mesh has E <= 0 or nu outside (-1, 0.5)");
    elem_set_material(F, B->E_t.as<double>(), B->nu_t.as<double>(), 0.0, 0.0, s);
    // vertex ranges of the meshes: the grouping of verts by mesh (sorted, so contiguous)
    auto grp = build_group(vr, fields->vert_mesh, s);
    F->mesh_vptr.assign((size_t)nm + 1, 0);
    HIPCHK(hipMemcpyAsync(F->mesh_vptr.data(), grp->row_ptr.get(), (nm + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                          s));
    // tet ranges of the meshes (the tets are sorted by mesh, checked above)
    auto tgrp = build_group(tr, fields->tet_mesh, s);
    F->mesh_tptr.assign((size_t)nm + 1, 0);
    HIPCHK(hipMemcpyAsync(F->mesh_tptr.data(), tgrp->row_ptr.get(), (nm + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                          s));
    F->nm = nm;
    F->tmesh = tk.ptr;
    F->status.reset((size_t)std::max<int64_t>(nm, 4) * sizeof(unsigned long long), s);
    HIPCHK(hipMemsetAsync(F->status.get(), 0, (size_t)std::max<int64_t>(nm, 4) * sizeof(unsigned long long), s));
    F->batch_owned = true;
    HIPCHK(hipStreamSynchronize(s));
    fem_register(F);
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        g_batches.insert(B.get());
    }
    *out = B.release();
    EBBX_API_END
}

ebbx_status ebbx_batch_destroy(ebbx_batch batch) {
    EBBX_API_BEGIN
    auto *B = check_batch(batch);
    HIPCHK(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        g_batches.erase(B);
    }
    delete B;
    EBBX_API_END
}

ebbx_status ebbx_batch_fem(ebbx_batch batch, ebbx_fem *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = check_batch(batch)->fem.get();
    EBBX_API_END
}

ebbx_status ebbx_batch_implicit_step(ebbx_batch batch, double *d, double *v, const ebbx_step_params *params,
                                     ebbx_step_stats *per_mesh_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *B = check_batch(batch);
    implicit_step(B->fem.get(), d, v, params, per_mesh_dev, (hipStream_t)stream);
    EBBX_API_END
}

}  // extern "C"
