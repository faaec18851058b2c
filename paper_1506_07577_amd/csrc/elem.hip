// elem.hip -- the element-parallel map over the tets relation.
//
// One thread per tet (the paper's GPU specialisation maps one relation row to
// one thread; Runtime Implementation, "CPU/GPU Specialization").  Each thread
// gathers the vertex fields of its four corners through the tets.v key-field,
// evaluates the hyperelastic element quantity and reduces (+=) twelve results
// into a vertex field (Runtime Implementation, "Reductions").  The per-tet
// quantities are those of the paper's Vega (StVK) and FreeFem++ (neo-Hookean)
// workloads (Performance Evaluation); the textbook formulas are written in the
// displacement-gradient form G = dD B, F = I + G, so that single precision
// keeps its accuracy near the rest shape (no F - I or F - F^-T cancellation).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "fem.h"

namespace ebbx {

enum Scatter { SC_ATOMIC = 0, SC_PART = 1, SC_BLOCK = 2 };

template <class T> __device__ __forceinline__ T t_log1p(T x);
template <> __device__ __forceinline__ float t_log1p<float>(float x) { return log1pf(x); }
template <> __device__ __forceinline__ double t_log1p<double>(double x) { return log1p(x); }

// ---- 3x3 algebra on registers (row-major, M[3*i + j]) ---------------------------

template <class T> __device__ __forceinline__ T det3(const T *A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// C = A B
template <class T> __device__ __forceinline__ void mul3(const T *A, const T *B, T *C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// C = A^T B
template <class T> __device__ __forceinline__ void mulTN3(const T *A, const T *B, T *C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}

// C = A B^T
template <class T> __device__ __forceinline__ void mulNT3(const T *A, const T *B, T *C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}

// cofactor matrix of F = I + G: F^-T = cof(F) / det(F)
template <class T> __device__ __forceinline__ void cof_IpG(const T *G, T *C) {
    const T f0 = T(1) + G[0], f1 = G[1], f2 = G[2], f3 = G[3], f4 = T(1) + G[4], f5 = G[5], f6 = G[6],
            f7 = G[7], f8 = T(1) + G[8];
    C[0] = f4 * f8 - f5 * f7;
    C[1] = f5 * f6 - f3 * f8;
    C[2] = f3 * f7 - f4 * f6;
    C[3] = f2 * f7 - f1 * f8;
    C[4] = f0 * f8 - f2 * f6;
    C[5] = f1 * f6 - f0 * f7;
    C[6] = f1 * f5 - f2 * f4;
    C[7] = f2 * f3 - f0 * f5;
    C[8] = f0 * f4 - f1 * f3;
}

// J - 1 = det(I + G) - 1 = tr G + ((tr G)^2 - tr(G G))/2 + det G, free of cancellation
template <class T> __device__ __forceinline__ T jm1_of(const T *G) {
    const T tr = G[0] + G[4] + G[8];
    const T trGG = G[0] * G[0] + G[4] * G[4] + G[8] * G[8] + T(2) * (G[1] * G[3] + G[2] * G[6] + G[5] * G[7]);
    return tr + T(0.5) * (tr * tr - trGG) + det3(G);
}

// ---- constitutive models -----------------------------------------------------------

// StVK: S = 2 mu E + lam tr(E) I with E = (G + G^T + G^T G)/2 (symmetric, full 3x3)
template <class T> __device__ __forceinline__ void stvk_S(T mu, T lam, const T *G, T *S) {
    T GtG[9];
    mulTN3(G, G, GtG);
    T E[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) E[3 * i + j] = T(0.5) * (G[3 * i + j] + G[3 * j + i] + GtG[3 * i + j]);
    const T le = lam * (E[0] + E[4] + E[8]);
#pragma unroll
    for (int k = 0; k < 9; ++k) S[k] = T(2) * mu * E[k];
    S[0] += le;
    S[4] += le;
    S[8] += le;
}

// P(F) in G-form.  Returns false for an inverted neo-Hookean element.
template <class T, int MODEL> __device__ __forceinline__ bool stress(T mu, T lam, const T *G, T *P) {
    if (MODEL == EBBX_STVK) {
        T S[9], GS[9];
        stvk_S(mu, lam, G, S);
        mul3(G, S, GS);
#pragma unroll
        for (int k = 0; k < 9; ++k) P[k] = S[k] + GS[k];   // P = (I + G) S
        return true;
    } else {
        // P = F^-T [mu (G + G^T + G^T G) + lam ln J I] = cof(F) M / J
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T lnJ = t_log1p(jm1);
        T GtG[9], M[9], C[9];
        mulTN3(G, G, GtG);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[3 * i + j] = mu * (G[3 * i + j] + G[3 * j + i] + GtG[3 * i + j]);
        const T ll = lam * lnJ;
        M[0] += ll;
        M[4] += ll;
        M[8] += ll;
        cof_IpG(G, C);
        mul3(C, M, P);
        const T iJ = T(1) / J;
#pragma unroll
        for (int k = 0; k < 9; ++k) P[k] *= iJ;
        return J > T(0);
    }
}

// dP = dP/dF : dF at G.
template <class T, int MODEL> __device__ __forceinline__ bool dstress(T mu, T lam, const T *G, const T *dF, T *dP) {
    if (MODEL == EBBX_STVK) {
        // dP = dF S + F dS, dS = 2 mu sym(F^T dF) + lam tr(F^T dF) I
        T S[9], A[9], GtdF[9];
        stvk_S(mu, lam, G, S);
        mulTN3(G, dF, GtdF);
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = dF[k] + GtdF[k];   // F^T dF
        T dS[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dS[3 * i + j] = mu * (A[3 * i + j] + A[3 * j + i]);
        const T lt = lam * (A[0] + A[4] + A[8]);
        dS[0] += lt;
        dS[4] += lt;
        dS[8] += lt;
        T dFS[9], GdS[9];
        mul3(dF, S, dFS);
        mul3(G, dS, GdS);
#pragma unroll
        for (int k = 0; k < 9; ++k) dP[k] = dFS[k] + dS[k] + GdS[k];
        return true;
    } else {
        // dP = mu dF + (mu - lam ln J) N dF^T N + lam (N : dF) N, N = F^-T
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T lnJ = t_log1p(jm1);
        T N[9];
        cof_IpG(G, N);
        const T iJ = T(1) / J;
#pragma unroll
        for (int k = 0; k < 9; ++k) N[k] *= iJ;
        T X[9], Y[9];
        mulNT3(N, dF, X);   // N dF^T
        mul3(X, N, Y);      // N dF^T N
        T ndf = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) ndf += N[k] * dF[k];
        const T c = mu - lam * lnJ;
        const T ln = lam * ndf;
#pragma unroll
        for (int k = 0; k < 9; ++k) dP[k] = mu * dF[k] + c * Y[k] + ln * N[k];
        return J > T(0);
    }
}

// The 12 diagonal entries K[(a,c),(a,c)] = -V0 dP(e_c b_a^T) : (e_c b_a^T) of one tet,
// in closed form for a rank-one dF = e_c b^T:
//   StVK: b^T S b + mu (|f_c|^2 |b|^2 + (f_c . b)^2) + lam (f_c . b)^2, f_c = row c of F
//   NH:   mu |b|^2 + (mu + lam (1 - ln J)) ((N b)_c)^2
template <class T, int MODEL> __device__ __forceinline__ bool diag12(T mu, T lam, const T *G, const T *b, T V0, T *h) {
    T ba[4][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        ba[1][j] = b[j];
        ba[2][j] = b[3 + j];
        ba[3][j] = b[6 + j];
        ba[0][j] = -(b[j] + b[3 + j] + b[6 + j]);
    }
    if (MODEL == EBBX_STVK) {
        T S[9];
        stvk_S(mu, lam, G, S);
        T F[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) F[k] = G[k];
        F[0] += T(1);
        F[4] += T(1);
        F[8] += T(1);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const T *v = ba[a];
            T Sb0 = S[0] * v[0] + S[1] * v[1] + S[2] * v[2];
            T Sb1 = S[3] * v[0] + S[4] * v[1] + S[5] * v[2];
            T Sb2 = S[6] * v[0] + S[7] * v[1] + S[8] * v[2];
            const T bSb = v[0] * Sb0 + v[1] * Sb1 + v[2] * Sb2;
            const T bb = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T fb = F[3 * c] * v[0] + F[3 * c + 1] * v[1] + F[3 * c + 2] * v[2];
                const T ff = F[3 * c] * F[3 * c] + F[3 * c + 1] * F[3 * c + 1] + F[3 * c + 2] * F[3 * c + 2];
                h[3 * a + c] = -V0 * (bSb + mu * (ff * bb + fb * fb) + lam * fb * fb);
            }
        }
        return true;
    } else {
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T lnJ = t_log1p(jm1);
        T N[9];
        cof_IpG(G, N);
        const T iJ = T(1) / J;
#pragma unroll
        for (int k = 0; k < 9; ++k) N[k] *= iJ;
        const T cc = mu + lam * (T(1) - lnJ);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const T *v = ba[a];
            const T bb = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T nb = N[3 * c] * v[0] + N[3 * c + 1] * v[1] + N[3 * c + 2] * v[2];
                h[3 * a + c] = -V0 * (mu * bb + cc * nb * nb);
            }
        }
        return J > T(0);
    }
}

// ---- gather / element evaluation ----------------------------------------------------

// M = dD B with dD = [q1-q0 | q2-q0 | q3-q0]; differences in FP64, then rounded to T
template <class T>
__device__ __forceinline__ void grad_from(const double (&q)[4][3], const T *b, T *M) {
    T D[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) D[3 * r + c] = (T)(q[c + 1][r] - q[0][r]);
    mul3(D, b, M);
}

// H = -V0 P B^T -> corners 1..3 get the columns of H, corner 0 minus their sum
template <class T> __device__ __forceinline__ void corner_forces(const T *P, const T *b, T V0, T *h) {
    T H[9];
    mulNT3(P, b, H);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const T h1 = -V0 * H[3 * r], h2 = -V0 * H[3 * r + 1], h3 = -V0 * H[3 * r + 2];
        h[3 + r] = h1;
        h[6 + r] = h2;
        h[9 + r] = h3;
        h[r] = -(h1 + h2 + h3);
    }
}

template <class T, int MODEL, int OP>
__device__ __forceinline__ bool eval_tet(T mu, T lam, const T *b, T V0, const double (&qd)[4][3],
                                         const double (&qu)[4][3], T *h) {
    T G[9];
    grad_from(qd, b, G);
    if (OP == OP_FORCE) {
        T P[9];
        bool ok = stress<T, MODEL>(mu, lam, G, P);
        corner_forces(P, b, V0, h);
        return ok;
    } else if (OP == OP_KMUL) {
        T dF[9], dP[9];
        grad_from(qu, b, dF);
        bool ok = dstress<T, MODEL>(mu, lam, G, dF, dP);
        corner_forces(dP, b, V0, h);
        return ok;
    } else {
        return diag12<T, MODEL>(mu, lam, G, b, V0, h);
    }
}

// ---- the element kernel ------------------------------------------------------------

template <class T, int MODEL, int OP, int SC>
__global__ __launch_bounds__(256) void k_elem(ElemArgs a) {
    const int64_t nt = a.nt, nv = a.nv;
    extern __shared__ double s_dyn[];
    if (a.skip && *a.skip) return;   // uniform over the grid
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;

    // block strategy: stage the block's vertices in LDS
    int nvb = 0, vbase = 0;
    double *s_d = s_dyn, *s_u = nullptr, *s_acc = nullptr;
    if (SC == SC_BLOCK) {
        vbase = a.blk_vptr[blockIdx.x];
        nvb = a.blk_vptr[blockIdx.x + 1] - vbase;
        const int nq = (OP == OP_KMUL) ? 2 : 1;
        s_u = s_d + 3 * nvb;
        s_acc = s_d + 3 * nq * nvb;
        for (int i = threadIdx.x; i < nvb; i += blockDim.x) {
            const int64_t gv = a.blk_verts[vbase + i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s_d[k * nvb + i] = a.d[k * nv + gv];
                if (OP == OP_KMUL) s_u[k * nvb + i] = a.u[k * nv + gv];
                s_acc[k * nvb + i] = 0.0;
            }
        }
        __syncthreads();
    }

    if (t < nt) {
        const T *Bp = (const T *)a.B;
        T b[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) b[k] = Bp[k * nt + t];
        const T V0 = ((const T *)a.V0)[t];
        T mu, lam;
        if (a.mat) {
            mu = ((const T *)a.mat)[t];
            lam = ((const T *)a.mat)[nt + t];
        } else {
            mu = (T)a.mu;
            lam = (T)a.lam;
        }
        double qd[4][3], qu[4][3];
        int slot[4];
        int64_t v[4];
        if (SC == SC_BLOCK) {
#pragma unroll
            for (int c = 0; c < 4; ++c) slot[c] = a.blk_local[c * nt + t];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    qd[c][k] = s_d[k * nvb + slot[c]];
                    qu[c][k] = (OP == OP_KMUL) ? s_u[k * nvb + slot[c]] : 0.0;
                }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = a.keys[c * nt + t];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    qd[c][k] = a.d[k * nv + v[c]];
                    qu[c][k] = (OP == OP_KMUL) ? a.u[k * nv + v[c]] : 0.0;
                }
        }
        T h[12];
        const bool ok = eval_tet<T, MODEL, OP>(mu, lam, b, V0, qd, qu, h);
        if (MODEL == EBBX_NH && !ok && OP == OP_FORCE) atomicAdd(a.n_inv, 1ull);
        if (SC == SC_ATOMIC) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) atomicAdd(&a.out[k * nv + v[c]], (double)h[3 * c + k]);
        } else if (SC == SC_PART) {
            T *pp = (T *)a.part + 12 * t;
#pragma unroll
            for (int k = 0; k < 12; ++k) pp[k] = h[k];
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) atomicAdd(&s_acc[k * nvb + slot[c]], (double)h[3 * c + k]);
        }
    }

    if (SC == SC_BLOCK) {
        __syncthreads();
        for (int i = threadIdx.x; i < nvb; i += blockDim.x) {
            const int64_t gv = a.blk_verts[vbase + i];
            const bool own = a.blk_own[vbase + i] != 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double val = s_acc[k * nvb + i];
                if (own)
                    a.out[k * nv + gv] = val;   // sole writer; out was pre-set for accumulate
                else
                    atomicAdd(&a.out[k * nv + gv], val);
            }
        }
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

// Zero only the vertices the block strategy adds atomically into.
__global__ void k_zero_shared(double *out, int64_t nv, const int32_t *verts, const uint8_t *own, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!own[i]) {
            const int64_t v = verts[i];
            out[v] = 0.0;
            out[nv + v] = 0.0;
            out[2 * nv + v] = 0.0;
        }
}

__global__ void k_axpy_inplace(double *y, const double *x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
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

template <class T, int MODEL, int OP, int SC>
static void launch_k(const ElemArgs &a, int block, size_t shmem, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_elem<T, MODEL, OP, SC>), dim3(grid), dim3(block), shmem, s, a);
    HIPCHK(hipGetLastError());
}

template <class T, int MODEL, int OP>
static void launch_sc(int sc, const ElemArgs &a, int block, size_t shmem, unsigned grid, hipStream_t s) {
    if (sc == SC_ATOMIC) launch_k<T, MODEL, OP, SC_ATOMIC>(a, block, shmem, grid, s);
    else if (sc == SC_PART) launch_k<T, MODEL, OP, SC_PART>(a, block, shmem, grid, s);
    else launch_k<T, MODEL, OP, SC_BLOCK>(a, block, shmem, grid, s);
}

template <class T>
static void launch_model_op(int model, ElemOp op, int sc, const ElemArgs &a, int block, size_t shmem, unsigned grid,
                            hipStream_t s) {
    if (model == EBBX_STVK) {
        if (op == OP_FORCE) launch_sc<T, EBBX_STVK, OP_FORCE>(sc, a, block, shmem, grid, s);
        else if (op == OP_KMUL) launch_sc<T, EBBX_STVK, OP_KMUL>(sc, a, block, shmem, grid, s);
        else launch_sc<T, EBBX_STVK, OP_DIAG>(sc, a, block, shmem, grid, s);
    } else {
        if (op == OP_FORCE) launch_sc<T, EBBX_NH, OP_FORCE>(sc, a, block, shmem, grid, s);
        else if (op == OP_KMUL) launch_sc<T, EBBX_NH, OP_KMUL>(sc, a, block, shmem, grid, s);
        else launch_sc<T, EBBX_NH, OP_DIAG>(sc, a, block, shmem, grid, s);
    }
}

static ElemArgs base_args(ebbx_fem_s *F) {
    ElemArgs a{};
    a.nt = F->nt;
    a.nv = F->nv;
    a.keys = F->keys;
    a.B = F->B.get();
    a.V0 = F->V0.get();
    a.mat = F->per_tet ? F->mat.get() : nullptr;
    a.mu = F->mu;
    a.lam = F->lam;
    a.n_inv = F->status.as<unsigned long long>();
    a.blk_vptr = F->blk_vptr.as<int32_t>();
    a.blk_verts = F->blk_verts.as<int32_t>();
    a.blk_own = F->blk_own.as<uint8_t>();
    a.blk_local = F->blk_local.as<uint16_t>();
    return a;
}

void elem_launch(ebbx_fem_s *F, ElemOp op, const double *d, const double *u, double *out, int accumulate,
                 hipStream_t s, const int *skip) {
    const int64_t nt = F->nt, nv = F->nv;
    if (nv == 0) return;
    if (nt == 0) {
        if (!accumulate) fill_f64(out, 3 * nv, 0.0, s);
        return;
    }
    ElemArgs a = base_args(F);
    a.d = d;
    a.u = u;
    a.out = out;
    a.part = F->part.get();
    a.skip = skip;
    const int sc = F->strategy == EBBX_STRAT_SEG ? SC_PART : F->strategy == EBBX_STRAT_BLOCK ? SC_BLOCK : SC_ATOMIC;
    int block = F->block > 0 ? F->block : 256;
    size_t shmem = 0;
    unsigned grid = grid_n(nt, block, 1ll << 31);
    double *target = out;
    if (sc == SC_BLOCK) {
        block = F->blk_tets;
        grid = (unsigned)F->nblk;
        const int nq = (op == OP_KMUL) ? 2 : 1;
        shmem = (size_t)3 * (nq + 1) * F->blk_maxv * sizeof(double);
        if (shmem > 64 * 1024)
            fail(EBBX_E_STATE, "block strategy needs %zu bytes of LDS per block (%d vertices); reorder the mesh "
                 "(Morton) or use a smaller block", shmem, F->blk_maxv);
        if (accumulate) {
            // owned vertices are stored, not added: reduce into zeroed scratch, then add
            target = F->scratch.as<double>();
            a.out = target;
            fill_f64(target, 3 * nv, 0.0, s);
        } else {
            // zero what is added atomically (shared and isolated vertices)
            hipLaunchKernelGGL(k_zero_shared, dim3(grid_n(F->blk_nverts, 256, 8192)), dim3(256), 0, s, target, nv,
                               F->blk_verts.as<int32_t>(), F->blk_own.as<uint8_t>(), F->blk_nverts);
            HIPCHK(hipGetLastError());
        }
    } else if (sc == SC_ATOMIC && !accumulate) {
        fill_f64(out, 3 * nv, 0.0, s);
    }
    if (F->prec == EBBX_F32) launch_model_op<float>(F->model, op, sc, a, block, shmem, grid, s);
    else launch_model_op<double>(F->model, op, sc, a, block, shmem, grid, s);
    if (sc == SC_PART) {
        const unsigned g = grid_n(nv, 256, 1ll << 31);
        if (F->prec == EBBX_F32)
            hipLaunchKernelGGL(k_seg_gather<float>, dim3(g), dim3(256), 0, s, (const float *)F->part.get(),
                               F->group->row_ptr.as<int64_t>(), F->group->inc.as<int32_t>(), nv, out, accumulate);
        else
            hipLaunchKernelGGL(k_seg_gather<double>, dim3(g), dim3(256), 0, s, (const double *)F->part.get(),
                               F->group->row_ptr.as<int64_t>(), F->group->inc.as<int32_t>(), nv, out, accumulate);
        HIPCHK(hipGetLastError());
    }
    if (sc == SC_BLOCK && accumulate) {
        hipLaunchKernelGGL(k_axpy_inplace, dim3(grid_n(3 * nv, 256, 8192)), dim3(256), 0, s, out,
                           (const double *)target, 3 * nv);
        HIPCHK(hipGetLastError());
    }
}

// ---- energy ------------------------------------------------------------------------------

template <class T, int MODEL>
__global__ __launch_bounds__(256) void k_energy(ElemArgs a, double *part) {
    __shared__ double s_w[4];
    const int64_t nt = a.nt, nv = a.nv;
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        double b[9];
        for (int k = 0; k < 9; ++k) b[k] = (double)((const T *)a.B)[k * nt + t];
        const double V0 = (double)((const T *)a.V0)[t];
        double mu = a.mu, lam = a.lam;
        if (a.mat) {
            mu = (double)((const T *)a.mat)[t];
            lam = (double)((const T *)a.mat)[nt + t];
        }
        double q[4][3];
        for (int c = 0; c < 4; ++c) {
            const int64_t v = a.keys[c * nt + t];
            for (int k = 0; k < 3; ++k) q[c][k] = a.d[k * nv + v];
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
    a.d = d;
    const unsigned g = 1024;
    double *part = F->scratch.as<double>();   // scratch holds >= 3 nv >= 1024 doubles
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

// ---- block tables -----------------------------------------------------------------------

// Tets are cut into blocks of blk_tets consecutive rows.  Per block: the sorted
// set of vertices it touches, each corner's slot in that set, and whether the
// block holds every incident tet of a vertex (then it is the vertex's only
// writer and stores instead of adding atomically).
void build_blocks(ebbx_fem_s *F, hipStream_t s) {
    const int64_t nt = F->nt, nv = F->nv;
    const int bt = F->block > 0 ? F->block : 256;
    F->blk_tets = bt;
    F->nblk = (nt + bt - 1) / bt;
    std::vector<int32_t> keys((size_t)(4 * nt));
    if (nt > 0) HIPCHK(hipMemcpy(keys.data(), F->keys, keys.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> rp((size_t)(nv + 1));
    HIPCHK(hipMemcpy(rp.data(), F->group->row_ptr.get(), rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> vptr((size_t)F->nblk + 2, 0), verts;
    std::vector<uint8_t> own;
    std::vector<uint16_t> local((size_t)(4 * nt));
    verts.reserve((size_t)(nt + 16));
    own.reserve((size_t)(nt + 16));
    std::vector<std::pair<int32_t, int32_t>> buf;   // (vertex, corner index in block)
    int32_t maxv = 1;
    for (int64_t b = 0; b < F->nblk; ++b) {
        const int64_t t0 = b * bt, t1 = std::min<int64_t>(nt, t0 + bt);
        buf.clear();
        for (int64_t t = t0; t < t1; ++t)
            for (int c = 0; c < 4; ++c) buf.push_back({keys[(size_t)(c * nt + t)], (int32_t)(c * bt + (t - t0))});
        std::sort(buf.begin(), buf.end());
        int32_t nb = 0;
        size_t i = 0;
        while (i < buf.size()) {
            size_t j = i;
            while (j < buf.size() && buf[j].first == buf[i].first) ++j;
            const int32_t v = buf[i].first;
            for (size_t k = i; k < j; ++k) {
                const int c = buf[k].second / bt, tl = buf[k].second % bt;
                local[(size_t)(c * nt + t0 + tl)] = (uint16_t)nb;
            }
            verts.push_back(v);
            own.push_back((int64_t)(j - i) == rp[(size_t)v + 1] - rp[(size_t)v] ? 1 : 0);
            ++nb;
            i = j;
        }
        maxv = std::max(maxv, nb);
        vptr[(size_t)b + 1] = (int32_t)verts.size();
    }
    if (maxv > 65535) fail(EBBX_E_ARG, "block touches %d vertices (limit 65535)", maxv);
    vptr[(size_t)F->nblk + 1] = maxv;
    // vertices no tet touches: listed after the blocks as shared, so that they are zeroed
    for (int64_t v = 0; v < nv; ++v)
        if (rp[(size_t)v + 1] == rp[(size_t)v]) {
            verts.push_back((int32_t)v);
            own.push_back(0);
        }
    F->blk_maxv = maxv;
    F->blk_nverts = (int64_t)verts.size();
    F->blk_vptr.reset(vptr.size() * sizeof(int32_t), s);
    F->blk_verts.reset(std::max<size_t>(verts.size(), 1) * sizeof(int32_t), s);
    F->blk_own.reset(std::max<size_t>(own.size(), 1), s);
    F->blk_local.reset(std::max<size_t>(local.size(), 1) * sizeof(uint16_t), s);
    HIPCHK(hipMemcpy(F->blk_vptr.get(), vptr.data(), vptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!verts.empty()) {
        HIPCHK(hipMemcpy(F->blk_verts.get(), verts.data(), verts.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(F->blk_own.get(), own.data(), own.size(), hipMemcpyHostToDevice));
    }
    if (!local.empty())
        HIPCHK(hipMemcpy(F->blk_local.get(), local.data(), local.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    F->blocks_built = true;
}

}  // namespace ebbx
