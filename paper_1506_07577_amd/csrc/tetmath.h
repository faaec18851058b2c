// tetmath.h -- per-tet hyperelastic element math shared by the element maps
// and the stiffness assembly: loads through scalar bases, the displacement-
// gradient (G-form) stress, its first and second directional derivatives,
// the Jacobi diagonal and the per-tet evaluation of each element map.
#pragma once

#include "fem.h"

namespace ebbx {

// ---- scalar helpers ------------------------------------------------------------

// Element idx of a column: a 64-bit base in scalar registers plus a 32-bit byte
// offset (sizes are checked on the host so that idx * sizeof(T) fits 32 bits).
template <class T> __device__ __forceinline__ T ldc(const void *base, uint32_t idx) {
    return *(const T *)((const char *)base + idx * (uint32_t)sizeof(T));
}
template <class T> __device__ __forceinline__ void stc(void *base, uint32_t idx, T v) {
    *(T *)((char *)base + idx * (uint32_t)sizeof(T)) = v;
}
template <class T> __device__ __forceinline__ T *atc(void *base, uint32_t idx) {
    return (T *)((char *)base + idx * (uint32_t)sizeof(T));
}

__device__ __forceinline__ float t_rcp(float x) { return __builtin_amdgcn_rcpf(x); }   // 1 ulp
__device__ __forceinline__ double t_rcp(double x) { return 1.0 / x; }

// ln(1 + x).  Near zero (|x| < 1/4, the range of elastic volume change met in
// practice) through ln(1+x) = 2 atanh(s), s = x / (2 + x), and the odd series
// of atanh to s^9 (truncation below 1e-9 relative); elsewhere the library log1p.
__device__ __forceinline__ float t_log1p(float x) {
    if (fabsf(x) < 0.25f) {
        const float s = x * __builtin_amdgcn_rcpf(2.0f + x);
        const float s2 = s * s;
        float p = fmaf(s2, 1.0f / 9.0f, 1.0f / 7.0f);
        p = fmaf(s2, p, 0.2f);
        p = fmaf(s2, p, 1.0f / 3.0f);
        return 2.0f * fmaf(s * s2, p, s);
    }
    return log1pf(x);
}
__device__ __forceinline__ double t_log1p(double x) { return log1p(x); }

// ---- 3x3 algebra on registers (row-major, M[3*i + j]) ---------------------------

template <class T> __device__ __forceinline__ T det3(const T *A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Rest volume from B = Dm^-1: V0 = det(Dm)/6 = 1/(6 det B).  The element maps
// derive it instead of streaming a V0 column (one load fewer per tet).
template <class T> __device__ __forceinline__ T tet_V0(const T *b) { return t_rcp(T(6) * det3(b)); }

// C = A B
template <class T> __device__ __forceinline__ void mul3(const T *A, const T *B, T *C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// C = A0 + A B
template <class T> __device__ __forceinline__ void muladd3(const T *A0, const T *A, const T *B, T *C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A0[3 * i + j] + A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
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

// G^T G (symmetric), as the full 3x3
template <class T> __device__ __forceinline__ void gtg_sym(const T *G, T *S) {
    S[0] = G[0] * G[0] + G[3] * G[3] + G[6] * G[6];
    S[4] = G[1] * G[1] + G[4] * G[4] + G[7] * G[7];
    S[8] = G[2] * G[2] + G[5] * G[5] + G[8] * G[8];
    S[1] = S[3] = G[0] * G[1] + G[3] * G[4] + G[6] * G[7];
    S[2] = S[6] = G[0] * G[2] + G[3] * G[5] + G[6] * G[8];
    S[5] = S[7] = G[1] * G[2] + G[4] * G[5] + G[7] * G[8];
}

// ---- constitutive models: each returns -V0 P (or -V0 dP) -----------------------------

// StVK S = 2 mu E + lam tr(E) I, E = (G + G^T + G^T G)/2, scaled by `sc`
template <class T> __device__ __forceinline__ void stvk_S(T mu, T lam, const T *G, T sc, T *S) {
    T Q[9];
    gtg_sym(G, Q);
    const T e00 = G[0] + T(0.5) * Q[0], e11 = G[4] + T(0.5) * Q[4], e22 = G[8] + T(0.5) * Q[8];
    const T e01 = T(0.5) * (G[1] + G[3] + Q[1]), e02 = T(0.5) * (G[2] + G[6] + Q[2]),
            e12 = T(0.5) * (G[5] + G[7] + Q[5]);
    const T m2 = T(2) * mu * sc, le = lam * (e00 + e11 + e22) * sc;
    S[0] = m2 * e00 + le;
    S[4] = m2 * e11 + le;
    S[8] = m2 * e22 + le;
    S[1] = S[3] = m2 * e01;
    S[2] = S[6] = m2 * e02;
    S[5] = S[7] = m2 * e12;
}

// -V0 P(F); returns false for an inverted neo-Hookean element
template <class T, int MODEL> __device__ __forceinline__ bool stress_scaled(T mu, T lam, T V0, const T *G, T *P) {
    if (MODEL == EBBX_STVK) {
        T S[9];
        stvk_S(mu, lam, G, -V0, S);
        muladd3(S, G, S, P);   // P = S + G S
        return true;
    } else {
        // P = F^-T [mu (G + G^T + G^T G) + lam ln J I] = cof(F) M / J
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T iJ = t_rcp(J);
        const T lnJ = t_log1p(jm1);
        T Q[9], M[9], C[9];
        gtg_sym(G, Q);
        const T ms = -V0 * iJ * mu, ll = -V0 * iJ * lam * lnJ;
        M[0] = ms * (T(2) * G[0] + Q[0]) + ll;
        M[4] = ms * (T(2) * G[4] + Q[4]) + ll;
        M[8] = ms * (T(2) * G[8] + Q[8]) + ll;
        M[1] = M[3] = ms * (G[1] + G[3] + Q[1]);
        M[2] = M[6] = ms * (G[2] + G[6] + Q[2]);
        M[5] = M[7] = ms * (G[5] + G[7] + Q[5]);
        cof_IpG(G, C);
        mul3(C, M, P);
        return J > T(0);
    }
}

// -V0 dP, dP = dP/dF : dF at G
template <class T, int MODEL>
__device__ __forceinline__ bool dstress_scaled(T mu, T lam, T V0, const T *G, const T *dF, T *dP) {
    if (MODEL == EBBX_STVK) {
        // dP = dF S + F dS, dS = 2 mu sym(F^T dF) + lam tr(F^T dF) I
        T S[9], A[9];
        stvk_S(mu, lam, G, -V0, S);
        T GtdF[9];
        mulTN3(G, dF, GtdF);
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = dF[k] + GtdF[k];   // F^T dF
        const T mv = -V0 * mu, lt = -V0 * lam * (A[0] + A[4] + A[8]);
        T dS[9];
        dS[0] = T(2) * mv * A[0] + lt;
        dS[4] = T(2) * mv * A[4] + lt;
        dS[8] = T(2) * mv * A[8] + lt;
        dS[1] = dS[3] = mv * (A[1] + A[3]);
        dS[2] = dS[6] = mv * (A[2] + A[6]);
        dS[5] = dS[7] = mv * (A[5] + A[7]);
        T X[9];
        muladd3(dS, G, dS, X);   // F dS = dS + G dS
        muladd3(X, dF, S, dP);   // + dF S
        return true;
    } else {
        // dP = mu dF + (mu - lam ln J) N dF^T N + lam (N : dF) N, N = cof(F) / J
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T iJ = t_rcp(J);
        const T lnJ = t_log1p(jm1);
        T C[9];
        cof_IpG(G, C);
        T X[9], Y[9];
        mulNT3(C, dF, X);   // C dF^T
        mul3(X, C, Y);      // C dF^T C
        T cdf = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) cdf += C[k] * dF[k];
        const T iJ2 = iJ * iJ;
        const T a = -V0 * mu, bY = -V0 * (mu - lam * lnJ) * iJ2, bC = -V0 * lam * cdf * iJ2;
#pragma unroll
        for (int k = 0; k < 9; ++k) dP[k] = a * dF[k] + bY * Y[k] + bC * C[k];
        return J > T(0);
    }
}

// -V0 d2P[A, W]: the derivative of dP[A] along W (symmetric in A and W)
template <class T, int MODEL>
__device__ __forceinline__ bool d2stress_scaled(T mu, T lam, T V0, const T *G, const T *A, const T *W, T *Q) {
    if (MODEL == EBBX_STVK) {
        // P = F S: d2P[A,W] = A S'[W] + W S'[A] + F S''[A,W],
        // S'[X] = 2 mu sym(F^T X) + lam tr(F^T X) I, S''[A,W] = 2 mu sym(A^T W) + lam tr(A^T W) I
        T FtA[9], FtW[9], AtW[9], GtA[9], GtW[9];
        mulTN3(G, A, GtA);
        mulTN3(G, W, GtW);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            FtA[k] = A[k] + GtA[k];
            FtW[k] = W[k] + GtW[k];
        }
        mulTN3(A, W, AtW);
        T SA[9], SW[9], S2[9];
        const T m = -V0 * mu, l = -V0 * lam;
        const T la = l * (FtA[0] + FtA[4] + FtA[8]), lw = l * (FtW[0] + FtW[4] + FtW[8]),
                l2 = l * (AtW[0] + AtW[4] + AtW[8]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                SA[3 * i + j] = m * (FtA[3 * i + j] + FtA[3 * j + i]);
                SW[3 * i + j] = m * (FtW[3 * i + j] + FtW[3 * j + i]);
                S2[3 * i + j] = m * (AtW[3 * i + j] + AtW[3 * j + i]);
            }
        SA[0] += la; SA[4] += la; SA[8] += la;
        SW[0] += lw; SW[4] += lw; SW[8] += lw;
        S2[0] += l2; S2[4] += l2; S2[8] += l2;
        T X[9], Y[9];
        mul3(A, SW, X);
        muladd3(X, W, SA, Y);     // A S'[W] + W S'[A]
        muladd3(Y, G, S2, X);     // + G S''
#pragma unroll
        for (int k = 0; k < 9; ++k) Q[k] = X[k] + S2[k];   // + S'' (the I of F = I + G)
        return true;
    } else {
        // d/dW of  mu A + c N A^T N + lam (N:A) N,  dN[W] = -N W^T N,  dc[W] = -lam (N:W)
        const T jm1 = jm1_of(G);
        const T J = T(1) + jm1;
        const T iJ = t_rcp(J);
        const T lnJ = t_log1p(jm1);
        T N[9];
        cof_IpG(G, N);
#pragma unroll
        for (int k = 0; k < 9; ++k) N[k] *= iJ;
        T NAt[9], NAtN[9], NWt[9], NWtN[9], X1[9], X2[9];
        mulNT3(N, A, NAt);
        mul3(NAt, N, NAtN);
        mulNT3(N, W, NWt);
        mul3(NWt, N, NWtN);
        mulNT3(NWtN, A, X1);   // N W^T N A^T
        mul3(X1, N, X2);       // N W^T N A^T N
        mulNT3(NAtN, W, X1);   // N A^T N W^T
        T X3[9];
        mul3(X1, N, X3);       // N A^T N W^T N
        T NA = T(0), NW = T(0), NWNA = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            NA += N[k] * A[k];
            NW += N[k] * W[k];
            NWNA += NWtN[k] * A[k];
        }
        const T c = mu - lam * lnJ;
        const T s1 = V0 * lam * NW, s2 = V0 * lam * NA, s3 = V0 * c, s4 = V0 * lam * NWNA;
#pragma unroll
        for (int k = 0; k < 9; ++k) Q[k] = s1 * NAtN[k] + s2 * NWtN[k] + s3 * (X2[k] + X3[k]) + s4 * N[k];
        return J > T(0);
    }
}

// The 12 diagonal entries K[(a,c),(a,c)] = -V0 dP(e_c b_a^T) : (e_c b_a^T) of one
// tet, in closed form for a rank-one dF = e_c b^T:
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
        stvk_S(mu, lam, G, T(1), S);
        T F[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) F[k] = G[k];
        F[0] += T(1);
        F[4] += T(1);
        F[8] += T(1);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const T *v = ba[a];
            const T Sb0 = S[0] * v[0] + S[1] * v[1] + S[2] * v[2];
            const T Sb1 = S[3] * v[0] + S[4] * v[1] + S[5] * v[2];
            const T Sb2 = S[6] * v[0] + S[7] * v[1] + S[8] * v[2];
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
        const T iJ = t_rcp(J);
        const T lnJ = t_log1p(jm1);
        T N[9];
        cof_IpG(G, N);
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

// ---- tet blocks -------------------------------------------------------------------

// B = Dm^-1 and V0 = det(Dm)/6 of one tet from its corners' rest positions staged in
// LDS (three columns of stride S): Dm from FP64 differences rounded to T, then the
// adjugate over the determinant.  Recomputing B costs ~60 VALU per tet and saves the
// 9 per-tet B values (36 B in FP32) of the stream.
template <class T>
__device__ __forceinline__ void rest_B(const double *s_x, uint32_t S, const uint32_t *sl, T *b, T &V0) {
    double x0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) x0[k] = s_x[k * S + sl[0]];
    T Dm[9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) Dm[3 * k + c] = (T)(s_x[k * S + sl[c + 1]] - x0[k]);
    const T det = det3(Dm);
    const T idet = t_rcp(det);
    b[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) * idet;
    b[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) * idet;
    b[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) * idet;
    b[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) * idet;
    b[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) * idet;
    b[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) * idet;
    b[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) * idet;
    b[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) * idet;
    b[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) * idet;
    V0 = det * T(1.0 / 6.0);
}

// The same from block-local FP32 rest positions (each block vertex's offset from the block's
// first vertex, precomputed once): Dm from FP32 differences of the offsets.
__device__ __forceinline__ void rest_B_local(const float *s_xf, uint32_t S, const uint32_t *sl, float *b, float &V0) {
    float x0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) x0[k] = s_xf[k * S + sl[0]];
    float Dm[9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) Dm[3 * k + c] = s_xf[k * S + sl[c + 1]] - x0[k];
    const float det = det3(Dm);
    const float idet = t_rcp(det);
    b[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) * idet;
    b[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) * idet;
    b[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) * idet;
    b[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) * idet;
    b[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) * idet;
    b[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) * idet;
    b[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) * idet;
    b[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) * idet;
    b[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) * idet;
    V0 = det * (1.0f / 6.0f);
}

// ---- gather / element evaluation ----------------------------------------------------

// M = dD B with dD = [q1-q0 | q2-q0 | q3-q0]; differences in FP64, then rounded to T
template <class T> __device__ __forceinline__ void grad_from(const double (&q)[4][3], const T *b, T *M) {
    T D[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) D[3 * r + c] = (T)(q[c + 1][r] - q[0][r]);
    mul3(D, b, M);
}

// H = Ps B^T (Ps already carries -V0): corners 1..3 get the columns of H,
// corner 0 minus their sum.  h[3 a + r].
template <class T> __device__ __forceinline__ void corner_out(const T *Ps, const T *b, T *h) {
    T H[9];
    mulNT3(Ps, b, H);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        h[3 + r] = H[3 * r];
        h[6 + r] = H[3 * r + 1];
        h[9 + r] = H[3 * r + 2];
        h[r] = -(H[3 * r] + H[3 * r + 1] + H[3 * r + 2]);
    }
}

template <class T, int MODEL, int OP>
__device__ __forceinline__ bool eval_tet(T mu, T lam, const T *b, T V0, const double (&qd)[4][3],
                                         const double (&qu)[4][3], T *h, const double (*qw)[3] = nullptr) {
    T G[9];
    grad_from(qd, b, G);
    if (OP == OP_TMUL) {
        T FA[9], FW[9], Q[9];
        grad_from(qu, b, FA);
        grad_from(*(const double(*)[4][3])qw, b, FW);
        const bool ok = d2stress_scaled<T, MODEL>(mu, lam, V0, G, FA, FW, Q);
        corner_out(Q, b, h);
        return ok;
    }
    if (OP == OP_FORCE) {
        T P[9];
        const bool ok = stress_scaled<T, MODEL>(mu, lam, V0, G, P);
        corner_out(P, b, h);
        return ok;
    } else if (OP == OP_KMUL) {
        T dF[9], dP[9];
        grad_from(qu, b, dF);
        const bool ok = dstress_scaled<T, MODEL>(mu, lam, V0, G, dF, dP);
        corner_out(dP, b, h);
        return ok;
    } else {
        return diag12<T, MODEL>(mu, lam, G, b, V0, h);
    }
}

}  // namespace ebbx
