// fem.hip -- the tet-FEM domain object, its C-ABI, and the implicit step.
//
// The implicit step is the linearised backward-Euler step of the paper's Vega
// workload, solved with a Jacobi-preconditioned conjugate gradient written as
// data-parallel kernels (Performance Evaluation, Vega).  CG scalars live on
// the device; dot products are two-pass block reductions whose first pass is
// fused into the vector kernels (Runtime Implementation, "Reductions"), with
// wavefront shuffles and a fixed summation order so results are reproducible.
// The iterations are captured once into a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

#include "fem.h"

namespace ebbx {

// CG state kept on the device.
struct CGState {
    double rz, rr, pq, alpha, beta, bnorm;
    int iters, status, done, converged;
    unsigned long long n_inv;
};

constexpr int VT = 256;          // threads of the vertex kernels
constexpr int NPB_MAX = 1024;    // blocks of the vertex kernels (fixed per nv: deterministic partials)

static int npb_for(int64_t nv) { return (int)std::max<int64_t>(1, std::min<int64_t>(NPB_MAX, (nv + VT - 1) / VT)); }

// Sum of one double over a 256-thread block (fixed order).
__device__ __forceinline__ double block_sum(double x, double *s4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = x;
    __syncthreads();
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// Fixed-order sum of n partials with stride 2 (offset o) in one block.
__device__ __forceinline__ double sum_parts(const double *part, int n, int o, double *sbuf) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[2 * i + o];
    return block_sum(acc, sbuf);
}

struct StepVec {
    double *dn, *vn, *f, *y, *r, *z, *p, *q, *x, *diag;
};

__global__ void k_step_begin(CGState *st, unsigned long long *n_inv) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rz = st->rr = st->pq = st->alpha = st->beta = st->bnorm = 0.0;
        st->iters = 0;
        st->status = EBBX_OK;
        st->done = 0;
        st->converged = 0;
        st->n_inv = 0;
        *n_inv = 0ull;
    }
}

// b = dt (f + M g + dt K v); diag = M - dt^2 Kdiag (1 on pinned rows); r = Pi b;
// z = D^-1 r; p = z; x = 0; partials (r.z, r.r)
// mode 0 (step): b = dt (f + M g + dt y), with f = f(d_n) and y = K(d_n) v_n;
// mode 1 (adjoint solve): b = f, the right-hand side placed in f beforehand.
__global__ __launch_bounds__(VT) void k_step_rhs(StepVec w, const double *mass, const uint8_t *pinned, int64_t nv,
                                                 double dt, double gx, double gy, double gz, int precond, int mode,
                                                 double *part) {
    __shared__ double s4[4];
    double rz = 0.0, rr = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x; v < nv; v += (int64_t)gridDim.x * VT) {
        const double m = mass[v];
        const bool pin = pinned[v] != 0;
        const double g[3] = {gx, gy, gz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            const double b = mode ? w.f[i] : dt * (w.f[i] + m * g[k] + dt * w.y[i]);
            const double dg = pin ? 1.0 : (precond ? m - dt * dt * w.diag[i] : 1.0);
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
        part[2 * blockIdx.x] = rz;
        part[2 * blockIdx.x + 1] = rr;
    }
}

__global__ __launch_bounds__(VT) void k_step_init(CGState *st, const double *part, int npb,
                                                  const unsigned long long *n_inv) {
    __shared__ double s4[4];
    const double rz = sum_parts(part, npb, 0, s4);
    const double rr = sum_parts(part, npb, 1, s4);
    if (threadIdx.x == 0) {
        st->rz = rz;
        st->rr = rr;
        st->bnorm = sqrt(rr);
        st->n_inv = *n_inv;
        if (st->n_inv > 0) {
            st->status = EBBX_E_INVERTED;
            st->done = 1;
        } else if (rr == 0.0) {
            st->done = 1;
            st->converged = 1;
        }
    }
}

// q = Pi (M p - dt^2 y); partial p.q
__global__ __launch_bounds__(VT) void k_cg_Ap(StepVec w, const double *mass, const uint8_t *pinned, int64_t nv,
                                              double dt, const CGState *st, double *part) {
    __shared__ double s4[4];
    if (st->done) return;
    double pq = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x; v < nv; v += (int64_t)gridDim.x * VT) {
        const double m = mass[v];
        const bool pin = pinned[v] != 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            const double p = w.p[i];
            const double q = pin ? 0.0 : m * p - dt * dt * w.y[i];
            w.q[i] = q;
            pq += p * q;
        }
    }
    pq = block_sum(pq, s4);
    if (threadIdx.x == 0) part[2 * blockIdx.x] = pq;
}

__global__ __launch_bounds__(VT) void k_cg_alpha(CGState *st, const double *part, int npb) {
    __shared__ double s4[4];
    if (st->done) return;
    const double pq = sum_parts(part, npb, 0, s4);
    if (threadIdx.x == 0) {
        st->pq = pq;
        if (!(pq > 0.0)) {
            st->status = EBBX_E_NOT_SPD;
            st->done = 1;
        } else {
            st->alpha = st->rz / pq;
        }
    }
}

// x += alpha p; r -= alpha q; z = D^-1 r; partials (r.z, r.r)
__global__ __launch_bounds__(VT) void k_cg_update(StepVec w, int64_t nv, const CGState *st, double *part) {
    __shared__ double s4[4];
    if (st->done) return;
    const double alpha = st->alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x; v < nv; v += (int64_t)gridDim.x * VT) {
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
        part[2 * blockIdx.x] = rz;
        part[2 * blockIdx.x + 1] = rr;
    }
}

__global__ __launch_bounds__(VT) void k_cg_beta(CGState *st, const double *part, int npb, double tol, int maxit) {
    __shared__ double s4[4];
    if (st->done) return;
    const double rz = sum_parts(part, npb, 0, s4);
    const double rr = sum_parts(part, npb, 1, s4);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = rr;
        if (sqrt(rr) <= tol * st->bnorm || rz == 0.0) {
            st->converged = 1;
            st->done = 1;
        } else {
            st->beta = rz / st->rz;
            st->rz = rz;
            if (st->iters >= maxit) st->done = 1;
        }
    }
}

// p = z + beta p
__global__ __launch_bounds__(VT) void k_cg_p(StepVec w, int64_t nv, const CGState *st) {
    if (st->done) return;
    const double beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * VT)
        w.p[i] = w.z[i] + beta * w.p[i];
}

// diag = m - dt^2 Kdiag
__global__ void k_diag_finish(double *dg, const double *m, int64_t nv, double dt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * blockDim.x)
        dg[i] = m[i % nv] - dt * dt * dg[i];
}

__global__ void k_copy_in(const double *d, const double *v, double *dn, double *vn, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        dn[i] = d[i];
        vn[i] = v[i];
    }
}

// v = v_n + x, d = d_n + dt v (unless the solve broke down); stats out
__global__ void k_step_end(StepVec w, int64_t n, double dt, double tol, const CGState *st, double *d, double *v,
                           ebbx_step_stats *stats) {
    const bool apply = st->status == EBBX_OK;
    if (apply)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
            const double vv = w.vn[i] + w.x[i];
            v[i] = vv;
            d[i] = w.dn[i] + dt * vv;
        }
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) {
        int status = st->status;
        if (status == EBBX_OK && !st->converged && tol > 0.0) status = EBBX_E_NOT_CONVERGED;
        stats->iters = st->iters;
        stats->status = status;
        stats->rel_res = st->bnorm > 0.0 ? sqrt(st->rr) / st->bnorm : 0.0;
        stats->n_inverted = (int64_t)st->n_inv;
    }
}

// adjoint: d_n copied in, g^ = gv + dt gx into f (the solve's right-hand side)
__global__ void k_vjp_prep(const double *d, const double *gx, const double *gv, double dt, StepVec w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w.dn[i] = d[i];
        w.f[i] = gv[i] + dt * gx[i];
    }
}

// adjoint: d_bar = gx + dt K w + dt^2 T[v', w];  v_bar = g^ + dt^2 K w
// (K w in y, T[v', w] in q, g^ in f); stats out
__global__ void k_vjp_end(StepVec w, const double *gx, double dt, int64_t n, double *d_bar, double *v_bar,
                          const CGState *st, double tol, ebbx_step_stats *stats) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double kw = w.y[i];
        d_bar[i] = gx[i] + dt * kw + dt * dt * w.q[i];
        v_bar[i] = w.f[i] + dt * dt * kw;
    }
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) {
        int status = st->status;
        if (status == EBBX_OK && !st->converged && tol > 0.0) status = EBBX_E_NOT_CONVERGED;
        stats->iters = st->iters;
        stats->status = status;
        stats->rel_res = st->bnorm > 0.0 ? sqrt(st->rr) / st->bnorm : 0.0;
        stats->n_inverted = (int64_t)st->n_inv;
    }
}

}  // namespace ebbx

using namespace ebbx;

struct ebbx_fem_s::Step {
    DevBuf vec, part, state;
    StepVec w{};
    int npb = 1;
    // graphs: preambles of the step (0) and of the adjoint solve (1), and a chunk of CG iterations
    hipGraphExec_t pre[2] = {nullptr, nullptr}, chunk = nullptr;
    hipGraph_t g_pre[2] = {nullptr, nullptr}, g_chunk = nullptr;
    hipStream_t cap = nullptr;
    int chunk_iters = 0;
    // parameters baked into the graphs
    double dt = -1, g[3] = {0, 0, 0}, tol = -1;
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
    }
    ~Step() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (h_done) (void)hipHostFree(h_done);
    }
};

ebbx_fem_s::~ebbx_fem_s() = default;

namespace {

std::mutex g_fem_mu;
std::set<ebbx_fem_s *> g_fems;

ebbx_fem_s *check_fem(ebbx_fem f) {
    std::lock_guard<std::mutex> lk(g_fem_mu);
    if (!f || !g_fems.count(f)) fail(EBBX_E_ARG, "invalid FEM handle");
    return f;
}

bool overlap(const void *a, const void *b, size_t bytes) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

// `block`: threads per workgroup for ATOMIC and SEG (64..256, multiple of 64);
// tets per block for BLOCK (64, 128, 256, 512 or 1024).  0 = default.
void set_strategy(ebbx_fem_s *F, int32_t strategy, int32_t block, hipStream_t s) {
    if (strategy < EBBX_STRAT_AUTO || strategy > EBBX_STRAT_BLOCK_LDS) fail(EBBX_E_ARG, "bad strategy %d", strategy);
    if (strategy == EBBX_STRAT_AUTO) strategy = EBBX_STRAT_BLOCK;
    if (strategy == EBBX_STRAT_BLOCK || strategy == EBBX_STRAT_BLOCK_LDS) {
        const int32_t bt = block ? block : 256;
        if (bt > 512) fail(EBBX_E_ARG, "block strategies take at most 512 tets per block");
        if (!F->blocks_built || F->blk_tets != bt) build_blocks(F, bt, s);
        F->strategy = strategy;
        F->blk_red = strategy == EBBX_STRAT_BLOCK_LDS ? 1 : 0;
        F->block = bt;
        return;
    }
    if (block != 0 && (block < 64 || block > 256 || block % 64))
        fail(EBBX_E_ARG, "block %d must be a multiple of 64 in [64, 256]", block);
    if (strategy == EBBX_STRAT_SEG && !F->part.get())
        F->part.reset((size_t)std::max<int64_t>(F->nt, 1) * 12 * F->esize, s);
    F->strategy = strategy;
    F->block = block ? block : 256;
}

}  // namespace

extern "C" {

ebbx_status ebbx_fem_create(ebbx_relation tets, const char *keyfield, ebbx_relation verts, const char *pos_field,
                            const char *pinned_field, const ebbx_fem_params *params, ebbx_fem *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = nullptr;
    if (!params) fail(EBBX_E_ARG, "params is NULL");
    auto *tr = check_rel(tets);
    auto *vr = check_rel(verts);
    KeyField &kf = get_key(tr, keyfield);
    if (kf.target != vr) fail(EBBX_E_ARG, "key-field '%s' does not target '%s'", keyfield, vr->name.c_str());
    if (kf.arity != 4) fail(EBBX_E_SHAPE, "key-field '%s' has arity %d, tets need 4", keyfield, kf.arity);
    const Field &X = get_field(vr, pos_field, EBBX_F64, 3);
    const uint8_t *pin = nullptr;
    if (pinned_field) pin = (const uint8_t *)get_field(vr, pinned_field, EBBX_U8, 1).ptr;
    const double *E_tet = nullptr;
    if (params->E_field) E_tet = (const double *)get_field(tr, params->E_field, EBBX_F64, 1).ptr;
    if (params->model != EBBX_STVK && params->model != EBBX_NH) fail(EBBX_E_ARG, "bad model %d", params->model);
    if (params->elem_prec != EBBX_F32 && params->elem_prec != EBBX_F64) fail(EBBX_E_DTYPE, "elem_prec must be F32 or F64");
    if (!(params->rho > 0.0)) fail(EBBX_E_ARG, "rho must be > 0");
    if (!(params->nu > -1.0 && params->nu < 0.5)) fail(EBBX_E_ARG, "nu must be in (-1, 0.5)");
    // kernels address columns with 32-bit byte offsets (8-byte elements)
    if (tr->size >= (int64_t(1) << 29) || vr->size >= (int64_t(1) << 29))
        fail(EBBX_E_ARG, "FEM relations are limited to 2^29 rows");
    hipStream_t s = nullptr;
    std::unique_ptr<ebbx_fem_s> F(new ebbx_fem_s());
    F->tets = tr;
    F->verts = vr;
    F->keyname = keyfield;
    F->keys = kf.ptr;
    F->nt = tr->size;
    F->nv = vr->size;
    F->model = params->model;
    F->prec = params->elem_prec;
    F->esize = F->prec == EBBX_F32 ? 4 : 8;
    F->rho = params->rho;
    F->E = params->E;
    F->nu = params->nu;
    F->mu = params->E / (2.0 * (1.0 + params->nu));
    F->lam = params->E * params->nu / ((1.0 + params->nu) * (1.0 - 2.0 * params->nu));
    F->per_tet = E_tet != nullptr;
    F->E_tet = E_tet;
    F->group = build_group(tr, keyfield, s);
    const int64_t nt = std::max<int64_t>(F->nt, 1), nv = std::max<int64_t>(F->nv, 1);
    F->B.reset((size_t)nt * 9 * F->esize, s);
    F->V0.reset((size_t)nt * F->esize, s);
    if (F->per_tet) F->mat.reset((size_t)nt * 2 * F->esize, s);
    F->mass.reset((size_t)nv * sizeof(double), s);
    F->pinned.reset((size_t)nv, s);
    F->status.reset(sizeof(unsigned long long) * 4, s);
    F->scratch.reset((size_t)std::max<int64_t>(3 * nv, 4096) * sizeof(double), s);
    HIPCHK(hipMemsetAsync(F->status.get(), 0, sizeof(unsigned long long) * 4, s));
    if (pin) HIPCHK(hipMemcpyAsync(F->pinned.get(), pin, (size_t)F->nv, hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemsetAsync(F->pinned.get(), 0, (size_t)nv, s));
    const int64_t nbad = elem_precompute(F.get(), (const double *)X.ptr, E_tet, s);
    if (nbad > 0) fail(EBBX_E_DEGENERATE, "%lld rest tets have V0 <= 0", (long long)nbad);
    set_strategy(F.get(), params->strategy, params->block, s);
    HIPCHK(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lk(g_fem_mu);
        g_fems.insert(F.get());
    }
    *out = F.release();
    EBBX_API_END
}

ebbx_status ebbx_fem_destroy(ebbx_fem fem) {
    EBBX_API_BEGIN
    check_fem(fem);
    HIPCHK(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lk(g_fem_mu);
        g_fems.erase(fem);
    }
    delete fem;
    EBBX_API_END
}

ebbx_status ebbx_fem_set_strategy(ebbx_fem fem, int32_t strategy, int32_t block) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    HIPCHK(hipDeviceSynchronize());
    set_strategy(F, strategy, block, nullptr);
    HIPCHK(hipDeviceSynchronize());
    EBBX_API_END
}

ebbx_status ebbx_fem_get_strategy(ebbx_fem fem, int32_t *strategy, int32_t *block) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (strategy) *strategy = F->strategy;
    if (block) *block = F->block;
    EBBX_API_END
}

ebbx_status ebbx_fem_forces(ebbx_fem fem, const double *d, double *f, int32_t accumulate, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !f) && F->nv > 0) fail(EBBX_E_ARG, "d or f is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0 && overlap(d, f, bytes)) fail(EBBX_E_PHASE, "f aliases d (read-only and reduce phases overlap)");
    elem_launch(F, OP_FORCE, d, nullptr, f, accumulate ? 1 : 0, (hipStream_t)stream);
    EBBX_API_END
}

ebbx_status ebbx_fem_Kmul(ebbx_fem fem, const double *d, const double *u, double *y, int32_t accumulate,
                          ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !u || !y) && F->nv > 0) fail(EBBX_E_ARG, "d, u or y is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0 && (overlap(d, y, bytes) || overlap(u, y, bytes)))
        fail(EBBX_E_PHASE, "y aliases d or u (read-only and reduce phases overlap)");
    elem_launch(F, OP_KMUL, d, u, y, accumulate ? 1 : 0, (hipStream_t)stream);
    EBBX_API_END
}

ebbx_status ebbx_fem_energy(ebbx_fem fem, const double *d, double *out_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (!out_dev || (!d && F->nv > 0)) fail(EBBX_E_ARG, "d or out_dev is NULL");
    elem_energy(F, d, out_dev, (hipStream_t)stream);
    EBBX_API_END
}

ebbx_status ebbx_fem_jacobi_diag(ebbx_fem fem, const double *d, double dt, double *diag, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !diag) && F->nv > 0) fail(EBBX_E_ARG, "d or diag is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0 && overlap(d, diag, bytes)) fail(EBBX_E_PHASE, "diag aliases d");
    hipStream_t s = (hipStream_t)stream;
    elem_launch(F, OP_DIAG, d, nullptr, diag, 0, s);
    if (F->nv > 0) {
        hipLaunchKernelGGL(k_diag_finish, dim3(npb_for(3 * F->nv)), dim3(VT), 0, s, diag, F->mass.as<double>(), F->nv, dt);
        HIPCHK(hipGetLastError());
    }
    EBBX_API_END
}

ebbx_status ebbx_fem_mass(ebbx_fem fem, double *mass_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (!mass_dev && F->nv > 0) fail(EBBX_E_ARG, "mass_dev is NULL");
    if (F->nv > 0)
        HIPCHK(hipMemcpyAsync(mass_dev, F->mass.get(), (size_t)F->nv * sizeof(double), hipMemcpyDeviceToDevice,
                              (hipStream_t)stream));
    EBBX_API_END
}

ebbx_status ebbx_fem_status(ebbx_fem fem, int64_t *n_inverted, int32_t reset, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long h = 0;
    HIPCHK(hipMemcpyAsync(&h, F->status.get(), sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (reset) {
        HIPCHK(hipMemsetAsync(F->status.get(), 0, sizeof(unsigned long long), s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (n_inverted) *n_inverted = (int64_t)h;
    EBBX_API_END
}

}  // extern "C"

// ---- implicit step ----------------------------------------------------------------------

namespace {

void capture_begin(hipStream_t cap) { HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)); }

hipGraphExec_t capture_end(hipStream_t cap, hipGraph_t *g) {
    HIPCHK(hipStreamEndCapture(cap, g));
    hipGraphExec_t ex = nullptr;
    HIPCHK(hipGraphInstantiate(&ex, *g, nullptr, nullptr, 0));
    return ex;
}

// Capture the preamble of `mode` (0: step, 1: adjoint solve) and, if the
// parameters changed, the CG chunk shared by both.
void build_graphs(ebbx_fem_s *F, const ebbx_step_params &p, int mode) {
    auto &S = *F->step;
    const bool same = S.dt == p.dt && !std::memcmp(S.g, p.g, sizeof S.g) && S.tol == p.tol && S.maxit == p.maxit &&
                      S.precond == p.precond && S.strategy == F->strategy && S.block == F->block && S.chunk;
    if (!same) S.drop_graphs();
    if (S.pre[mode] && S.chunk) return;
    const int64_t nv = F->nv;
    const int npb = S.npb;
    CGState *st = S.state.as<CGState>();
    double *part = S.part.as<double>();
    unsigned long long *n_inv = F->status.as<unsigned long long>();
    hipStream_t cs = S.cap;
    // preamble: (step) forces and K v; Jacobi diagonal; rhs; initial residual
    capture_begin(cs);
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, cs, st, n_inv);
    if (mode == 0) {
        elem_launch(F, OP_FORCE, S.w.dn, nullptr, S.w.f, 0, cs);
        elem_launch(F, OP_KMUL, S.w.dn, S.w.vn, S.w.y, 0, cs);
    }
    if (p.precond == EBBX_PRECOND_JACOBI) elem_launch(F, OP_DIAG, S.w.dn, nullptr, S.w.diag, 0, cs);
    hipLaunchKernelGGL(k_step_rhs, dim3(npb), dim3(VT), 0, cs, S.w, F->mass.as<double>(), F->pinned.as<uint8_t>(), nv,
                       p.dt, p.g[0], p.g[1], p.g[2], p.precond, mode, part);
    hipLaunchKernelGGL(k_step_init, dim3(1), dim3(VT), 0, cs, st, (const double *)part, npb,
                       (const unsigned long long *)n_inv);
    HIPCHK(hipGetLastError());
    S.pre[mode] = capture_end(cs, &S.g_pre[mode]);
    if (!S.chunk) {
        // a chunk of CG iterations, each kernel predicated on the device flag st->done
        S.chunk_iters = std::max(1, std::min(p.maxit, 128));
        capture_begin(cs);
        for (int it = 0; it < S.chunk_iters; ++it) {
            elem_launch(F, OP_KMUL, S.w.dn, S.w.p, S.w.y, 0, cs, &st->done);
            hipLaunchKernelGGL(k_cg_Ap, dim3(npb), dim3(VT), 0, cs, S.w, F->mass.as<double>(), F->pinned.as<uint8_t>(),
                               nv, p.dt, (const CGState *)st, part);
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(VT), 0, cs, st, (const double *)part, npb);
            hipLaunchKernelGGL(k_cg_update, dim3(npb), dim3(VT), 0, cs, S.w, nv, (const CGState *)st, part);
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(VT), 0, cs, st, (const double *)part, npb, p.tol, p.maxit);
            hipLaunchKernelGGL(k_cg_p, dim3(npb), dim3(VT), 0, cs, S.w, nv, (const CGState *)st);
        }
        HIPCHK(hipGetLastError());
        S.chunk = capture_end(cs, &S.g_chunk);
    }
    S.dt = p.dt;
    std::memcpy(S.g, p.g, sizeof S.g);
    S.tol = p.tol;
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
    if (p.precond != EBBX_PRECOND_NONE && p.precond != EBBX_PRECOND_JACOBI) fail(EBBX_E_ARG, "bad precond");
}

void ensure_step(ebbx_fem_s *F, hipStream_t s) {
    if (F->step) return;
    const int64_t nv = F->nv;
    auto S = std::make_unique<ebbx_fem_s::Step>();
    const int64_t n3 = 3 * std::max<int64_t>(nv, 1);
    S->vec.reset((size_t)n3 * 10 * sizeof(double), s);
    double *b = S->vec.as<double>();
    S->w = StepVec{b, b + n3, b + 2 * n3, b + 3 * n3, b + 4 * n3, b + 5 * n3, b + 6 * n3, b + 7 * n3, b + 8 * n3,
                   b + 9 * n3};
    S->npb = npb_for(nv);
    S->part.reset((size_t)S->npb * 2 * sizeof(double), s);
    S->state.reset(sizeof(CGState), s);
    HIPCHK(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void **)&S->h_done, sizeof(int), hipHostMallocDefault));
    HIPCHK(hipStreamSynchronize(s));
    F->step = std::move(S);
}

// Launch the preamble of `mode` and the CG chunks on s.
void run_solve(ebbx_fem_s *F, const ebbx_step_params &p, int mode, hipStream_t s) {
    build_graphs(F, p, mode);
    auto &S = *F->step;
    HIPCHK(hipGraphLaunch(S.pre[mode], s));
    const int nchunks = p.maxit > 0 ? (p.maxit + S.chunk_iters - 1) / S.chunk_iters : 0;
    CGState *st = S.state.as<CGState>();
    for (int c = 0; c < nchunks; ++c) {
        HIPCHK(hipGraphLaunch(S.chunk, s));
        // with a tolerance, stop launching once the device reports convergence
        if (p.tol > 0.0 && c + 1 < nchunks) {
            HIPCHK(hipMemcpyAsync(S.h_done, &st->done, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (*S.h_done) break;
        }
    }
}

}  // namespace

extern "C" ebbx_status ebbx_implicit_step(ebbx_fem fem, double *d, double *v, const ebbx_step_params *params,
                                          ebbx_step_stats *stats_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    check_step_params(params);
    const ebbx_step_params &p = *params;
    const int64_t nv = F->nv;
    if (nv > 0 && (!d || !v)) fail(EBBX_E_ARG, "d or v is NULL");
    if (nv > 0 && overlap(d, v, (size_t)(3 * nv) * sizeof(double))) fail(EBBX_E_PHASE, "d aliases v");
    hipStream_t s = (hipStream_t)stream;
    ensure_step(F, s);
    auto &S = *F->step;
    if (nv > 0) {
        hipLaunchKernelGGL(k_copy_in, dim3(npb_for(3 * nv)), dim3(VT), 0, s, (const double *)d, (const double *)v,
                           S.w.dn, S.w.vn, 3 * nv);
        HIPCHK(hipGetLastError());
    }
    run_solve(F, p, 0, s);
    hipLaunchKernelGGL(k_step_end, dim3(npb_for(3 * std::max<int64_t>(nv, 1))), dim3(VT), 0, s, S.w, 3 * nv, p.dt,
                       p.tol, (const CGState *)S.state.as<CGState>(), d, v, stats_dev);
    HIPCHK(hipGetLastError());
    EBBX_API_END
}

extern "C" ebbx_status ebbx_implicit_step_vjp(ebbx_fem fem, const double *d_n, const double *v_np1,
                                              const ebbx_step_params *params, const double *gx, const double *gv,
                                              double *d_bar, double *v_bar, double *E_bar,
                                              ebbx_step_stats *stats_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
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
        hipLaunchKernelGGL(k_vjp_prep, dim3(npb_for(3 * nv)), dim3(VT), 0, s, d_n, gx, gv, p.dt, S.w, 3 * nv);
        HIPCHK(hipGetLastError());
    }
    // A w = Pi (gv + dt gx), with A = M - dt^2 K(d_n); w ends in x
    run_solve(F, p, 1, s);
    elem_launch(F, OP_KMUL, S.w.dn, S.w.x, S.w.y, 0, s);
    elem_launch(F, OP_TMUL, S.w.dn, v_np1, S.w.q, 0, s, nullptr, S.w.x);
    hipLaunchKernelGGL(k_vjp_end, dim3(npb_for(3 * std::max<int64_t>(nv, 1))), dim3(VT), 0, s, S.w, gx, p.dt, 3 * nv,
                       d_bar, v_bar, (const CGState *)S.state.as<CGState>(), p.tol, stats_dev);
    HIPCHK(hipGetLastError());
    if (E_bar) elem_egrad(F, S.w.dn, v_np1, S.w.x, p.dt, E_bar, s);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_Tmul(ebbx_fem fem, const double *d, const double *a, const double *w, double *out,
                                     int32_t accumulate, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !a || !w || !out) && F->nv > 0) fail(EBBX_E_ARG, "a vector argument is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0 && (overlap(out, d, bytes) || overlap(out, a, bytes) || overlap(out, w, bytes)))
        fail(EBBX_E_PHASE, "out aliases an input");
    elem_launch(F, OP_TMUL, d, a, out, accumulate ? 1 : 0, (hipStream_t)stream, nullptr, w);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_E_grad(ebbx_fem fem, const double *d, const double *v, const double *w, double dt,
                                       double *E_bar, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !v || !w) && F->nv > 0) fail(EBBX_E_ARG, "a vector argument is NULL");
    if (!E_bar && F->nt > 0) fail(EBBX_E_ARG, "E_bar is NULL");
    elem_egrad(F, d, v, w, dt, E_bar, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_set_material(ebbx_fem fem, const double *E_tet, const double *nu_tet, double E,
                                             double nu, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (!E_tet && !(E > 0.0)) fail(EBBX_E_ARG, "E must be > 0");
    if (!nu_tet && !(nu > -1.0 && nu < 0.5)) fail(EBBX_E_ARG, "nu must be in (-1, 0.5)");
    const bool had = F->per_tet;
    elem_set_material(F, E_tet, nu_tet, E, nu, (hipStream_t)stream);
    // captured solver graphs read the material arrays only if they existed then
    if (!had && F->step) F->step->drop_graphs();
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

// ---- cache flush ---------------------------------------------------------------------------

namespace {
// Reads the buffer (clean lines only, so the next kernel does not pay for write-backs).
__global__ void k_flush(const double4 *p, int64_t n, double *sink) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double4 v = p[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc != 0.0) sink[0] = acc;   // the buffer is zero: never taken
}
std::mutex g_flush_mu;
std::map<int, std::pair<void *, size_t>> g_flush_buf;   // per device, kept until the process ends
}  // namespace

extern "C" ebbx_status ebbx_cache_flush(size_t bytes, ebbx_stream stream) {
    EBBX_API_BEGIN
    if (bytes == 0) return EBBX_OK;
    const int dev = current_device();
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_flush_mu);
        auto &e = g_flush_buf[dev];
        if (e.second < bytes) {
            if (e.first) HIPCHK(hipFree(e.first));
            e.first = nullptr;
            e.second = 0;
            HIPCHK(hipMalloc(&e.first, bytes + 64));
            HIPCHK(hipMemset(e.first, 0, bytes + 64));
            e.second = bytes;
        }
        p = e.first;
    }
    const int64_t n = (int64_t)(bytes / sizeof(double4));
    hipLaunchKernelGGL(k_flush, dim3(8192), dim3(256), 0, (hipStream_t)stream, (const double4 *)p, n, (double *)p);
    HIPCHK(hipGetLastError());
    EBBX_API_END
}
