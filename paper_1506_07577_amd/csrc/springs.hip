// springs.hip -- the spring-mass workload of the paper's introductory example
// (a spring on every directed edge of a tet mesh; Ebb by example), on the same
// relational runtime as the FEM domain.
//
//  - rest lengths: one pass over the edges (the example's per-edge kernel);
//  - forces: each vertex loops over the edges leaving it (the grouping of the
//    edges by their tail key-field) and reduces (+=) the spring forces into its
//    force field: four lanes per vertex, each lane a stride of the vertex's
//    edges with two edges' loads in flight, the row sum a fixed butterfly over
//    the four lanes, one division per edge and K applied to the sum;
//  - apply: the exclusive per-vertex update (integrate, clear the force);
//  - kinetic energy: a global += as a fixed-order two-pass sum;
//  - run: nsteps replayed from a captured HIP graph of 32 steps, each step one
//    fused kernel (forces and update of a vertex together, positions ping-ponged
//    through a second buffer so that no vertex reads an advanced neighbour).
// Springs restore: edge (v -> h) adds K (dq - L dq/|dq|), dq = q_h - q_v.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "fem.h"

struct ebbx_springs_s {
    const ebbx_relation_s *edges = nullptr, *verts = nullptr;   // the relations the row copies follow
    int64_t nv = 0, ne = 0;
    double K = 0.0;
    ebbx::DevBuf row;    // int32 (nv + 1): vertex v's edges are [row[v], row[v+1])
    ebbx::DevBuf head;   // int32 (ne): head vertex of each edge, in row order
    ebbx::DevBuf rest;   // FP64 (ne): rest length of each edge, in row order
    ebbx::DevBuf part;   // FP64 partials of the energy sum
    ebbx::DevBuf q2;     // FP64 (3 nv): the other position buffer of the fused steps of a run
    // captured steps of ebbx_springs_run
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
    const void *key[4] = {nullptr, nullptr, nullptr, nullptr};
    double key_dt = 0.0;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~ebbx_springs_s() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace ebbx {

namespace {

constexpr int LANES = 4;              // lanes per vertex in the force pass (14 edges per interior vertex)
constexpr int UNROLL = 2;             // edges per lane with their loads in flight together
constexpr int RUN_CHUNK = 32;         // steps per captured graph
constexpr int EN_THREADS = 256;

std::mutex g_mu;
std::set<ebbx_springs_s *> g_springs;

}  // namespace

const char *springs_relation_user(const ebbx_relation_s *r) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const ebbx_springs_s *S : g_springs)
        if (S->edges == r || S->verts == r) return "a springs domain";
    return nullptr;
}

namespace {

ebbx_springs_s *check_springs(ebbx_springs p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!p || !g_springs.count(p)) fail(EBBX_E_ARG, "invalid springs handle");
    return p;
}

unsigned blocks_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// Row-order copies of the heads and the rest lengths |X_h - X_v|.
__global__ void k_spring_setup(const int64_t *rp, const int32_t *inc, const int32_t *head_rel, const double *X,
                               int64_t nv, int32_t *row, int32_t *head, double *rest) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > nv) return;
    row[v] = (int32_t)rp[v];
    if (v == nv) return;
    const double x0 = X[v], x1 = X[nv + v], x2 = X[2 * nv + v];
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
        const int32_t h = head_rel[inc[p]];
        head[p] = h;
        const double a = X[h] - x0, b = X[nv + h] - x1, c = X[2 * nv + h] - x2;
        rest[p] = sqrt(a * a + b * b + c * c);
    }
}

// Sum over the edges leaving vertex v ([e0, e1) of the rows) of dq - L dq/|dq|, dq = q_h - q_v
// (K is applied once to the sum): lane `lane` of the vertex's L lanes takes edges e0 + lane,
// e0 + lane + L, ..., with the loads of U edges in flight at once; the lane sums are then
// combined by a fixed butterfly, so every lane returns the same, order-fixed total.
template <int L, int U>
__device__ __forceinline__ void spring_sum(const int32_t *head, const double *rest, const double *q, uint32_t nv,
                                           uint32_t v, int32_t e0, int32_t e1, uint32_t lane, double &f0, double &f1,
                                           double &f2) {
    const double q0 = q[v], q1 = q[nv + v], q2 = q[2 * nv + v];
    f0 = f1 = f2 = 0.0;
    for (int32_t e = e0 + (int32_t)lane; e < e1; e += U * L) {
        uint32_t h[U];
        double len[U], a[U], b[U], c[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = e + u * L < e1;
            h[u] = ok[u] ? (uint32_t)head[e + u * L] : v;
            len[u] = ok[u] ? rest[e + u * L] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = q[h[u]] - q0;
            b[u] = q[nv + h[u]] - q1;
            c[u] = q[2 * nv + h[u]] - q2;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const double n = sqrt(a[u] * a[u] + b[u] * b[u] + c[u] * c[u]);
            const double sc = n > 0.0 ? len[u] / n : 0.0;   // a zero-length spring pulls with K dq
            f0 += fma(-sc, a[u], a[u]);
            f1 += fma(-sc, b[u], b[u]);
            f2 += fma(-sc, c[u], c[u]);
        }
    }
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) {
        f0 += __shfl_xor(f0, m, L);
        f1 += __shfl_xor(f1, m, L);
        f2 += __shfl_xor(f2, m, L);
    }
}

// The exclusive update of one vertex component: a = f / m, q += qd dt + a dt^2 / 2, qd += a dt.
// Both the update pass and the fused step call it, so the two agree bit for bit.
__device__ __forceinline__ void integrate(double q, double qd, double a, double dt, double &q_new, double &qd_new) {
    q_new = q + (qd * dt + 0.5 * a * dt * dt);
    qd_new = qd + a * dt;
}

// Force pass: lanes 0..2 of each vertex's group store (or += into) the x, y, z components.
template <int L, int U>
__global__ __launch_bounds__(256) void k_spring_forces(const int32_t *row, const int32_t *head, const double *rest,
                                                       double K, const double *q, double *f, uint32_t nv,
                                                       int accumulate) {
    // XCD x takes one contiguous range of vertices (Morton-ordered), whose neighbours' positions
    // it then mostly finds in its own L2
    const uint32_t g = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / L;
    const uint32_t lane = threadIdx.x % L;
    const uint32_t v = g < nv ? g : nv - 1;   // whole groups stay in the shuffles
    const int32_t e0 = row[v], e1 = g < nv ? row[v + 1] : e0;
    double f0, f1, f2;
    spring_sum<L, U>(head, rest, q, nv, v, e0, e1, lane, f0, f1, f2);
    if (g < nv && lane < 3) {
        const size_t i = (size_t)lane * nv + v;
        double fk = K * (lane == 0 ? f0 : lane == 1 ? f1 : f2);
        if (accumulate) fk += f[i];
        f[i] = fk;
    }
}

// One whole step for every vertex (forces from q, then the exclusive update) writing the new
// positions to q_out, so that no vertex reads a position already advanced.  With take_f the
// force field's contents join the spring forces and are cleared, as in the separate passes.
template <int L, int U>
__global__ __launch_bounds__(256) void k_spring_step(const int32_t *row, const int32_t *head, const double *rest,
                                                     double K, const double *mass, double dt, const double *q,
                                                     double *q_out, double *qd, double *f, int take_f, uint32_t nv) {
    // XCD x takes one contiguous range of vertices (Morton-ordered), whose neighbours' positions
    // it then mostly finds in its own L2
    const uint32_t g = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / L;
    const uint32_t lane = threadIdx.x % L;
    const uint32_t v = g < nv ? g : nv - 1;
    const int32_t e0 = row[v], e1 = g < nv ? row[v + 1] : e0;
    double f0, f1, f2;
    spring_sum<L, U>(head, rest, q, nv, v, e0, e1, lane, f0, f1, f2);
    if (g < nv && lane < 3) {
        const size_t i = (size_t)lane * nv + v;
        double fk = K * (lane == 0 ? f0 : lane == 1 ? f1 : f2);
        if (take_f) {
            fk += f[i];
            f[i] = 0.0;
        }
        integrate(q[i], qd[i], fk / mass[v], dt, q_out[i], qd[i]);
    }
}

__global__ void k_spring_apply(const double *mass, double dt, double *q, double *qd, double *f, int64_t nv) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const double m = mass[v];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t i = k * nv + v;
            integrate(q[i], qd[i], f[i] / m, dt, q[i], qd[i]);
            f[i] = 0.0;
        }
    }
}

__device__ __forceinline__ double block_total(double x, double *s4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = x;
    __syncthreads();
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// pass 1: one partial per workgroup (fixed order); pass 2: their fixed-order sum added to E
__global__ __launch_bounds__(EN_THREADS) void k_kinetic_part(const double *mass, const double *qd, int64_t nv,
                                                             double *part) {
    __shared__ double s4[4];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (v < nv) {
        const double a = qd[v], b = qd[nv + v], c = qd[2 * nv + v];
        e = 0.5 * mass[v] * (a * a + b * b + c * c);
    }
    e = block_total(e, s4);
    if (threadIdx.x == 0) part[blockIdx.x] = e;
}

__global__ __launch_bounds__(EN_THREADS) void k_kinetic_sum(const double *part, int n, double *E) {
    __shared__ double s4[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += EN_THREADS) acc += part[i];
    acc = block_total(acc, s4);
    if (threadIdx.x == 0) E[0] += acc;
}

void launch_forces(ebbx_springs_s *S, const double *q, double *f, int accumulate, hipStream_t s) {
    if (S->nv == 0) return;
    hipLaunchKernelGGL((k_spring_forces<LANES, UNROLL>), dim3(blocks_of(S->nv * LANES, 256)), dim3(256), 0, s,
                       S->row.as<int32_t>(), S->head.as<int32_t>(), S->rest.as<double>(), S->K, q, f,
                       (uint32_t)S->nv, accumulate);
    HIPCHK(hipGetLastError());
}

void launch_step(ebbx_springs_s *S, const double *mass, double dt, const double *q, double *q_out, double *qd,
                 double *f, int take_f, hipStream_t s) {
    hipLaunchKernelGGL((k_spring_step<LANES, UNROLL>), dim3(blocks_of(S->nv * LANES, 256)), dim3(256), 0, s,
                       S->row.as<int32_t>(), S->head.as<int32_t>(), S->rest.as<double>(), S->K, mass, dt, q, q_out,
                       qd, f, take_f, (uint32_t)S->nv);
    HIPCHK(hipGetLastError());
}

void launch_apply(ebbx_springs_s *S, const double *mass, double dt, double *q, double *qd, double *f, hipStream_t s) {
    if (S->nv == 0) return;
    hipLaunchKernelGGL(k_spring_apply, dim3(std::min<unsigned>(blocks_of(S->nv, 256), 16384)), dim3(256), 0, s, mass,
                       dt, q, qd, f, S->nv);
    HIPCHK(hipGetLastError());
}

// n steps ending with the positions in q: fused steps in pairs (q -> q2 -> q), the first of
// them taking the force field's contents; an odd n starts with one step of the separate passes.
void emit_steps(ebbx_springs_s *S, const double *mass, double dt, int32_t n, double *q, double *qd, double *force,
                hipStream_t s) {
    int32_t k = 0;
    if (n % 2) {
        launch_forces(S, q, force, 1, s);
        launch_apply(S, mass, dt, q, qd, force, s);
        k = 1;
    }
    double *q2 = S->q2.as<double>();
    for (; k < n; k += 2) {
        launch_step(S, mass, dt, q, q2, qd, force, k == 0, s);
        launch_step(S, mass, dt, q2, q, qd, force, 0, s);
    }
}

void check_vec(const void *p, const char *what, int64_t nv) {
    if (nv > 0 && !p) fail(EBBX_E_ARG, "%s is NULL", what);
}

}  // namespace
}  // namespace ebbx

using namespace ebbx;

extern "C" ebbx_status ebbx_springs_create(ebbx_relation edges, const char *tail, const char *head, ebbx_relation verts,
                                          const char *pos_field, double K, ebbx_springs *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    auto *er = check_rel(edges);
    auto *vr = check_rel(verts);
    if (!tail || !head || !pos_field) fail(EBBX_E_ARG, "a field name is NULL");
    if (!std::isfinite(K)) fail(EBBX_E_ARG, "K must be finite");
    KeyField &kt = get_key(er, tail);
    KeyField &kh = get_key(er, head);
    if (kt.target != vr || kh.target != vr) fail(EBBX_E_ARG, "tail and head must target '%s'", vr->name.c_str());
    if (kt.arity != 1 || kh.arity != 1) fail(EBBX_E_SHAPE, "tail and head must have arity 1");
    const Field &X = get_field(vr, pos_field, EBBX_F64, 3);
    auto S = std::make_unique<ebbx_springs_s>();
    S->edges = er;
    S->verts = vr;
    S->nv = vr->size;
    S->ne = er->size;
    S->K = K;
    if (S->ne >= (int64_t(1) << 31)) fail(EBBX_E_ARG, "too many edges");
    auto g = build_group(er, tail, nullptr);
    S->row.reset((size_t)(S->nv + 1) * sizeof(int32_t));
    S->head.reset((size_t)std::max<int64_t>(S->ne, 1) * sizeof(int32_t));
    S->rest.reset((size_t)std::max<int64_t>(S->ne, 1) * sizeof(double));
    S->part.reset((size_t)blocks_of(std::max<int64_t>(S->nv, 1), EN_THREADS) * sizeof(double));
    hipLaunchKernelGGL(k_spring_setup, dim3(blocks_of(S->nv + 1, 256)), dim3(256), 0, nullptr,
                       g->row_ptr.as<int64_t>(), g->inc.as<int32_t>(), kh.ptr, (const double *)X.ptr, S->nv,
                       S->row.as<int32_t>(), S->head.as<int32_t>(), S->rest.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    HIPCHK(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_springs.insert(S.get());
    }
    *out = S.release();
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_destroy(ebbx_springs sp) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    HIPCHK(hipDeviceSynchronize());
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_springs.erase(S);
    }
    delete S;
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_rest(ebbx_springs sp, double *rest_dev, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    if (S->ne > 0 && !rest_dev) fail(EBBX_E_ARG, "rest_dev is NULL");
    if (S->ne > 0)
        HIPCHK(hipMemcpyAsync(rest_dev, S->rest.get(), (size_t)S->ne * sizeof(double), hipMemcpyDeviceToDevice,
                              (hipStream_t)stream));
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_forces(ebbx_springs sp, const double *q, double *force, int32_t accumulate,
                                          ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    check_vec(q, "q", S->nv);
    check_vec(force, "force", S->nv);
    if (S->nv > 0 && overlap(q, force, (size_t)(3 * S->nv) * sizeof(double))) fail(EBBX_E_PHASE, "force aliases q");
    launch_forces(S, q, force, accumulate, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_apply(ebbx_springs sp, const double *mass, double dt, double *q, double *qd,
                                         double *force, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    const int64_t nv = S->nv;
    for (const void *p : {(const void *)mass, (const void *)q, (const void *)qd, (const void *)force})
        check_vec(p, "a vertex field", nv);
    if (!std::isfinite(dt)) fail(EBBX_E_ARG, "dt must be finite");
    const size_t b = (size_t)(3 * nv) * sizeof(double);
    if (nv > 0 && (overlap(q, qd, b) || overlap(q, force, b) || overlap(qd, force, b)))
        fail(EBBX_E_PHASE, "q, qd and force must not alias");
    launch_apply(S, mass, dt, q, qd, force, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_kinetic_energy(ebbx_springs sp, const double *mass, const double *qd, double *E_dev,
                                                  ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    if (!E_dev) fail(EBBX_E_ARG, "E_dev is NULL");
    check_vec(mass, "mass", S->nv);
    check_vec(qd, "qd", S->nv);
    if (S->nv == 0) return EBBX_OK;
    hipStream_t s = (hipStream_t)stream;
    const unsigned nb = blocks_of(S->nv, EN_THREADS);
    hipLaunchKernelGGL(k_kinetic_part, dim3(nb), dim3(EN_THREADS), 0, s, mass, qd, S->nv, S->part.as<double>());
    hipLaunchKernelGGL(k_kinetic_sum, dim3(1), dim3(EN_THREADS), 0, s, (const double *)S->part.get(), (int)nb, E_dev);
    HIPCHK(hipGetLastError());
    EBBX_API_END
}

extern "C" ebbx_status ebbx_springs_run(ebbx_springs sp, const double *mass, double dt, int32_t nsteps, double *q,
                                       double *qd, double *force, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *S = check_springs(sp);
    const int64_t nv = S->nv;
    if (nsteps < 0) fail(EBBX_E_ARG, "nsteps must be >= 0");
    for (const void *p : {(const void *)mass, (const void *)q, (const void *)qd, (const void *)force})
        check_vec(p, "a vertex field", nv);
    if (!std::isfinite(dt)) fail(EBBX_E_ARG, "dt must be finite");
    const size_t b = (size_t)(3 * nv) * sizeof(double);
    if (nv > 0 && (overlap(q, qd, b) || overlap(q, force, b) || overlap(qd, force, b)))
        fail(EBBX_E_PHASE, "q, qd and force must not alias");
    if (nv == 0 || nsteps == 0) return EBBX_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!S->q2.get()) S->q2.reset((size_t)(3 * nv) * sizeof(double), s);
    const void *key[4] = {mass, q, qd, force};
    if (nsteps >= RUN_CHUNK && (!S->exec || !std::equal(key, key + 4, S->key) || S->key_dt != dt)) {
        S->drop_graph();
        HIPCHK(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
        CaptureGuard guard(S->cap);
        emit_steps(S, mass, dt, RUN_CHUNK, q, qd, force, S->cap);
        guard.disarm();
        HIPCHK(hipStreamEndCapture(S->cap, &S->graph));
        HIPCHK(hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0));
        std::copy(key, key + 4, S->key);
        S->key_dt = dt;
    }
    int32_t left = nsteps;
    for (; left >= RUN_CHUNK; left -= RUN_CHUNK) HIPCHK(hipGraphLaunch(S->exec, s));
    emit_steps(S, mass, dt, left, q, qd, force, s);
    EBBX_API_END
}
