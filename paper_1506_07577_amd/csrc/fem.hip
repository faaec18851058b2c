// fem.hip -- the tet-FEM domain object and its C-ABI: creation, strategies,
// and the element maps (forces, stiffness product, diagonal, energy, adjoint
// products) over the tets relation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

#include "fem.h"

namespace ebbx {

namespace {
constexpr int VT = 256;
unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + VT - 1) / VT)); }
}  // namespace

// diag = m - dt^2 Kdiag
__global__ void k_diag_finish(double *dg, const double *m, int64_t nv, double dt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += (int64_t)gridDim.x * blockDim.x)
        dg[i] = m[i % nv] - dt * dt * dg[i];
}

std::mutex g_fem_mu;
std::set<ebbx_fem_s *> g_fems;

ebbx_fem_s *check_fem(ebbx_fem f) {
    std::lock_guard<std::mutex> lk(g_fem_mu);
    if (!f || !g_fems.count(f)) fail(EBBX_E_ARG, "invalid FEM handle");
    return f;
}

void fem_register(ebbx_fem_s *F) {
    std::lock_guard<std::mutex> lk(g_fem_mu);
    g_fems.insert(F);
}

void fem_unregister(ebbx_fem_s *F) {
    std::lock_guard<std::mutex> lk(g_fem_mu);
    g_fems.erase(F);
}

const char *fem_relation_user(const ebbx_relation_s *r) {
    std::lock_guard<std::mutex> lk(g_fem_mu);
    for (const ebbx_fem_s *F : g_fems)
        if (F->tets == r || F->verts == r) return F->batch_owned ? "the union domain of a batch" : "a FEM domain";
    return nullptr;
}

// `block`: threads per workgroup for ATOMIC and SEG (64..256, multiple of 64);
// tets per block for BLOCK (a multiple of 64 from 64 to 1024).  0 = default.
void set_strategy(ebbx_fem_s *F, int32_t strategy, int32_t block, hipStream_t s) {
    if (strategy < EBBX_STRAT_AUTO || strategy > EBBX_STRAT_LANES) fail(EBBX_E_ARG, "bad strategy %d", strategy);
    // captured solver graphs hold pointers into the block, halo and owner tables that the
    // table builders below free and reallocate: drop them whenever the strategy is set
    step_drop_graphs(F);
    if (strategy == EBBX_STRAT_AUTO) strategy = EBBX_STRAT_BLOCK;
    if (strategy == EBBX_STRAT_OWNER) {
        int32_t vb = block ? block : (F->prec == EBBX_F32 ? 128 : 64);
        if (F->own_vb != vb) build_owner(F, vb, s);
        // default size: fall back to 64 owned vertices when the T-product's LDS
        // (staged d, a and w, and the owned rows) would exceed what a workgroup may hold
        const size_t tmul_lds = (size_t)9 * F->own_maxv * sizeof(double) + (size_t)3 * F->own_maxinc * F->esize;
        int dev = 0, lim = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (!block && vb > 64 && tmul_lds > (size_t)std::max(lim, 64 * 1024)) {
            vb = 64;
            build_owner(F, vb, s);
        }
        F->strategy = strategy;
        F->block = vb;
        return;
    }
    if (strategy == EBBX_STRAT_PIPE) {
        const int32_t g = block ? block : 6;
        if (F->halo_level != g) build_pipe(F, g, s);
        F->strategy = strategy;
        F->block = g;
        return;
    }
    if (strategy == EBBX_STRAT_BLOCK || strategy == EBBX_STRAT_BLOCK_LDS || strategy == EBBX_STRAT_LANES) {
        const bool two = (block & EBBX_BLOCK_TPT2) != 0;
        const int32_t bt = (block & ~EBBX_BLOCK_TPT2) ? (block & ~EBBX_BLOCK_TPT2) : 256;
        if (bt > 1024) fail(EBBX_E_ARG, "block strategies take at most 1024 tets per block");
        if (strategy == EBBX_STRAT_LANES && (bt > 256 || two))
            fail(EBBX_E_ARG, "the multi-lane product takes at most 256 tets per block (four lanes each)");
        if (two && bt < 128) fail(EBBX_E_ARG, "two tets per thread need blocks of at least 128 tets");
        if ((two || bt > 512) && bt % 128)
            fail(EBBX_E_ARG, "two tets per thread need a multiple of 128 tets per block (got %d)", bt);
        if (!F->blocks_built || F->blk_tets != bt || F->halo_level != 0) build_blocks(F, bt, s);
        F->strategy = strategy;
        F->blk_red = strategy == EBBX_STRAT_BLOCK_LDS ? 1 : 0;
        F->blk_tpt = (two || bt > 512) ? 2 : 1;
        F->block = two ? (bt | EBBX_BLOCK_TPT2) : bt;
        return;
    }
    if (block != 0 && (block < 64 || block > 256 || block % 64))
        fail(EBBX_E_ARG, "block %d must be a multiple of 64 in [64, 256]", block);
    if (strategy == EBBX_STRAT_SEG && !F->part.get())
        F->part.reset((size_t)std::max<int64_t>(F->nt, 1) * 12 * F->esize, s);
    F->strategy = strategy;
    F->block = block ? block : 256;
}

std::unique_ptr<ebbx_fem_s> fem_build(ebbx_relation_s *tr, const char *keyfield, ebbx_relation_s *vr,
                                      const char *pos_field, const char *pinned_field, const ebbx_fem_params &prm,
                                      const double *E_tet) {
    const ebbx_fem_params *params = &prm;
    KeyField &kf = get_key(tr, keyfield);
    if (kf.target != vr) fail(EBBX_E_ARG, "key-field '%s' does not target '%s'", keyfield, vr->name.c_str());
    if (kf.arity != 4) fail(EBBX_E_SHAPE, "key-field '%s' has arity %d, tets need 4", keyfield, kf.arity);
    const Field &X = get_field(vr, pos_field, EBBX_F64, 3);
    const uint8_t *pin = nullptr;
    if (pinned_field) pin = (const uint8_t *)get_field(vr, pinned_field, EBBX_U8, 1).ptr;
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
    F->mesh_vptr = {0, F->nv};
    F->status.reset(sizeof(unsigned long long) * 4, s);
    F->scratch.reset((size_t)std::max<int64_t>(3 * nv, 4096) * sizeof(double), s);
    HIPCHK(hipMemsetAsync(F->status.get(), 0, sizeof(unsigned long long) * 4, s));
    if (pin) HIPCHK(hipMemcpyAsync(F->pinned.get(), pin, (size_t)F->nv, hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemsetAsync(F->pinned.get(), 0, (size_t)nv, s));
    const int64_t nbad = elem_precompute(F.get(), (const double *)X.ptr, E_tet, s);
    F->Xc.reset((size_t)std::max<int64_t>(3 * vr->size, 1) * sizeof(double), s);
    if (vr->size > 0)
        HIPCHK(hipMemcpy(F->Xc.get(), X.ptr, (size_t)(3 * vr->size) * sizeof(double), hipMemcpyDeviceToDevice));
    if (nbad > 0) fail(EBBX_E_DEGENERATE, "%lld rest tets have V0 <= 0", (long long)nbad);
    set_strategy(F.get(), params->strategy, params->block, s);
    HIPCHK(hipStreamSynchronize(s));
    return F;
}

}  // namespace ebbx

using namespace ebbx;

extern "C" {

ebbx_status ebbx_fem_create(ebbx_relation tets, const char *keyfield, ebbx_relation verts, const char *pos_field,
                            const char *pinned_field, const ebbx_fem_params *params, ebbx_fem *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = nullptr;
    if (!params) fail(EBBX_E_ARG, "params is NULL");
    auto *tr = check_rel(tets);
    auto *vr = check_rel(verts);
    const double *E_tet = nullptr;
    if (params->E_field) E_tet = (const double *)get_field(tr, params->E_field, EBBX_F64, 1).ptr;
    auto F = fem_build(tr, keyfield, vr, pos_field, pinned_field, *params, E_tet);
    fem_register(F.get());
    *out = F.release();
    EBBX_API_END
}

ebbx_status ebbx_fem_destroy(ebbx_fem fem) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (F->batch_owned) fail(EBBX_E_STATE, "this FEM domain belongs to a batch; destroy the batch");
    HIPCHK(hipDeviceSynchronize());
    fem_unregister(F);
    delete F;
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
        hipLaunchKernelGGL(k_diag_finish, dim3(grid_for(3 * F->nv)), dim3(VT), 0, s, diag, F->mass.as<double>(), F->nv, dt);
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
    std::vector<unsigned long long> h((size_t)F->nm);
    HIPCHK(hipMemcpyAsync(h.data(), F->status.get(), h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (reset) {
        HIPCHK(hipMemsetAsync(F->status.get(), 0, h.size() * sizeof(unsigned long long), s));
        HIPCHK(hipStreamSynchronize(s));
    }
    unsigned long long tot = 0;
    for (auto x : h) tot += x;
    if (n_inverted) *n_inverted = (int64_t)tot;
    EBBX_API_END
}

}  // extern "C"

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
    elem_egrad(F, d, v, w, dt, dt * dt, E_bar, (hipStream_t)stream);
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_forces_vjp(ebbx_fem fem, const double *d, const double *w, double *d_bar,
                                           double *E_bar, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !w) && F->nv > 0) fail(EBBX_E_ARG, "d or w is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (d_bar && F->nv > 0 && (overlap(d_bar, d, bytes) || overlap(d_bar, w, bytes)))
        fail(EBBX_E_PHASE, "d_bar aliases d or w");
    hipStream_t s = (hipStream_t)stream;
    if (d_bar) elem_launch(F, OP_KMUL, d, w, d_bar, 1, s);          // (df/dd)^T w = K w (K symmetric)
    if (E_bar) elem_egrad(F, d, nullptr, w, 1.0, 0.0, E_bar, s);    // w_t . f_t / E_t
    EBBX_API_END
}

extern "C" ebbx_status ebbx_fem_Kmul_vjp(ebbx_fem fem, const double *d, const double *u, const double *w,
                                         double *d_bar, double *u_bar, double *E_bar, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !u || !w) && F->nv > 0) fail(EBBX_E_ARG, "d, u or w is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0)
        for (const void *o : {(const void *)d_bar, (const void *)u_bar})
            if (o && (overlap(o, d, bytes) || overlap(o, u, bytes) || overlap(o, w, bytes)))
                fail(EBBX_E_PHASE, "an output aliases d, u or w");
    if (d_bar && u_bar && F->nv > 0 && overlap(d_bar, u_bar, bytes)) fail(EBBX_E_PHASE, "d_bar aliases u_bar");
    hipStream_t s = (hipStream_t)stream;
    if (d_bar) elem_launch(F, OP_TMUL, d, u, d_bar, 1, s, nullptr, w);   // grad_d (w . K(d) u) = T[u, w]
    if (u_bar) elem_launch(F, OP_KMUL, d, w, u_bar, 1, s);               // K^T w = K w
    if (E_bar) elem_egrad(F, d, u, w, 0.0, 1.0, E_bar, s);                // w_t . K_t u / E_t
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
    if (!had) step_drop_graphs(F);
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
