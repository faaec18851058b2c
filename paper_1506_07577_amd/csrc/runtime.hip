// runtime.hip -- relations, fields, key-fields, grouping and reordering.
//
// The relational layer of Ebb's runtime (Runtime Implementation, "Data Layout
// and Management" and "Relational Primitives Implementations"): column-store
// fields, key-fields checked to stay in range, grouping by a key-field into a
// CSR-style inverted index, and a locality reorder that the opaque-key model
// permits.  All device work here is one-time setup; the hot element map lives
// in fem.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>

#include "internal.h"

namespace ebbx {

// ---- errors ----------------------------------------------------------------

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(ebbx_status code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, std::string(buf)};
}

size_t dtype_size(ebbx_dtype t) {
    switch (t) {
        case EBBX_F32: return 4;
        case EBBX_F64: return 8;
        case EBBX_I32: return 4;
        case EBBX_U8: return 1;
        case EBBX_I64: return 8;
    }
    fail(EBBX_E_DTYPE, "unknown dtype %d", (int)t);
}

int current_device() {
    int d = 0;
    HIPCHK(hipGetDevice(&d));
    return d;
}

// ---- allocator -----------------------------------------------------------------

static std::mutex g_alloc_mu;
static Allocator g_alloc;

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void DevBuf::reset(size_t bytes, hipStream_t s) {
    release();
    if (bytes == 0) return;
    a_ = current_allocator();
    void *p = nullptr;
    if (a_.alloc) {
        p = a_.alloc(bytes, a_.ctx, (ebbx_stream)s);
        if (!p) fail(EBBX_E_OOM, "allocator hook returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess || !p) fail(EBBX_E_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    p_ = p;
    bytes_ = bytes;
}

void DevBuf::release() {
    if (!p_) return;
    if (a_.alloc) {
        if (a_.free_fn) a_.free_fn(p_, a_.ctx);
    } else {
        (void)hipFree(p_);
    }
    p_ = nullptr;
    bytes_ = 0;
}

// ---- registry of live relations (for key remapping on reorder) -----------------

static std::mutex g_rel_mu;
static std::set<ebbx_relation_s *> g_rels;

ebbx_relation_s *check_rel(ebbx_relation r) {
    std::lock_guard<std::mutex> lk(g_rel_mu);
    if (!r || !g_rels.count(r)) fail(EBBX_E_ARG, "invalid relation handle");
    return r;
}

const Field &get_field(ebbx_relation_s *r, const char *name, ebbx_dtype dt, int32_t ncomp) {
    if (!name) fail(EBBX_E_ARG, "field name is NULL");
    auto it = r->fields.find(name);
    if (it == r->fields.end())
        fail(EBBX_E_NOT_FOUND, "relation '%s' has no field '%s'", r->name.c_str(), name);
    if (it->second.dtype != dt)
        fail(EBBX_E_DTYPE, "field '%s.%s' has dtype %d, expected %d", r->name.c_str(), name,
             (int)it->second.dtype, (int)dt);
    if (ncomp > 0 && it->second.ncomp != ncomp)
        fail(EBBX_E_SHAPE, "field '%s.%s' has %d components, expected %d", r->name.c_str(), name,
             it->second.ncomp, ncomp);
    return it->second;
}

KeyField &get_key(ebbx_relation_s *r, const char *name) {
    if (!name) fail(EBBX_E_ARG, "key-field name is NULL");
    auto it = r->keys.find(name);
    if (it == r->keys.end())
        fail(EBBX_E_NOT_FOUND, "relation '%s' has no key-field '%s'", r->name.c_str(), name);
    return it->second;
}

// ---- device primitives -------------------------------------------------------------

static inline unsigned grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

__device__ __forceinline__ long long wave_incl_scan(long long x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

constexpr int SCAN_T = 256;
constexpr int SCAN_I = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

// Exclusive scan of one 1024-entry tile per block; tile totals to sums[].
__global__ __launch_bounds__(SCAN_T) void k_scan_tile(int64_t *data, int64_t n, int64_t *sums) {
    __shared__ long long s_w[SCAN_T / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_I;
    long long v[SCAN_I];
    long long tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        v[i] = (base + i < n) ? data[base + i] : 0;
        tot += v[i];
    }
    long long incl = wave_incl_scan(tot, lane);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    long long wave_off = 0;
    for (int w = 0; w < wave; ++w) wave_off += s_w[w];
    long long run = wave_off + incl - tot;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
    if (tid == SCAN_T - 1) sums[blockIdx.x] = wave_off + incl;
}

__global__ void k_scan_add(int64_t *data, int64_t n, const int64_t *offs) {
    const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    const int64_t add = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t j = i + (int64_t)k * SCAN_T;
        if (j < n) data[j] += add;
    }
}

void exclusive_scan_i64(int64_t *data, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    DevBuf sums((size_t)nb * sizeof(int64_t), s);
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(SCAN_T), 0, s, data, n, sums.as<int64_t>());
    HIPCHK(hipGetLastError());
    if (nb > 1) {
        exclusive_scan_i64(sums.as<int64_t>(), nb, s);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_T), 0, s, data, n, sums.as<int64_t>());
        HIPCHK(hipGetLastError());
    }
    // keep `sums` alive until the kernels that read it have run
    HIPCHK(hipStreamSynchronize(s));
}

// Stable LSD radix sort, 8-bit digits.  Per pass: per-tile digit histograms
// (digit-major), one exclusive scan, then a stable scatter in which every
// wave ranks its 64 keys with ballots (lanes holding the same digit are
// found bit by bit) and waves and rounds are combined in order.
constexpr int RS_T = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_T * RS_ROUNDS;

template <class K>
__global__ __launch_bounds__(RS_T) void k_rs_hist(const K *keys, int64_t n, int shift, int64_t ntiles,
                                                  int64_t *hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + (int64_t)r * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 255)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const K *kin, const uint32_t *vin, K *kout,
                                                     uint32_t *vout, int64_t n, int shift,
                                                     int64_t ntiles, const int64_t *offs) {
    __shared__ int s_base[256];
    __shared__ int s_wcnt[RS_T / 64][256];
    __shared__ long long s_goff[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_base[tid] = 0;
    s_goff[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
        for (int w = 0; w < RS_T / 64; ++w) s_wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = tile0 + (int64_t)r * RS_T + tid;
        const bool valid = i < n;
        K key = valid ? kin[i] : (K)0;
        uint32_t val = valid ? vin[i] : 0u;
        const int dig = (int)((key >> shift) & 255);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (dig >> b) & 1;
            unsigned long long bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) s_wcnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int off = s_base[dig] + rank;
            for (int w = 0; w < wave; ++w) off += s_wcnt[w][dig];
            const int64_t dst = s_goff[dig] + off;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int w = 0; w < RS_T / 64; ++w) add += s_wcnt[w][tid];
        s_base[tid] += add;
    }
}

template <class K>
static void radix_sort_pairs(K *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    DevBuf kb((size_t)n * sizeof(K), s), vb((size_t)n * sizeof(uint32_t), s);
    DevBuf hist((size_t)(256 * ntiles) * sizeof(int64_t), s);
    K *ka = keys, *kx = kb.as<K>();
    uint32_t *va = vals, *vx = vb.as<uint32_t>();
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)ntiles), dim3(RS_T), 0, s, ka, n, shift, ntiles,
                           hist.as<int64_t>());
        HIPCHK(hipGetLastError());
        exclusive_scan_i64(hist.as<int64_t>(), 256 * ntiles, s);
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)ntiles), dim3(RS_T), 0, s, ka, va, kx, vx, n,
                           shift, ntiles, hist.as<int64_t>());
        HIPCHK(hipGetLastError());
        std::swap(ka, kx);
        std::swap(va, vx);
    }
    if (ka != keys) {
        HIPCHK(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
}

void radix_sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s) {
    radix_sort_pairs<uint32_t>(keys, vals, n, bits, s);
}
void radix_sort_pairs_u64(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s) {
    radix_sort_pairs<uint64_t>(keys, vals, n, bits, s);
}

static int bits_for(int64_t n) {   // bits needed for values in [0, n)
    int b = 0;
    while (b < 63 && (int64_t(1) << b) < n) ++b;
    return b < 1 ? 1 : b;
}

// ---- key validation ---------------------------------------------------------------------

__global__ void k_key_range(const int32_t *keys, int64_t n, int64_t nmax, unsigned int *bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t k = keys[i];
        if (k < 0 || (int64_t)k >= nmax) atomicOr(bad, 1u);
    }
}

// ---- grouping -------------------------------------------------------------------------

__global__ void k_group_count(const int32_t *keys, int64_t n, int arity, unsigned long long *cnt) {
    const int64_t total = n * arity;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[keys[i]], 1ull);
}

// pairs in incidence order e = arity*row + slot; the key-field is column-stored
__global__ void k_group_pairs(const int32_t *keys, int64_t n, int arity, uint32_t *k_out,
                              uint32_t *v_out) {
    const int64_t total = n * arity;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t row = e / arity;
        int slot = (int)(e - row * arity);
        k_out[e] = (uint32_t)keys[(int64_t)slot * n + row];
        v_out[e] = (uint32_t)e;
    }
}

std::shared_ptr<Grouping> build_group(ebbx_relation_s *rel, const char *name, hipStream_t s) {
    KeyField &kf = get_key(rel, name);
    if (kf.group) return kf.group;
    const int64_t n = rel->size, nt_target = kf.target->size;
    const int64_t total = n * kf.arity;
    if (total >= (int64_t(1) << 31)) fail(EBBX_E_ARG, "grouping of %lld incidences exceeds int32", (long long)total);
    auto g = std::make_shared<Grouping>();
    g->n_target = nt_target;
    g->arity = kf.arity;
    g->row_ptr.reset((size_t)(nt_target + 1) * sizeof(int64_t), s);
    g->inc.reset((size_t)std::max<int64_t>(total, 1) * sizeof(int32_t), s);
    int64_t *rp = g->row_ptr.as<int64_t>();
    HIPCHK(hipMemsetAsync(rp, 0, (size_t)(nt_target + 1) * sizeof(int64_t), s));
    if (total > 0) {
        hipLaunchKernelGGL(k_group_count, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, kf.ptr, n,
                           kf.arity, (unsigned long long *)rp);
        HIPCHK(hipGetLastError());
    }
    exclusive_scan_i64(rp, nt_target + 1, s);
    if (total > 0) {
        DevBuf keys((size_t)total * sizeof(uint32_t), s);
        hipLaunchKernelGGL(k_group_pairs, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, kf.ptr, n,
                           kf.arity, keys.as<uint32_t>(), g->inc.as<uint32_t>());
        HIPCHK(hipGetLastError());
        radix_sort_pairs_u32(keys.as<uint32_t>(), g->inc.as<uint32_t>(), total, bits_for(nt_target), s);
    }
    HIPCHK(hipStreamSynchronize(s));
    kf.group = g;
    return g;
}

// ---- Morton order ----------------------------------------------------------------------

__global__ void k_bbox(const double *X, int64_t nv, double *part) {
    __shared__ double s[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            double x = X[(int64_t)a * nv + i];
            lo[a] = fmin(lo[a], x);
            hi[a] = fmax(hi[a], x);
        }
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) part[6 * blockIdx.x + a] = s[a][0];
}

__device__ __forceinline__ uint64_t spread3(uint64_t x) {   // bit b -> bit 3b
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

struct MortonFrame {
    double lo[3], sc[3];
};

__global__ void k_morton_codes(const double *X, int64_t nv, MortonFrame fr, uint64_t *codes,
                               uint32_t *ids) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t code = 0;
        for (int a = 0; a < 3; ++a) {
            // one rounded subtract and one rounded multiply, never fused
            double s = __dmul_rn(__dsub_rn(X[(int64_t)a * nv + i], fr.lo[a]), fr.sc[a]);
            double fl = floor(s);
            uint64_t q = fl >= 2097151.0 ? 2097151ull : (uint64_t)fl;
            code |= spread3(q) << a;
        }
        codes[i] = code;
        ids[i] = (uint32_t)i;
    }
}

// out[i] = key[ids[i]]: the sort keys of a permutation's entries
__global__ void k_gather_key(const int32_t *key, const uint32_t *ids, int64_t n, uint32_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)key[ids[i]];
}

__global__ void k_invert(const uint32_t *perm, int64_t n, int32_t *inv) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        inv[perm[i]] = (int32_t)i;
}

__global__ void k_min_key(const int32_t *keys, int64_t n, int arity, const int32_t *inv, uint32_t *kout,
                          uint32_t *ids) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t m = inv[keys[t]];
        for (int c = 1; c < arity; ++c) m = min(m, inv[keys[(int64_t)c * n + t]]);
        kout[t] = (uint32_t)m;
        ids[t] = (uint32_t)t;
    }
}

// ---- reorder ---------------------------------------------------------------------------

template <class E>
__global__ void k_gather_rows(const E *src, E *dst, const int32_t *perm, int64_t n, int ncomp) {
    const int64_t total = n * ncomp;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = j / n, i = j - c * n;
        dst[j] = src[c * n + perm[i]];
    }
}

__global__ void k_remap_keys(int32_t *keys, int64_t total, const int32_t *inv) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * blockDim.x)
        keys[j] = inv[keys[j]];
}

__global__ void k_check_perm(const int32_t *perm, int64_t n, unsigned int *seen, unsigned int *bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = perm[i];
        if (p < 0 || p >= n) {
            atomicOr(bad, 1u);
        } else if (atomicOr(&seen[p], 1u) != 0u) {
            atomicOr(bad, 1u);
        }
    }
}

static void permute_column_block(void *ptr, size_t esize, int64_t n, int ncomp, const int32_t *perm,
                                 hipStream_t s) {
    const int64_t total = n * ncomp;
    DevBuf tmp((size_t)total * esize, s);
    const unsigned g = grid_for(total, 256, 65536);
    switch (esize) {
        case 1:
            hipLaunchKernelGGL(k_gather_rows<uint8_t>, dim3(g), dim3(256), 0, s, (const uint8_t *)ptr,
                               tmp.as<uint8_t>(), perm, n, ncomp);
            break;
        case 4:
            hipLaunchKernelGGL(k_gather_rows<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t *)ptr,
                               tmp.as<uint32_t>(), perm, n, ncomp);
            break;
        case 8:
            hipLaunchKernelGGL(k_gather_rows<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t *)ptr,
                               tmp.as<uint64_t>(), perm, n, ncomp);
            break;
        default: fail(EBBX_E_DTYPE, "unsupported element size %zu", esize);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ptr, tmp.get(), (size_t)total * esize, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace ebbx

using namespace ebbx;

// ---- C ABI ---------------------------------------------------------------------------------

extern "C" {

const char *ebbx_last_error(void) { return g_last_error.c_str(); }

int32_t ebbx_version(void) { return 100; }

ebbx_status ebbx_set_allocator(void *(*alloc)(size_t, void *, ebbx_stream), void (*free_fn)(void *, void *),
                               void *ctx) {
    EBBX_API_BEGIN
    if (alloc && !free_fn) fail(EBBX_E_ARG, "allocator hook needs a free function");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free_fn = alloc ? free_fn : nullptr;
    g_alloc.ctx = alloc ? ctx : nullptr;
    EBBX_API_END
}

ebbx_status ebbx_relation_create(const char *name, int64_t size, ebbx_relation *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = nullptr;
    if (size < 0 || size >= (int64_t(1) << 31)) fail(EBBX_E_ARG, "relation size %lld out of range", (long long)size);
    auto *r = new ebbx_relation_s();
    r->name = name ? name : "";
    r->size = size;
    {
        std::lock_guard<std::mutex> lk(g_rel_mu);
        g_rels.insert(r);
    }
    *out = r;
    EBBX_API_END
}

ebbx_status ebbx_relation_destroy(ebbx_relation rel) {
    EBBX_API_BEGIN
    check_rel(rel);
    std::lock_guard<std::mutex> lk(g_rel_mu);
    for (auto *o : g_rels)
        if (o != rel)
            for (auto &kv : o->keys)
                if (kv.second.target == rel)
                    fail(EBBX_E_STATE, "relation '%s' is the target of key-field '%s.%s'", rel->name.c_str(),
                         o->name.c_str(), kv.first.c_str());
    g_rels.erase(rel);
    delete rel;
    EBBX_API_END
}

ebbx_status ebbx_relation_size(ebbx_relation rel, int64_t *out) {
    EBBX_API_BEGIN
    if (!out) fail(EBBX_E_ARG, "out is NULL");
    *out = check_rel(rel)->size;
    EBBX_API_END
}

ebbx_status ebbx_field_bind(ebbx_relation rel, const char *name, ebbx_dtype dtype, int32_t ncomp, void *dev_ptr) {
    EBBX_API_BEGIN
    auto *r = check_rel(rel);
    if (!name || !*name) fail(EBBX_E_ARG, "field name is empty");
    if (ncomp < 1 || ncomp > 64) fail(EBBX_E_SHAPE, "ncomp %d out of range", ncomp);
    size_t es = dtype_size(dtype);
    if (!dev_ptr && r->size > 0) fail(EBBX_E_ARG, "field '%s' pointer is NULL", name);
    if ((uintptr_t)dev_ptr % es) fail(EBBX_E_LAYOUT, "field '%s' pointer is not %zu-byte aligned", name, es);
    if (r->keys.count(name)) fail(EBBX_E_ARG, "'%s' is already a key-field", name);
    r->fields[name] = Field{dtype, ncomp, dev_ptr};
    EBBX_API_END
}

ebbx_status ebbx_keyfield_bind(ebbx_relation rel, const char *name, ebbx_relation target, int32_t arity,
                               int32_t *dev_ptr) {
    EBBX_API_BEGIN
    auto *r = check_rel(rel);
    auto *tg = check_rel(target);
    if (!name || !*name) fail(EBBX_E_ARG, "key-field name is empty");
    if (arity < 1 || arity > 16) fail(EBBX_E_SHAPE, "arity %d out of range", arity);
    if (!dev_ptr && r->size > 0) fail(EBBX_E_ARG, "key-field '%s' pointer is NULL", name);
    if ((uintptr_t)dev_ptr % 4) fail(EBBX_E_LAYOUT, "key-field '%s' pointer is not 4-byte aligned", name);
    if (r->fields.count(name)) fail(EBBX_E_ARG, "'%s' is already a field", name);
    const int64_t total = r->size * arity;
    if (total > 0) {
        hipStream_t s = nullptr;
        DevBuf flag(sizeof(unsigned int), s);
        HIPCHK(hipMemsetAsync(flag.get(), 0, sizeof(unsigned int), s));
        hipLaunchKernelGGL(k_key_range, dim3(grid_for(total, 256, 8192)), dim3(256), 0, s, dev_ptr, total,
                           tg->size, flag.as<unsigned int>());
        HIPCHK(hipGetLastError());
        unsigned int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, flag.get(), sizeof bad, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad)
            fail(EBBX_E_KEY_RANGE, "key-field '%s.%s' holds a key outside [0, %lld)", r->name.c_str(), name,
                 (long long)tg->size);
    }
    r->keys[name] = KeyField{tg, arity, dev_ptr, nullptr};
    EBBX_API_END
}

ebbx_status ebbx_relation_group_by(ebbx_relation rel, const char *keyfield) {
    EBBX_API_BEGIN
    auto *r = check_rel(rel);
    build_group(r, keyfield, nullptr);
    EBBX_API_END
}

ebbx_status ebbx_group_export(ebbx_relation rel, const char *keyfield, int64_t *row_ptr_dev, int32_t *inc_dev) {
    EBBX_API_BEGIN
    auto *r = check_rel(rel);
    KeyField &kf = get_key(r, keyfield);
    if (!kf.group) fail(EBBX_E_NOT_GROUPED, "'%s' is not grouped by '%s'", r->name.c_str(), keyfield);
    const Grouping &g = *kf.group;
    if (row_ptr_dev)
        HIPCHK(hipMemcpy(row_ptr_dev, g.row_ptr.get(), (size_t)(g.n_target + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToDevice));
    if (inc_dev && r->size > 0)
        HIPCHK(hipMemcpy(inc_dev, g.inc.get(), (size_t)(r->size * g.arity) * sizeof(int32_t),
                         hipMemcpyDeviceToDevice));
    EBBX_API_END
}

ebbx_status ebbx_morton_order(ebbx_relation verts, const char *pos_field, const char *seg_keyfield,
                              ebbx_relation rel, const char *keyfield, uint64_t *codes_dev, int32_t *vperm_dev,
                              int32_t *tperm_dev) {
    EBBX_API_BEGIN
    auto *vr = check_rel(verts);
    auto *tr = check_rel(rel);
    const Field &X = get_field(vr, pos_field, EBBX_F64, 3);
    KeyField &kf = get_key(tr, keyfield);
    if (kf.target != vr) fail(EBBX_E_ARG, "key-field '%s' does not target '%s'", keyfield, vr->name.c_str());
    const KeyField *seg = nullptr;
    if (seg_keyfield) {
        seg = &get_key(vr, seg_keyfield);
        if (seg->arity != 1) fail(EBBX_E_SHAPE, "segment key-field '%s' must have arity 1", seg_keyfield);
    }
    const int64_t nv = vr->size, nt = tr->size;
    hipStream_t s = nullptr;
    // bounding box
    MortonFrame fr;
    for (int a = 0; a < 3; ++a) { fr.lo[a] = 0.0; fr.sc[a] = 0.0; }
    if (nv > 0) {
        const unsigned nb = grid_for(nv, 256, 1024);
        DevBuf part((size_t)nb * 6 * sizeof(double), s);
        hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, (const double *)X.ptr, nv, part.as<double>());
        HIPCHK(hipGetLastError());
        std::vector<double> h((size_t)nb * 6);
        HIPCHK(hipMemcpy(h.data(), part.get(), h.size() * sizeof(double), hipMemcpyDeviceToHost));
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (unsigned b = 0; b < nb; ++b)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], h[6 * b + a]);
                hi[a] = std::max(hi[a], h[6 * b + 3 + a]);
            }
        for (int a = 0; a < 3; ++a) {
            fr.lo[a] = lo[a];
            fr.sc[a] = hi[a] > lo[a] ? 2097152.0 / (hi[a] - lo[a]) : 0.0;
        }
    }
    DevBuf codes((size_t)std::max<int64_t>(nv, 1) * sizeof(uint64_t), s);
    DevBuf vids((size_t)std::max<int64_t>(nv, 1) * sizeof(uint32_t), s);
    if (nv > 0) {
        hipLaunchKernelGGL(k_morton_codes, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, s, (const double *)X.ptr,
                           nv, fr, codes.as<uint64_t>(), vids.as<uint32_t>());
        HIPCHK(hipGetLastError());
        if (codes_dev)
            HIPCHK(hipMemcpyAsync(codes_dev, codes.get(), (size_t)nv * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        radix_sort_pairs_u64(codes.as<uint64_t>(), vids.as<uint32_t>(), nv, 63, s);
        if (seg) {   // then a stable sort by segment: (segment, code, id)
            DevBuf sk((size_t)nv * sizeof(uint32_t), s);
            hipLaunchKernelGGL(k_gather_key, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, s, seg->ptr,
                               vids.as<uint32_t>(), nv, sk.as<uint32_t>());
            HIPCHK(hipGetLastError());
            radix_sort_pairs_u32(sk.as<uint32_t>(), vids.as<uint32_t>(), nv, bits_for(seg->target->size), s);
        }
    }
    if (vperm_dev && nv > 0)
        HIPCHK(hipMemcpyAsync(vperm_dev, vids.get(), (size_t)nv * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (tperm_dev && nt > 0) {
        DevBuf inv((size_t)std::max<int64_t>(nv, 1) * sizeof(int32_t), s);
        hipLaunchKernelGGL(k_invert, dim3(grid_for(nv, 256, 16384)), dim3(256), 0, s, vids.as<uint32_t>(), nv,
                           inv.as<int32_t>());
        HIPCHK(hipGetLastError());
        DevBuf tk((size_t)nt * sizeof(uint32_t), s), tid((size_t)nt * sizeof(uint32_t), s);
        hipLaunchKernelGGL(k_min_key, dim3(grid_for(nt, 256, 16384)), dim3(256), 0, s, kf.ptr, nt, kf.arity,
                           inv.as<int32_t>(), tk.as<uint32_t>(), tid.as<uint32_t>());
        HIPCHK(hipGetLastError());
        radix_sort_pairs_u32(tk.as<uint32_t>(), tid.as<uint32_t>(), nt, bits_for(nv), s);
        HIPCHK(hipMemcpyAsync(tperm_dev, tid.get(), (size_t)nt * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    EBBX_API_END
}

ebbx_status ebbx_relation_reorder(ebbx_relation rel, const int32_t *new_to_old_dev) {
    EBBX_API_BEGIN
    auto *r = check_rel(rel);
    const int64_t n = r->size;
    if (n == 0) return EBBX_OK;
    if (!new_to_old_dev) fail(EBBX_E_ARG, "permutation is NULL");
    // a domain built over r keeps per-row copies (B, mass, tables, row-ordered edges) in
    // r's present order: refuse rather than leave it silently inconsistent
    for (const char *user : {fem_relation_user(r), batch_relation_user(r), springs_relation_user(r)})
        if (user) fail(EBBX_E_STATE, "relation '%s' is in use by %s: destroy it before reordering", r->name.c_str(), user);
    hipStream_t s = nullptr;
    // validate: a permutation of [0, n)
    {
        DevBuf seen((size_t)n * sizeof(unsigned int), s), bad(sizeof(unsigned int), s);
        HIPCHK(hipMemsetAsync(seen.get(), 0, (size_t)n * sizeof(unsigned int), s));
        HIPCHK(hipMemsetAsync(bad.get(), 0, sizeof(unsigned int), s));
        hipLaunchKernelGGL(k_check_perm, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, new_to_old_dev, n,
                           seen.as<unsigned int>(), bad.as<unsigned int>());
        HIPCHK(hipGetLastError());
        unsigned int hb = 0;
        HIPCHK(hipMemcpy(&hb, bad.get(), sizeof hb, hipMemcpyDeviceToHost));
        if (hb) fail(EBBX_E_ARG, "reorder: not a permutation of [0, %lld)", (long long)n);
    }
    for (auto &kv : r->fields)
        permute_column_block(kv.second.ptr, dtype_size(kv.second.dtype), n, kv.second.ncomp, new_to_old_dev, s);
    for (auto &kv : r->keys) {
        permute_column_block(kv.second.ptr, 4, n, kv.second.arity, new_to_old_dev, s);
        kv.second.group.reset();
    }
    DevBuf inv((size_t)n * sizeof(int32_t), s);
    hipLaunchKernelGGL(k_invert, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, (const uint32_t *)new_to_old_dev,
                       n, inv.as<int32_t>());
    HIPCHK(hipGetLastError());
    std::lock_guard<std::mutex> lk(g_rel_mu);
    for (auto *o : g_rels)
        for (auto &kv : o->keys)
            if (kv.second.target == r) {
                const int64_t total = o->size * kv.second.arity;
                if (total > 0) {
                    hipLaunchKernelGGL(k_remap_keys, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, kv.second.ptr,
                                       total, inv.as<int32_t>());
                    HIPCHK(hipGetLastError());
                }
                kv.second.group.reset();
            }
    HIPCHK(hipStreamSynchronize(s));
    EBBX_API_END
}

}  // extern "C"
