// tune.hip -- the autotuner of the element maps.
//
// The paper reports that the solver kernels of its GPU runtime are sensitive
// to the block size (up to 2x; Performance Evaluation, Vega) and that the
// per-element matrix work is register-heavy (Discussion).  Here the choice
// between scatter strategies, their block sizes and tets per thread is made
// by timing the stiffness product, the call a CG iteration spends most of its
// time in, on the domain itself.  Choices are cached in a small JSON file keyed by the
// device, the element model and precision, the sizes and a fingerprint of
// the tets' keys (locality decides between strategies).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fem.h"

using namespace ebbx;

namespace {

struct Candidate {
    int32_t strategy, block;
};

const Candidate kCandidates[] = {
    {EBBX_STRAT_BLOCK, 128},     {EBBX_STRAT_BLOCK, 256},     {EBBX_STRAT_BLOCK, 512},
    {EBBX_STRAT_BLOCK_LDS, 128}, {EBBX_STRAT_BLOCK_LDS, 256}, {EBBX_STRAT_BLOCK_LDS, 512},
    {EBBX_STRAT_SEG, 128},       {EBBX_STRAT_SEG, 256},       {EBBX_STRAT_ATOMIC, 128},
    {EBBX_STRAT_ATOMIC, 256},    {EBBX_STRAT_BLOCK, 64},      {EBBX_STRAT_OWNER, 64},
    {EBBX_STRAT_OWNER, 128},     {EBBX_STRAT_OWNER, 256},     {EBBX_STRAT_PIPE, 2},
    {EBBX_STRAT_PIPE, 4},        {EBBX_STRAT_PIPE, 6},        {EBBX_STRAT_PIPE, 8},
    {EBBX_STRAT_LANES, 64},      {EBBX_STRAT_LANES, 128},     {EBBX_STRAT_LANES, 256},
    // two tets per thread
    {EBBX_STRAT_BLOCK, 128 | EBBX_BLOCK_TPT2}, {EBBX_STRAT_BLOCK, 256 | EBBX_BLOCK_TPT2},
    {EBBX_STRAT_BLOCK, 512 | EBBX_BLOCK_TPT2},
};

uint64_t fnv1a(const void *p, size_t n, uint64_t h) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// device | model | precision | material | sizes | fingerprint of up to 64Ki sampled keys
std::string cache_key(ebbx_fem_s *F, hipStream_t s) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    const int64_t n4 = 4 * F->nt;
    const int64_t ns = std::min<int64_t>(n4, 65536);
    std::vector<int32_t> sample((size_t)ns);
    const int64_t stride = ns > 0 ? std::max<int64_t>(1, n4 / ns) : 1;
    if (ns > 0) {
        // strided copy of the key columns (contiguous 4*nt int32)
        HIPCHK(hipMemcpy2DAsync(sample.data(), sizeof(int32_t), F->keys, stride * sizeof(int32_t), sizeof(int32_t),
                                (size_t)ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const uint64_t h = fnv1a(sample.data(), sample.size() * sizeof(int32_t), 1469598103934665603ull);
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s/%dcu|m%d|p%d|e%d|nt%lld|nv%lld|nm%lld|k%016llx", prop.gcnArchName,
                  prop.multiProcessorCount, F->model, F->prec, F->per_tet ? 1 : 0, (long long)F->nt, (long long)F->nv,
                  (long long)F->nm, (unsigned long long)h);
    for (char *c = buf; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    return buf;
}

struct CacheEntry {
    std::string key;
    int32_t strategy = 0, block = 0;
    double us = 0.0;
};

// One entry per line:  "key": {"strategy": S, "block": B, "us": T},
std::vector<CacheEntry> cache_read(const char *path) {
    std::vector<CacheEntry> out;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        CacheEntry e;
        e.key = line.substr(q0 + 1, q1 - q0 - 1);
        if (std::sscanf(line.c_str() + q1 + 1, ": {\"strategy\": %d, \"block\": %d, \"us\": %lf", &e.strategy, &e.block,
                        &e.us) == 3)
            out.push_back(e);
    }
    return out;
}

void cache_write(const char *path, const std::vector<CacheEntry> &entries) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) fail(EBBX_E_ARG, "cannot write the tuning cache '%s'", path);
        o << "{\n";
        for (size_t i = 0; i < entries.size(); ++i) {
            char buf[96];
            std::snprintf(buf, sizeof buf, "{\"strategy\": %d, \"block\": %d, \"us\": %.3f}", entries[i].strategy,
                          entries[i].block, entries[i].us);
            o << "\"" << entries[i].key << "\": " << buf << (i + 1 < entries.size() ? ",\n" : "\n");
        }
        o << "}\n";
        if (!o) fail(EBBX_E_ARG, "cannot write the tuning cache '%s'", path);
    }
    if (std::rename(tmp.c_str(), path) != 0) fail(EBBX_E_ARG, "cannot replace the tuning cache '%s'", path);
}

}  // namespace

extern "C" ebbx_status ebbx_fem_autotune(ebbx_fem fem, const double *d, const double *u, const char *cache_path,
                                         ebbx_tune_entry *results, int32_t cap, int32_t *n_results,
                                         ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if (n_results) *n_results = 0;
    if (cap < 0 || (cap > 0 && !results)) fail(EBBX_E_ARG, "results capacity without a results array");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipDeviceSynchronize());
    const std::string key = cache_key(F, s);
    std::vector<CacheEntry> cache;
    if (cache_path) {
        cache = cache_read(cache_path);
        for (const auto &e : cache)
            if (e.key == key) {
                set_strategy(F, e.strategy, e.block, s);
                HIPCHK(hipStreamSynchronize(s));
                return EBBX_OK;
            }
    }
    const int64_t nv = F->nv, n3 = 3 * std::max<int64_t>(nv, 1);
    DevBuf tmp((size_t)n3 * 3 * sizeof(double), s);
    double *dd = tmp.as<double>(), *uu = dd + n3, *yy = uu + n3;
    if (d) HIPCHK(hipMemcpyAsync(dd, d, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemsetAsync(dd, 0, (size_t)n3 * sizeof(double), s));
    if (u) HIPCHK(hipMemcpyAsync(uu, u, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    else fill_f64(uu, n3, 1.0, s);
    const int32_t keep_s = F->strategy, keep_b = F->block;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<ebbx_tune_entry> timed;
    try {
        for (const Candidate &c : kCandidates) {
            try {
                set_strategy(F, c.strategy, c.block, s);
            } catch (const Error &) {
                continue;   // e.g. blocks too large for LDS on this mesh
            }
            auto run = [&]() { elem_launch(F, OP_KMUL, dd, uu, yy, 0, s); };
            try {
                run();
                run();
            } catch (const Error &) {
                continue;
            }
            const int reps = 5;
            HIPCHK(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run();
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            timed.push_back(ebbx_tune_entry{c.strategy, c.block, 1e3 * (double)ms / reps});
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        set_strategy(F, keep_s, keep_b, s);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (timed.empty()) {
        set_strategy(F, keep_s, keep_b, s);
        fail(EBBX_E_STATE, "no strategy could run on this domain");
    }
    const auto best = *std::min_element(timed.begin(), timed.end(), [](const ebbx_tune_entry &a,
                                                                          const ebbx_tune_entry &b) { return a.us < b.us; });
    set_strategy(F, best.strategy, best.block, s);
    HIPCHK(hipStreamSynchronize(s));
    if (cache_path) {
        cache.push_back(CacheEntry{key, best.strategy, best.block, best.us});
        cache_write(cache_path, cache);
    }
    const int32_t n = std::min<int32_t>(cap, (int32_t)timed.size());
    for (int32_t i = 0; i < n; ++i) results[i] = timed[(size_t)i];
    if (n_results) *n_results = (int32_t)timed.size();
    EBBX_API_END
}
