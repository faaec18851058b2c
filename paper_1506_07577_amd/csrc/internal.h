// internal.h -- host-side structures shared by the ebbx translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "ebbx.h"

namespace ebbx {

// Errors travel as C++ exceptions inside the library and become status codes
// at the C boundary (EBBX_API_BEGIN / EBBX_API_END).
struct Error {
    ebbx_status code;
    std::string msg;
};

[[noreturn]] void fail(ebbx_status code, const char *fmt, ...);
void set_last_error(const std::string &msg);

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::ebbx::fail(EBBX_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                          \
    } while (0)

#define EBBX_API_BEGIN try {
#define EBBX_API_END                                                                   \
    }                                                                                  \
    catch (const ::ebbx::Error &e) {                                                   \
        ::ebbx::set_last_error(e.msg);                                                 \
        return e.code;                                                                 \
    }                                                                                  \
    catch (const std::bad_alloc &) {                                                   \
        ::ebbx::set_last_error("host allocation failed");                              \
        return EBBX_E_OOM;                                                             \
    }                                                                                  \
    catch (...) {                                                                      \
        ::ebbx::set_last_error("unexpected internal error");                           \
        return EBBX_E_ARG;                                                             \
    }                                                                                  \
    return EBBX_OK;

// ---- device memory -----------------------------------------------------------

struct Allocator {
    void *(*alloc)(size_t, void *, ebbx_stream) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();

// An owned device buffer, released through the allocator it came from.
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(size_t bytes, hipStream_t s = nullptr) { reset(bytes, s); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p_ = o.p_; bytes_ = o.bytes_; a_ = o.a_;
            o.p_ = nullptr; o.bytes_ = 0;
        }
        return *this;
    }
    void reset(size_t bytes, hipStream_t s = nullptr);
    void release();
    void *get() const { return p_; }
    template <class T> T *as() const { return static_cast<T *>(p_); }
    size_t bytes() const { return bytes_; }

  private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
    Allocator a_;
};

// Ends a stream capture that an error left open, discarding the partial graph, so that the
// capture stream stays usable for the next call; disarm() once the capture has been ended
// the normal way.
class CaptureGuard {
  public:
    explicit CaptureGuard(hipStream_t s) : s_(s) {}
    ~CaptureGuard() {
        if (!s_) return;
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(s_, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
    }
    void disarm() { s_ = nullptr; }
    CaptureGuard(const CaptureGuard &) = delete;
    CaptureGuard &operator=(const CaptureGuard &) = delete;

  private:
    hipStream_t s_;
};

// ---- relational model ------------------------------------------------------

struct Field {
    ebbx_dtype dtype;
    int32_t ncomp;
    void *ptr;
};

struct Grouping {
    DevBuf row_ptr;   // int64 [size(target) + 1]
    DevBuf inc;       // int32 [arity * size(rel)], entry = arity*row + slot
    int64_t n_target = 0;
    int32_t arity = 0;
};

struct KeyField {
    ebbx_relation_s *target;
    int32_t arity;
    int32_t *ptr;
    std::shared_ptr<Grouping> group;   // built by ebbx_relation_group_by
};

size_t dtype_size(ebbx_dtype t);

}  // namespace ebbx

struct ebbx_relation_s {
    std::string name;
    int64_t size = 0;
    std::map<std::string, ebbx::Field> fields;
    std::map<std::string, ebbx::KeyField> keys;
};

namespace ebbx {

ebbx_relation_s *check_rel(ebbx_relation r);
const Field &get_field(ebbx_relation_s *r, const char *name, ebbx_dtype dt, int32_t ncomp);
KeyField &get_key(ebbx_relation_s *r, const char *name);

// Build (or return) the grouping of rel by key-field `name`; synchronous on `s`.
std::shared_ptr<Grouping> build_group(ebbx_relation_s *rel, const char *name, hipStream_t s);

// Device primitives of the runtime (runtime.hip).
void exclusive_scan_i64(int64_t *data, int64_t n, hipStream_t s);  // in place, n entries
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
void radix_sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s);
void radix_sort_pairs_u64(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t s);

int current_device();

// Whether a live domain holds per-row data of relation r in r's present order (a FEM
// domain over r as its tets or verts, a batch over r as its meshes, a springs domain
// over r as its edges or verts); those relations must not be reordered.  Each returns a
// description of the first such domain, or NULL.
const char *fem_relation_user(const ebbx_relation_s *r);
const char *batch_relation_user(const ebbx_relation_s *r);
const char *springs_relation_user(const ebbx_relation_s *r);

}  // namespace ebbx
