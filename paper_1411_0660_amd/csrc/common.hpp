// common.hpp -- shared host-side plumbing of libmbl: status handling, device
// buffers, timing.  No numerical method lives here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mbl.h"

namespace mbl {

// Error carried from the point of failure to the ABI boundary, where it is
// turned into a status code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define MBL_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            int code_ = (e_ == hipErrorOutOfMemory) ? MBL_ENOMEM : MBL_EDEVICE;\
            throw ::mbl::Error(code_, std::string(#call) + ": " +              \
                               hipGetErrorString(e_) + " at " + __FILE__ +     \
                               ":" + std::to_string(__LINE__));                \
        }                                                                      \
    } while (0)

#define MBL_CHECK_LAUNCH() MBL_HIP(hipGetLastError())

#define MBL_REQUIRE(cond, code, msg)                                           \
    do {                                                                       \
        if (!(cond)) throw ::mbl::Error((code), (msg));                        \
    } while (0)

// Device allocation accounting against the context budget.
struct Budget {
    size_t limit = 0, used = 0, peak = 0;
    // test hook: allocations fail once `armed` bytes have been allocated since
    // the hook was armed (0 = off)
    size_t armed = 0, since_armed = 0;
};

// Owning device buffer of bytes (typed views through ptr<T>()).
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { swap(o); }
    DevBuf &operator=(DevBuf &&o) noexcept { reset(); swap(o); return *this; }
    ~DevBuf() { reset(); }

    void alloc(size_t bytes, Budget *b) {
        reset();
        if (bytes == 0) return;
        if (b && b->limit && b->used + bytes > b->limit)
            throw Error(MBL_ENOMEM, "device budget exceeded: need " + std::to_string(bytes) +
                                        " B with " + std::to_string(b->used) + " of " +
                                        std::to_string(b->limit) + " B in use");
        if (b && b->armed) {
            if (b->since_armed + bytes > b->armed)
                throw Error(MBL_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                            " B refused by the fail_alloc_bytes test hook");
            b->since_armed += bytes;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            throw Error(MBL_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
        p_ = p; n_ = bytes; b_ = b;
        if (b) { b->used += bytes; if (b->used > b->peak) b->peak = b->used; }
    }
    // grow-only reallocation (contents not preserved)
    void ensure(size_t bytes, Budget *b) { if (bytes > n_) alloc(bytes, b); }
    void reset() {
        if (p_) {
            (void)hipFree(p_);
            if (b_) b_->used -= n_;
        }
        p_ = nullptr; n_ = 0; b_ = nullptr;
    }
    template <class T> T *ptr() const { return static_cast<T *>(p_); }
    size_t bytes() const { return n_; }

  private:
    void swap(DevBuf &o) { std::swap(p_, o.p_); std::swap(n_, o.n_); std::swap(b_, o.b_); }
    void *p_ = nullptr;
    size_t n_ = 0;
    Budget *b_ = nullptr;
};

// Page-locked host memory (hipHostMalloc), grow-only, for asynchronous
// device-to-host copies of small results.
class PinnedBuf {
  public:
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() { reset(); }
    void ensure(size_t bytes) {
        if (bytes <= n_) return;
        reset();
        void *p = nullptr;
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
        if (e != hipSuccess)
            throw Error(MBL_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        p_ = p;
        n_ = bytes;
    }
    void reset() {
        if (p_) (void)hipHostFree(p_);
        p_ = nullptr;
        n_ = 0;
    }
    template <class T> T *ptr() const { return static_cast<T *>(p_); }

  private:
    void *p_ = nullptr;
    size_t n_ = 0;
};

template <class T>
inline void h2d(T *dst, const T *src, size_t n, hipStream_t s) {
    if (n) MBL_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void d2h(T *dst, const T *src, size_t n, hipStream_t s) {
    if (n) MBL_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
}

double wall_seconds();
int debug_level();   // MBL_DEBUG environment variable (0 = quiet)

// Up spins of the sector: L / 2 (S^z = 0) for even L, (L + 1) / 2
// (S^z = +1/2) for odd L.
inline int sector_nup(int L) { return (L + 1) / 2; }

inline int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
    return r;
}

}  // namespace mbl
