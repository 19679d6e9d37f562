// Internal definitions shared by the HIP sources of libbfm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bfm.h"

namespace bfm {

// ---------------------------------------------------------------------------
// Errors: every internal failure throws bfm::Error; the C entry points catch
// it, store the message in a thread-local slot and return its code.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);

#define BFM_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::bfm::fail(BFM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BFM_CHECK(cond, code, msg)                  \
    do {                                            \
        if (!(cond)) ::bfm::fail((code), (msg));    \
    } while (0)

// Launch check: a bad configuration surfaces immediately, not at the next sync.
#define BFM_LAUNCHED() BFM_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Owning device buffer (hipMalloc'ed, grows on demand, never shrinks).
template <class T>
struct DevBuf {
    T *ptr = nullptr;
    size_t cap = 0;  // elements
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    T *ensure(size_t n) {
        if (n <= cap && ptr) return ptr;
        release();
        size_t bytes = sizeof(T) * (n ? n : 1);
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e != hipSuccess) {
            ptr = nullptr;
            fail(BFM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        cap = n ? n : 1;
        return ptr;
    }
    T *get() const { return ptr; }
    void swap(DevBuf &o) {
        std::swap(ptr, o.ptr);
        std::swap(cap, o.cap);
    }
};

// ---------------------------------------------------------------------------
// Expansion layout. Degrees n = 0..p-1; P = p^2 real coefficients per
// expansion, ordered by degree: slot n^2 holds the (real) order-0 value,
// slots n^2 + 2m - 1 and n^2 + 2m hold the real and imaginary parts of the
// order-m value for m = 1..n. Negative orders follow from the symmetry
// X_n^{-m} = (-1)^m conj(X_n^m) of every expansion used here.
constexpr int kMaxP = 20;
constexpr int kNumM2LOps = 316;  // offsets in [-3,3]^3 outside [-1,1]^3
constexpr double kInv4Pi = 0.079577471545947667884441881686257;

// Normalised solid harmonics (unit box scale). With
//   nu_n^m = sqrt((n-|m|)! (n+|m|)!),
//   Rt_n^m(v) = nu_n^m r^n P_n^m(cos t) e^{i m az} / (n+m)!    (regular)
//   It_n^m(v) = (n-m)! P_n^m(cos t) e^{i m az} / (nu_n^m r^{n+1})  (irregular)
// (P_n^m without the Condon-Shortley phase), the Laplace kernel expands as
//   1/|r - r'| = sum_{n,m} conj(Rt_n^m(r')) It_n^m(r),  |r'| < |r|,
// and both families obey three-term recurrences in Cartesian coordinates,
// evaluated here per order m (column) for n = m..p-1:
//   Rt_m^m = (x+iy) sqrt((2m-1)/(2m)) Rt_{m-1}^{m-1}
//   Rt_n^m = [(2n-1) z Rt_{n-1}^m - r^2 sqrt((n-m-1)(n+m-1)) Rt_{n-2}^m] / sqrt((n-m)(n+m))
//   It_m^m = (x+iy)/r^2 sqrt((2m-1)/(2m)) It_{m-1}^{m-1}
//   It_n^m = [(2n-1) z It_{n-1}^m - sqrt((n-m-1)(n+m-1)) It_{n-2}^m] / (r^2 sqrt((n-m)(n+m)))

}  // namespace bfm
