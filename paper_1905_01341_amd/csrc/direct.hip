// Direct (all-pairs) off-diagonal product of the discrete single- and
// double-layer operators on device arrays, without a handle (Section 3.2,
// ns1 with eq2_13):
//   out_k = 1/(4 pi) sum_{j != i} s_j [ f x_j / |r_i - r_j|
//                                       + g y_j n_j . (r_i - r_j) / |r_i - r_j|^3 ],
//   i = rows[k] (or k when rows is null).
// The sources are split into nsplit ranges so that a small receiver set
// still fills the device: one wave per (64 receivers, source range) writes a
// partial sum per receiver, and a second kernel adds each receiver's partials
// in a fixed order (bitwise reproducible). The partial sums are the scratch
// buffer: bfm_direct_dev allocates it per call, stream-ordered;
// bfm_direct_dev_noalloc uses the file-scope device array `scratch` below.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "direct.h"

namespace bfm {

constexpr int kDirThreads = 64;
constexpr double kInv4PiD = 0.079577471545947667884441881686257;

// Scratch of the allocation-free entry point (kDirectScratch doubles,
// 32 MiB): every device the library runs on holds its own copy until the
// process ends, and every call on that device shares it.
__device__ __align__(256) double scratch[kDirectScratch];

__device__ inline double rsqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// part[sp * nr + k] = sum over sources [j0, j1) of split sp for receiver k
// (without the 1/(4 pi)); a receiver index outside [0, n) gives NaN.
template <bool MONO, bool DIP>
__global__ void __launch_bounds__(kDirThreads) k_direct_part(int64_t n, const double *__restrict__ xyz,
                                                             const double *__restrict__ s,
                                                             const double *__restrict__ nrm, double f,
                                                             const double *__restrict__ x, double g,
                                                             const double *__restrict__ y, int64_t nr,
                                                             const int64_t *__restrict__ rows, int nsplit,
                                                             double *__restrict__ part) {
    const int64_t k = (int64_t)blockIdx.x * kDirThreads + threadIdx.x;
    const int sp = blockIdx.y;
    const bool live = k < nr;
    const int64_t i = live ? (rows ? rows[k] : k) : -1;
    const bool ok = live && i >= 0 && i < n;
    // idle or invalid receivers sit far away; their sums are never stored
    const double rx = ok ? xyz[3 * i] : 1e100, ry = ok ? xyz[3 * i + 1] : 0.0, rz = ok ? xyz[3 * i + 2] : 0.0;
    const int64_t j0 = n * sp / nsplit, j1 = n * (sp + 1) / nsplit;
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        // every lane reads source j: wave-uniform loads
        const double dx = rx - xyz[3 * j], dy = ry - xyz[3 * j + 1], dz = rz - xyz[3 * j + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv = (j != i) ? rsqrt_nr(r2) : 0.0;  // j == i excluded by index
        double t = 0.0;
        if (MONO) t = f * x[j] * inv;
        if (DIP) t += g * y[j] * (nrm[3 * j] * dx + nrm[3 * j + 1] * dy + nrm[3 * j + 2] * dz) * (inv * inv * inv);
        acc = fma(s[j], t, acc);
    }
    if (live) part[(int64_t)sp * nr + k] = ok ? acc : __builtin_nan("");
}

__global__ void k_direct_sum(const double *__restrict__ part, int64_t nr, int nsplit, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nr) return;
    double v = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) v += part[(int64_t)sp * nr + k];
    out[k] = kInv4PiD * v;
}

int direct_splits(int64_t n, int64_t nr) {
    const int64_t blocks = (nr + kDirThreads - 1) / kDirThreads;
    int64_t sp = (2048 + blocks - 1) / blocks;  // about 2048 waves in flight
    sp = std::min<int64_t>(sp, 64);
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, n / 64));  // at least 64 sources per split
    return (int)std::max<int64_t>(sp, 1);
}

void direct_check(const DirectArgs &a) {
    BFM_CHECK(a.n >= 1, BFM_EINVAL, "n must be >= 1");
    BFM_CHECK(a.nr >= 0, BFM_EINVAL, "nr must be >= 0");
    BFM_CHECK(a.xyz && a.s && a.out, BFM_EINVAL, "null argument");
    BFM_CHECK(a.f == 0.0 || a.x, BFM_EINVAL, "x required when f != 0");
    BFM_CHECK(a.g == 0.0 || (a.y && a.nrm), BFM_EINVAL, "y and nrm required when g != 0");
    BFM_CHECK(a.rows || a.nr <= a.n, BFM_EINVAL, "nr > n without a row list");
}

void direct_launch(const DirectArgs &a, double *part, int nsplit, hipStream_t st) {
    if (a.nr == 0) return;
    const bool mono = a.f != 0.0, dip = a.g != 0.0;
    const dim3 grid((unsigned)((a.nr + kDirThreads - 1) / kDirThreads), (unsigned)nsplit);
    if (mono && dip)
        k_direct_part<true, true><<<grid, kDirThreads, 0, st>>>(a.n, a.xyz, a.s, a.nrm, a.f, a.x, a.g, a.y, a.nr,
                                                                a.rows, nsplit, part);
    else if (mono)
        k_direct_part<true, false><<<grid, kDirThreads, 0, st>>>(a.n, a.xyz, a.s, a.nrm, a.f, a.x, a.g, a.y, a.nr,
                                                                 a.rows, nsplit, part);
    else if (dip)
        k_direct_part<false, true><<<grid, kDirThreads, 0, st>>>(a.n, a.xyz, a.s, a.nrm, a.f, a.x, a.g, a.y, a.nr,
                                                                 a.rows, nsplit, part);
    else
        k_direct_part<false, false><<<grid, kDirThreads, 0, st>>>(a.n, a.xyz, a.s, a.nrm, a.f, a.x, a.g, a.y,
                                                                  a.nr, a.rows, nsplit, part);
    BFM_LAUNCHED();
    k_direct_sum<<<(unsigned)((a.nr + 255) / 256), 256, 0, st>>>(part, a.nr, nsplit, a.out);
    BFM_LAUNCHED();
}

void direct_product(const DirectArgs &a, hipStream_t st) {
    direct_check(a);
    if (a.nr == 0) return;
    const int nsplit = direct_splits(a.n, a.nr);
    double *part = nullptr;
    BFM_HIP(hipMallocAsync((void **)&part, sizeof(double) * (size_t)nsplit * (size_t)a.nr, st));
    try {
        direct_launch(a, part, nsplit, st);
    } catch (...) {
        (void)hipFreeAsync(part, st);
        throw;
    }
    BFM_HIP(hipFreeAsync(part, st));
}

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current (in host code the array's name is a
// host-side stand-in, not a device address).
static double *scratch_ptr() {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptrs[kMaxDevices] = {nullptr};
    int dev = 0;
    BFM_HIP(hipGetDevice(&dev));
    BFM_CHECK(dev >= 0 && dev < kMaxDevices, BFM_EINVAL, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        BFM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        BFM_CHECK(p != nullptr, BFM_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        ptrs[dev] = static_cast<double *>(p);
    }
    return ptrs[dev];
}

void direct_product_noalloc(const DirectArgs &a, hipStream_t st) {
    direct_check(a);
    double *part = scratch_ptr();
    if (a.nr == 0) return;
    const int nsplit = direct_splits(a.n, a.nr);
    BFM_CHECK((int64_t)nsplit * a.nr <= kDirectScratch, BFM_EINVAL,
              "nr = " + std::to_string(a.nr) + " needs " + std::to_string((int64_t)nsplit * a.nr) +
                  " scratch doubles; the allocation-free entry point holds " + std::to_string(kDirectScratch));
    direct_launch(a, part, nsplit, st);
}

}  // namespace bfm
