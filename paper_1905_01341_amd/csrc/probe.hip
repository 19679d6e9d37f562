// Ceiling probes: kernels that issue one instruction mix back to back, so
// that the roofline of a hot kernel can be stated against what the device
// delivers for the same mix as well as against its published peak.
//
// kind 0  FP64 MFMA      v_mfma_f64_16x16x4f64, 4 independent accumulators per wave
// kind 1  FP64 FMA       8 independent fma chains per lane
// kind 2  FP32 FMA       the same in FP32 (scalar code: the build disables packed FP32)
// kind 3  FP64 pair      the symmetric near field's pair step: sources from LDS, four
//                        receivers per lane, r^2, -2/r by the hardware estimate and one
//                        Newton step, two fma accumulations (11 algorithmic flops per pair)
// kind 4  FP32 pair      the same with the FP32 estimate (v_rsq_f32) and no Newton step
// kind 5  BF16 MFMA      v_mfma_f32_16x16x32_bf16, 4 independent accumulators per wave
//
// Each lane writes its accumulators to out, so no step can be dropped; the
// operands come from in at run time.
#include <hip/hip_runtime.h>

#include "common.h"

namespace bfm {

typedef double pdbl4 __attribute__((ext_vector_type(4)));
typedef float pflt4 __attribute__((ext_vector_type(4)));
typedef __bf16 pbf8 __attribute__((ext_vector_type(8)));

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 4096;
constexpr int kProbeAcc = 4;      // independent MFMA accumulators per wave
constexpr int kProbeUnroll = 16;  // MFMA rounds per loop trip (the accumulators stay in place)

__global__ void __launch_bounds__(kProbeThreads) k_probe_mfma64(int iters, const double *in, double *out) {
    const int lane = threadIdx.x & 63;
    const double a = in[lane], b = in[64 + lane];
    pdbl4 acc[kProbeAcc];
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) acc[k] = pdbl4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kProbeAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kProbeThreads) k_probe_bf16(int iters, const double *in, double *out) {
    const int lane = threadIdx.x & 63;
    pbf8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(float)in[(lane + k) & 63];
        b[k] = (__bf16)(float)in[64 + ((lane + 3 * k) & 63)];
    }
    pflt4 acc[kProbeAcc];
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) acc[k] = pflt4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kProbeAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

template <class T>
__global__ void __launch_bounds__(kProbeThreads) k_probe_fma(int iters, const double *in, double *out) {
    const int lane = threadIdx.x & 63;
    const T a = (T)in[lane], b = (T)in[64 + lane];
    T x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (T)in[k];
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
    T s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = (double)s;
}

// Pair step of the near field: 64 sources in LDS, visited by the lanes in
// rotated order (lane l takes source (l + t) mod 64 at step t), four
// receivers per lane.
template <class T>
__global__ void __launch_bounds__(kProbeThreads) k_probe_pair(int iters, const double *in, double *out) {
    __shared__ T sx[kProbeThreads / 64][64], sy[kProbeThreads / 64][64], sz[kProbeThreads / 64][64],
        sq[kProbeThreads / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    sx[wave][lane] = (T)in[lane];
    sy[wave][lane] = (T)in[(lane + 7) & 63];
    sz[wave][lane] = (T)in[(lane + 19) & 63] + (T)3;
    sq[wave][lane] = (T)in[64 + lane];
    __syncthreads();
    T xi[4], yi[4], zi[4], acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xi[k] = (T)in[(lane + 11 * k) & 63] + (T)0.5;
        yi[k] = (T)in[(lane + 13 * k + 1) & 63];
        zi[k] = (T)in[(lane + 17 * k + 2) & 63];
        acc[k] = 0;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll 2
        for (int t = 0; t < 64; ++t) {
            const int s = (lane + t) & 63;
            const T ax = sx[wave][s], ay = sy[wave][s], az = sz[wave][s], q = sq[wave][s];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T dx = xi[k] - ax, dy = yi[k] - ay, dz = zi[k] - az;
                const T r2 = dx * dx + dy * dy + dz * dz;
                T inv;
                if constexpr (sizeof(T) == 8) {
                    const T y = __builtin_amdgcn_rsq(r2);
                    inv = y * fma(r2 * y, y, (T)-3);
                } else {
                    inv = __builtin_amdgcn_rsqf(r2);
                }
                acc[k] = fma(q, inv, acc[k]);
            }
        }
    }
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = (double)(acc[0] + acc[1] + acc[2] + acc[3]);
}

// ops per launch of kind at iters (flops; pairs x 11 for the pair probes)
static double probe_ops(int kind, int iters) {
    const double lanes = (double)kProbeBlocks * kProbeThreads, waves = lanes / 64.0;
    switch (kind) {
        case 0: return waves * iters * kProbeUnroll * kProbeAcc * (2.0 * 16 * 16 * 4);
        case 1:
        case 2: return lanes * iters * 8.0 * 2.0;
        case 3:
        case 4: return lanes * iters * 64.0 * 4.0 * 11.0;
        case 5: return waves * iters * kProbeUnroll * kProbeAcc * (2.0 * 16 * 16 * 32);
    }
    return 0.0;
}

void probe_run(int kind, int iters, double *ms, double *ops) {
    BFM_CHECK(kind >= 0 && kind <= 5, BFM_EINVAL, "probe kind must be 0..5");
    BFM_CHECK(iters >= 1 && iters <= (1 << 16), BFM_EINVAL, "probe iterations must be in [1, 2^16]");
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    double *in = nullptr, *out = nullptr;
    BFM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    auto cleanup = [&]() {
        if (in) (void)hipFree(in);
        if (out) (void)hipFree(out);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (st) (void)hipStreamDestroy(st);
    };
    try {
        BFM_HIP(hipEventCreate(&a));
        BFM_HIP(hipEventCreate(&b));
        BFM_HIP(hipMalloc((void **)&in, 128 * sizeof(double)));
        BFM_HIP(hipMalloc((void **)&out, sizeof(double) * kProbeBlocks * kProbeThreads));
        double h[128];
        for (int i = 0; i < 128; ++i) h[i] = 0.25 + 1e-3 * i;  // |a| < 1 keeps the chains finite
        BFM_HIP(hipMemcpyAsync(in, h, sizeof(h), hipMemcpyHostToDevice, st));
        auto launch = [&]() {
            const dim3 g(kProbeBlocks), t(kProbeThreads);
            switch (kind) {
                case 0: k_probe_mfma64<<<g, t, 0, st>>>(iters, in, out); break;
                case 1: k_probe_fma<double><<<g, t, 0, st>>>(iters, in, out); break;
                case 2: k_probe_fma<float><<<g, t, 0, st>>>(iters, in, out); break;
                case 3: k_probe_pair<double><<<g, t, 0, st>>>(iters, in, out); break;
                case 4: k_probe_pair<float><<<g, t, 0, st>>>(iters, in, out); break;
                case 5: k_probe_bf16<<<g, t, 0, st>>>(iters, in, out); break;
            }
            BFM_LAUNCHED();
        };
        launch();  // warm-up
        BFM_HIP(hipEventRecord(a, st));
        launch();
        BFM_HIP(hipEventRecord(b, st));
        BFM_HIP(hipEventSynchronize(b));
        float t = 0.f;
        BFM_HIP(hipEventElapsedTime(&t, a, b));
        *ms = t;
        *ops = probe_ops(kind, iters);
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace bfm
