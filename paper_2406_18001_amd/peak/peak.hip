// Peak microbenchmarks of the MI355X units the kernel-block products use:
// MFMA throughput per instruction shape (independent accumulator chains in
// every wave, no memory traffic) and HBM stream bandwidth (read-only
// reduction and copy).  Built into a library of its own; the product library
// does not use it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;   // independent accumulators per wave

template <int SHAPE>
__global__ __launch_bounds__(256) void mfma_loop(int iters, float *out)
{
    const int lane = threadIdx.x & 63;
    if constexpr (SHAPE == 0) {          // f64 16x16x4
        d4 acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
        const double a = 1e-3 * (lane + 1), b = 1e-3 * (64 - lane);
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        double s = 0.0;
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][3];
        if (s == -1.0) out[blockIdx.x] = (float)s;
    } else if constexpr (SHAPE == 1 || SHAPE == 3) {   // bf16 / f16 16x16x32
        f4 acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        bf8 ab;
        h8 ah;
        for (int e = 0; e < 8; ++e) {
            ab[e] = (__bf16)(1e-3f * (lane + e));
            ah[e] = (_Float16)(1e-3f * (lane + e));
        }
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (SHAPE == 1)
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, ab, acc[c], 0, 0, 0);
                else
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, ah, acc[c], 0, 0, 0);
            }
        float s = 0.f;
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][3];
        if (s == -1.f) out[blockIdx.x] = s;
    } else {                              // bf16 32x32x16 (SHAPE 2)
        f16v acc[kChains / 2];
        for (int c = 0; c < kChains / 2; ++c)
            for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
        bf8 ab;
        for (int e = 0; e < 8; ++e) ab[e] = (__bf16)(1e-3f * (lane + e));
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < kChains / 2; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, acc[c], 0, 0, 0);
        float s = 0.f;
        for (int c = 0; c < kChains / 2; ++c) s += acc[c][0] + acc[c][15];
        if (s == -1.f) out[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void stream_read(const double4 *__restrict__ x, int64_t n4,
                                                   double *__restrict__ out)
{
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double4 v = x[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == -1.0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void stream_copy(const double4 *__restrict__ x,
                                                   double4 *__restrict__ y, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

template <class F>
double time_ms(F launch, int reps)
{
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    launch();                                  // warm-up
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / reps;
}

}  // namespace

extern "C" {

/* MFMA throughput in TFLOP/s of one instruction shape: 0 = f64 16x16x4,
 * 1 = bf16 16x16x32, 2 = bf16 32x32x16, 3 = f16 16x16x32.  `waves_per_simd`
 * waves of independent chains on every SIMD of the device.  Returns < 0 on
 * a HIP error. */
double kdcd_peak_mfma(int shape, int waves_per_simd)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1.0;
    float *out = nullptr;
    const int blocks = cus * waves_per_simd;   // 4 waves per block: one per SIMD
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks) != hipSuccess) return -1.0;
    const int iters = 2048;
    double flops_per = 0.0;
    int per_iter = kChains;
    switch (shape) {
    case 0: flops_per = 2.0 * 16 * 16 * 4; break;
    case 1: case 3: flops_per = 2.0 * 16 * 16 * 32; break;
    case 2: flops_per = 2.0 * 32 * 32 * 16; per_iter = kChains / 2; break;
    default: (void)hipFree(out); return -1.0;
    }
    auto go = [&]() {
        switch (shape) {
        case 0: hipLaunchKernelGGL(mfma_loop<0>, dim3(blocks), dim3(256), 0, nullptr, iters, out); break;
        case 1: hipLaunchKernelGGL(mfma_loop<1>, dim3(blocks), dim3(256), 0, nullptr, iters, out); break;
        case 2: hipLaunchKernelGGL(mfma_loop<2>, dim3(blocks), dim3(256), 0, nullptr, iters, out); break;
        default: hipLaunchKernelGGL(mfma_loop<3>, dim3(blocks), dim3(256), 0, nullptr, iters, out); break;
        }
    };
    const double ms = time_ms(go, 5);
    const bool ok = hipGetLastError() == hipSuccess;
    (void)hipFree(out);
    if (!ok) return -1.0;
    const double flops = flops_per * per_iter * iters * (double)blocks * 4.0;
    return flops / (ms * 1e-3) / 1e12;
}

/* HBM stream bandwidth in GB/s over `bytes` (a multiple of 32): mode 0 reads
 * the buffer once (sum), mode 1 copies it (read + write counted). */
double kdcd_peak_stream(int mode, int64_t bytes)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1.0;
    const int64_t n4 = bytes / 32;
    double4 *x = nullptr, *y = nullptr;
    double *o = nullptr;
    if (hipMalloc(&x, (size_t)n4 * 32) != hipSuccess) return -1.0;
    if (mode == 1 && hipMalloc(&y, (size_t)n4 * 32) != hipSuccess) { (void)hipFree(x); return -1.0; }
    if (hipMalloc(&o, sizeof(double) * 65536) != hipSuccess) { (void)hipFree(x); (void)hipFree(y); return -1.0; }
    (void)hipMemset(x, 0, (size_t)n4 * 32);
    const int blocks = cus * 8;
    auto go = [&]() {
        if (mode == 0) hipLaunchKernelGGL(stream_read, dim3(blocks), dim3(256), 0, nullptr, x, n4, o);
        else hipLaunchKernelGGL(stream_copy, dim3(blocks), dim3(256), 0, nullptr, x, y, n4);
    };
    const double ms = time_ms(go, 10);
    const bool ok = hipGetLastError() == hipSuccess;
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipFree(o);
    if (!ok) return -1.0;
    const double moved = (double)n4 * 32.0 * (mode == 1 ? 2.0 : 1.0);
    return moved / (ms * 1e-3) / 1e9;
}

}  // extern "C"
