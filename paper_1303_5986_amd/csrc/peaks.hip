// peaks.hip -- microbenchmarks of the ceilings the kernels' rooflines are
// priced against, measured on the device at hand (gfx950): HBM copy
// bandwidth, LDS read bandwidth, FP64 FMA rate and 32-bit integer
// lane-operation rate.  Not part of the method; bench.py reports them beside
// the published figures.
//
// Each kernel does enough independent work per lane that its own pipeline,
// not latency, is the limit, and writes one value per thread so nothing is
// optimised away.
#include "we_internal.h"

#include <algorithm>

namespace {

__global__ __launch_bounds__(256) void pk_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 64 KB of LDS read as 16-byte words by every lane, consecutive lanes on
// consecutive words (conflict-free), the words xor-folded into a register.
#define PK_LDS_WORDS 4096
__global__ __launch_bounds__(256) void pk_lds(uint4 *__restrict__ out, int32_t iters) {
    __shared__ uint4 buf[PK_LDS_WORDS];
    for (int i = threadIdx.x; i < PK_LDS_WORDS; i += 256)
        buf[i] = make_uint4((uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int base = threadIdx.x;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint4 v = buf[(base + u * 256) & (PK_LDS_WORDS - 1)];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
        base = (base + 64) & (PK_LDS_WORDS - 1);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Eight independent FMA chains per lane.
__global__ __launch_bounds__(256) void pk_fp64(double *__restrict__ out, int32_t iters, double a, double b) {
    double x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (double)(threadIdx.x + c);
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Eight independent chains of x = (x ^ a) + b per lane: two 32-bit integer
// lane operations per step.
__global__ __launch_bounds__(256) void pk_int(uint32_t *__restrict__ out, int32_t iters, uint32_t a, uint32_t b) {
    uint32_t x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = threadIdx.x * 2654435761u + (uint32_t)c;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = (x[c] ^ a) + b;
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s ^= x[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Median of `reps` timed launches (after one untimed) of `launch`.
template <class F>
hipError_t time_ms(hipStream_t st, int reps, F launch, double *ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) { (void)hipEventDestroy(e0); return e; }
    std::vector<float> t;
    launch();
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) launch();
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float v = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&v, e0, e1);
        t.push_back(v);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return hipSuccess;
}

}  // namespace

extern "C" we_status we_measure_peaks(void *hip_stream, we_peaks *out) {
    if (!out) return we_fail(WE_EINVAL, "NULL output");
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus < 1) return we_fail(WE_EDEVICE, "no compute units reported");
    const int64_t n = (int64_t)1 << 26;              // 64 Mi x 16 B = 1 GiB per buffer
    uint4 *src = nullptr, *dst = nullptr;
    HIP_TRY(hipMalloc(&src, (size_t)n * 16));
    hipError_t e = hipMalloc(&dst, (size_t)n * 16);
    if (e != hipSuccess) { (void)hipFree(src); return we_hip_fail(e, "hipMalloc"); }
    const int blocks = cus * 8;
    void *scratch = nullptr;
    e = hipMalloc(&scratch, (size_t)blocks * 256 * 16);
    double ms = 0.0;
    if (e == hipSuccess) e = hipMemsetAsync(src, 1, (size_t)n * 16, st);
    if (e == hipSuccess)
        e = time_ms(st, 5, [&] { hipLaunchKernelGGL(pk_copy, dim3(blocks * 4), dim3(256), 0, st, src, dst, n); }, &ms);
    if (e == hipSuccess) out->hbm_gbs = 2.0 * 16.0 * (double)n / (ms * 1e-3) / 1e9;
    const int32_t lds_iters = 4096;
    if (e == hipSuccess)
        e = time_ms(st, 5, [&] {
            hipLaunchKernelGGL(pk_lds, dim3(blocks), dim3(256), 0, st, (uint4 *)scratch, lds_iters);
        }, &ms);
    if (e == hipSuccess) out->lds_tbs = (double)blocks * 256 * lds_iters * 16 * 16 / (ms * 1e-3) / 1e12;
    const int32_t f_iters = 16384;
    if (e == hipSuccess)
        e = time_ms(st, 5, [&] {
            hipLaunchKernelGGL(pk_fp64, dim3(blocks), dim3(256), 0, st, (double *)scratch, f_iters, 0.999999, 1e-7);
        }, &ms);
    if (e == hipSuccess) out->fp64_tflops = (double)blocks * 256 * f_iters * 8 * 2 / (ms * 1e-3) / 1e12;
    if (e == hipSuccess)
        e = time_ms(st, 5, [&] {
            hipLaunchKernelGGL(pk_int, dim3(blocks), dim3(256), 0, st, (uint32_t *)scratch, f_iters, 0x9E3779B9u,
                               0x7F4A7C15u);
        }, &ms);
    if (e == hipSuccess) out->int32_tops = (double)blocks * 256 * f_iters * 8 * 2 / (ms * 1e-3) / 1e12;
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipFree(scratch);
    if (e != hipSuccess) return we_hip_fail(e, "peak microbenchmarks");
    out->compute_units = cus;
    return WE_OK;
}
