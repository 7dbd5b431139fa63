// probe.hip -- microbenchmarks for the ceilings the scan kernels are held to
// on the part they run on: the plain (unpacked) FP32 FMA rate, the FP64 FMA
// rate, the issue cost of the FP64 reciprocal square root the traveltime
// starts from, and the LDS read bandwidth, with 16-byte reads and with the
// paired 4-byte reads the scan kernels' windows use.  Each kernel does a fixed amount of
// independent work (several dependence chains per lane, so latency is hidden)
// over 8 workgroups per CU, and is timed with HIP events; the results are the
// measured denominators of the scan kernels' executed-rate rooflines.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "semb.h"

namespace semb {
namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;
constexpr int kLdsVec = 2048;  // float4 words: 32 KB per workgroup

// accumulating FMAs with two per-lane register operands, the form of the
// scan's window loop (U += u f): v_fmac_f32 with VGPR sources
__global__ __launch_bounds__(kThreads) void probe_fma32_kernel(float *out, int iters, float a, float b)
{
    const float x = a + (float)threadIdx.x * 1e-9f;
    float y[kChains], v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        y[c] = b * (float)(c + 1);
        v[c] = 0.f;
    }
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = fmaf(x, y[c], v[c]);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void probe_fma64_kernel(float *out, int iters, double a, double b)
{
    const double x = a + (double)threadIdx.x * 1e-9;
    double y[kChains], v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        y[c] = b * (double)(c + 1);
        v[c] = 0.0;
    }
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = fma(x, y[c], v[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// iterated 1/sqrt converges to 1 from any positive start, so every operand
// stays a normal positive number
__global__ __launch_bounds__(kThreads) void probe_rsq64_kernel(float *out, int iters)
{
    double v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 1.0 + (double)(threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = __builtin_amdgcn_rsq(v[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[blockIdx.x * kThreads + threadIdx.x] = (float)s;
}

// 16-byte LDS reads, consecutive lanes on consecutive words (no bank
// conflicts); the base moves every iteration so no read can be hoisted.
// Indices: base <= 1023 plus offsets <= 7 * 128 stay below kLdsVec.
__global__ __launch_bounds__(kThreads) void probe_lds_kernel(float *out, int iters)
{
    __shared__ float4 buf[kLdsVec];
    for (int i = threadIdx.x; i < kLdsVec; i += kThreads)
        buf[i] = make_float4((float)i, (float)(i + 1), (float)(i + 2), (float)(i + 3));
    __syncthreads();
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        const int base = (threadIdx.x + i * 64) & 1023;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 t = buf[base + u * 128];
            acc ^= __float_as_uint(t.x) ^ __float_as_uint(t.y) ^ __float_as_uint(t.z) ^ __float_as_uint(t.w);
        }
    }
    out[blockIdx.x * kThreads + threadIdx.x] = __uint_as_float(acc & 0x3fffffffu);
}

// 4-byte LDS reads in the scan kernels' pattern: every lane reads 16
// consecutive words from its own start, the starts of neighbouring lanes one
// word apart, so the compiler pairs them into ds_read2_b32 with immediate
// offsets.  Indices: base <= 4095, plus lane <= 255, plus 15 stay below 8192.
__global__ __launch_bounds__(kThreads) void probe_lds2_kernel(float *out, int iters)
{
    __shared__ float buf[4 * kLdsVec];
    for (int i = threadIdx.x; i < 4 * kLdsVec; i += kThreads) buf[i] = (float)i;
    __syncthreads();
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        const float *p = &buf[((i * 192) & 4095) + threadIdx.x];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc ^= __float_as_uint(p[j]);
    }
    out[blockIdx.x * kThreads + threadIdx.x] = __uint_as_float(acc & 0x3fffffffu);
}

struct ProbeShape {
    int iters;
    double work_per_thread;  // flops, instructions or bytes per thread per launch
};

ProbeShape probe_shape(int probe)
{
    switch (probe) {
    case SEMB_PROBE_FMA_F32: return {32768, 32768.0 * kChains * 2};
    case SEMB_PROBE_FMA_F64: return {16384, 16384.0 * kChains * 2};
    case SEMB_PROBE_RSQ_F64: return {8192, 8192.0 * kChains};
    case SEMB_PROBE_LDS_READ2: return {8192, 8192.0 * 16 * 4};
    default: return {8192, 8192.0 * 8 * 16};
    }
}

void launch_probe(int probe, int blocks, float *out, int iters, hipStream_t st)
{
    switch (probe) {
    case SEMB_PROBE_FMA_F32:
        probe_fma32_kernel<<<blocks, kThreads, 0, st>>>(out, iters, 1e-3f, 1e-3f);
        break;
    case SEMB_PROBE_FMA_F64:
        probe_fma64_kernel<<<blocks, kThreads, 0, st>>>(out, iters, 1e-3, 1e-3);
        break;
    case SEMB_PROBE_RSQ_F64:
        probe_rsq64_kernel<<<blocks, kThreads, 0, st>>>(out, iters);
        break;
    case SEMB_PROBE_LDS_READ2:
        probe_lds2_kernel<<<blocks, kThreads, 0, st>>>(out, iters);
        break;
    default:
        probe_lds_kernel<<<blocks, kThreads, 0, st>>>(out, iters);
        break;
    }
}

}  // namespace

// Runs one probe: a warm-up launch, then `reps` timed launches on a stream of
// its own; rate = work per launch / mean launch time.  Returns a hipError_t.
int run_probe(int probe, int reps, double *rate, double *ms)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const int blocks = 8 * (cus > 0 ? cus : 1);
    const ProbeShape ps = probe_shape(probe);
    float *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    e = hipMalloc((void **)&out, sizeof(float) * (size_t)blocks * kThreads);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    float total = 0.f;
    if (e == hipSuccess) {
        launch_probe(probe, blocks, out, ps.iters, st);
        e = hipEventRecord(ev0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            launch_probe(probe, blocks, out, ps.iters, st);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(ev1, st);
        if (e == hipSuccess) e = hipEventSynchronize(ev1);
        if (e == hipSuccess) e = hipEventElapsedTime(&total, ev0, ev1);
    }
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    const double mean_ms = (double)total / reps;
    *ms = mean_ms;
    *rate = ps.work_per_thread * (double)blocks * kThreads / (mean_ms * 1e-3);
    return 0;
}

}  // namespace semb
