// Ceiling microbenchmarks for the roofline of the ray-march kernels on gfx950:
// HBM streaming copy, scattered FP32 atomics (device scope, and workgroup
// scope into a per-XCD private region), LDS FP32 atomics and the exp issue
// rate.  Each entry point allocates its own buffers, times its kernel with HIP
// events and returns operations (or bytes) per second.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

__device__ inline uint32_t lcg(uint32_t x) { return x * 1664525u + 1013904223u; }

__device__ inline int xcc_id()
{
    // hardware register XCC_ID (id 20), bits [3:0]: the XCD this wave runs on
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & 0xF;
}

__global__ void k_copy(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// scattered device-scope atomics over `nwords` floats
__global__ void k_atomic_dev(float *p, uint32_t nwords, int iters)
{
    uint32_t x = lcg(blockIdx.x * blockDim.x + threadIdx.x + 12345u);
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        __hip_atomic_fetch_add(p + (x % nwords), 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// scattered workgroup-scope atomics into the region private to this XCD
__global__ void k_atomic_xcd(float *p, uint32_t nwords_per_xcd, int iters)
{
    uint32_t x = lcg(blockIdx.x * blockDim.x + threadIdx.x + 777u);
    float *mine = p + (size_t)(xcc_id() & 7) * nwords_per_xcd;
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        __hip_atomic_fetch_add(mine + (x % nwords_per_xcd), 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// coalesced device-scope atomics: each instruction's lanes cover `group`
// consecutive floats at a random group-aligned base (64 lanes / group bases)
__global__ void k_atomic_grouped(float *p, uint32_t ngroups, int group, int iters)
{
    const int lane = threadIdx.x & 63;
    uint32_t x = lcg((blockIdx.x * blockDim.x + threadIdx.x) / group + 4242u);
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        __hip_atomic_fetch_add(p + (size_t)(x % ngroups) * group + (lane % group), 1.0f, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// FP64 atomics in groups of 8 consecutive doubles (one 64-byte row per group,
// 8 rows per 64-lane instruction) at random row indices
__global__ void k_atomic_rows_f64(double *p, uint32_t nrows, int iters)
{
    const int lane = threadIdx.x & 63;
    uint32_t x = lcg((blockIdx.x * blockDim.x + threadIdx.x) / 8 + 1717u);
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        __hip_atomic_fetch_add(p + (size_t)(x % nrows) * 8 + (lane & 7), 1.0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// FP32 atomics in 64-byte rows of 16 floats (4 rows per 64-lane instruction)
// at random row indices
__global__ void k_atomic_rows_f32(float *p, uint32_t nrows, int iters)
{
    const int lane = threadIdx.x & 63;
    uint32_t x = lcg((blockIdx.x * blockDim.x + threadIdx.x) / 16 + 2929u);
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        __hip_atomic_fetch_add(p + (size_t)(x % nrows) * 16 + (lane & 15), 1.0f, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_lds_atomic(float *out, int iters)
{
    __shared__ float s[4096];
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) s[i] = 0.f;
    __syncthreads();
    uint32_t x = lcg(threadIdx.x + 99u);
    for (int k = 0; k < iters; ++k) {
        x = lcg(x);
        atomicAdd(&s[x & 4095], 1.0f);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

__global__ void k_exp(float *out, int iters)
{
    float a = threadIdx.x * 1e-3f, b = 0.5f, c = 0.25f, d = 0.125f;
    for (int k = 0; k < iters; ++k) {
        a = __expf(-a);
        b = __expf(-b);
        c = __expf(-c);
        d = __expf(-d);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a + b + c + d;
}

__global__ void k_xcc_hist(int *hist)
{
    if (threadIdx.x == 0) atomicAdd(&hist[xcc_id()], 1);
}

struct Timer {
    hipEvent_t a, b;
    Timer()
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

// which: 0 copy (bytes/s, read + write), 1 device-scope atomics (ops/s),
// 2 per-XCD workgroup-scope atomics (ops/s), 3 LDS atomics (ops/s),
// 4 exp (ops/s), 5 atomics in groups of 64 consecutive floats, 6 in groups of
// 8 (lane-ops/s), 7 FP64 atomics in 64-byte rows of 8 doubles (rows/s),
// 8 FP32 atomics in 64-byte rows of 16 floats (rows/s).
// footprint: bytes for 0-2 and 5-8.  Returns 0 on success.
int drceil_run(int which, size_t footprint, int iters, double *per_s)
{
    Timer tm;
    float *buf = nullptr, *buf2 = nullptr;
    const int blocks = 4096, threads = 256;
    hipError_t e = hipSuccess;
    double ops = 0.0;
    if (which <= 2 || which >= 5) {   // footprint-sized buffer
        e = hipMalloc(&buf, footprint);
        if (e != hipSuccess) return -2;
        (void)hipMemset(buf, 0, footprint);
    } else {
        e = hipMalloc(&buf, sizeof(float) * blocks * threads);
        if (e != hipSuccess) return -2;
    }
    if (which == 0) {
        e = hipMalloc(&buf2, footprint);
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return -2;
        }
    }
    for (int rep = 0; rep < 2; ++rep) {   // first repetition warms up
        (void)hipEventRecord(tm.a, 0);
        if (which == 0) {
            const size_t n = footprint / sizeof(float4);
            hipLaunchKernelGGL(k_copy, dim3(blocks * 4), dim3(threads), 0, 0, (const float4 *)buf, (float4 *)buf2, n);
            ops = 2.0 * (double)n * sizeof(float4);
        } else if (which == 1) {
            hipLaunchKernelGGL(k_atomic_dev, dim3(blocks), dim3(threads), 0, 0, buf, (uint32_t)(footprint / 4), iters);
            ops = (double)blocks * threads * iters;
        } else if (which == 2) {
            hipLaunchKernelGGL(k_atomic_xcd, dim3(blocks), dim3(threads), 0, 0, buf, (uint32_t)(footprint / 4 / 8), iters);
            ops = (double)blocks * threads * iters;
        } else if (which == 7) {
            hipLaunchKernelGGL(k_atomic_rows_f64, dim3(blocks), dim3(threads), 0, 0, (double *)buf,
                               (uint32_t)(footprint / 64), iters);
            ops = (double)blocks * threads * iters / 8.0;
        } else if (which == 8) {
            hipLaunchKernelGGL(k_atomic_rows_f32, dim3(blocks), dim3(threads), 0, 0, buf, (uint32_t)(footprint / 64),
                               iters);
            ops = (double)blocks * threads * iters / 16.0;
        } else if (which == 5 || which == 6) {
            const int group = which == 5 ? 64 : 8;
            hipLaunchKernelGGL(k_atomic_grouped, dim3(blocks), dim3(threads), 0, 0, buf,
                               (uint32_t)(footprint / 4 / group), group, iters);
            ops = (double)blocks * threads * iters;
        } else if (which == 3) {
            hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(threads), 0, 0, buf, iters);
            ops = (double)blocks * threads * iters;
        } else {
            hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(threads), 0, 0, buf, iters);
            ops = 4.0 * blocks * threads * iters;
        }
        (void)hipEventRecord(tm.b, 0);
    }
    e = hipEventSynchronize(tm.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, tm.a, tm.b);
    (void)hipFree(buf);
    if (buf2) (void)hipFree(buf2);
    if (e != hipSuccess) return -3;
    *per_s = ops / (ms * 1e-3);
    return 0;
}

// Histogram of the XCD ids that `blocks` one-wave workgroups run on.
int drceil_xcc_hist(int blocks, int *hist8)
{
    int *d = nullptr;
    if (hipMalloc(&d, sizeof(int) * 16) != hipSuccess) return -2;
    (void)hipMemset(d, 0, sizeof(int) * 16);
    hipLaunchKernelGGL(k_xcc_hist, dim3(blocks), dim3(64), 0, 0, d);
    hipError_t e = hipMemcpy(hist8, d, sizeof(int) * 8, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? 0 : -3;
}

}  // extern "C"
