// Microbenchmarks of the two device limits the annealing kernels are
// measured against: the int32 vector (VALU) issue rate and the LDS read
// bandwidth of the CUs.  Each probe fills every CU with wavefronts doing
// nothing but the measured operation (independent chains, no memory traffic
// besides one store per lane at the end) and is timed with HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xzzx_internal.h"

namespace xzzx {

// Eight independent dependency chains per lane, 16 x 8 instructions of one
// kind per loop trip (the loop's own scalar work overlaps them).
template <int KIND>
__global__ __launch_bounds__(256) void k_probe_valu(uint32_t *out, uint32_t seed, int iters)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[8];
    uint64_t m[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = seed ^ (tid * 0x9E3779B9u + (uint32_t)i);
        m[i] = a[i];
    }
    const uint32_t b = tid | 1u, c = tid ^ seed;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if constexpr (KIND == 0) {
                    asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
                } else if constexpr (KIND == 1) {
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
                } else if constexpr (KIND == 2) {
                    asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[i]) : "v"(b), "v"(c));
                } else {
                    // one v_mad_u64_u32 (the multiply of a Philox round)
                    m[i] = (uint64_t)(uint32_t)m[i] * (uint64_t)b + m[i];
                }
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r ^= a[i] ^ (uint32_t)m[i] ^ (uint32_t)(m[i] >> 32);
    out[tid] = r;
}

// LDS reads of BYTES per lane, conflict-free (consecutive lanes read
// consecutive addresses), 16 distinct reads per loop trip at immediate
// offsets; the XOR of what was read keeps the loads.
constexpr int kProbeLdsBytes = 16384;   // per workgroup
template <typename T> __device__ __forceinline__ uint32_t fold(const T &v);
template <> __device__ __forceinline__ uint32_t fold(const uint32_t &v) { return v; }
template <> __device__ __forceinline__ uint32_t fold(const uint2 &v) { return v.x ^ v.y; }
template <> __device__ __forceinline__ uint32_t fold(const uint4 &v) { return v.x ^ v.y ^ v.z ^ v.w; }

template <typename T>
__global__ __launch_bounds__(256) void k_probe_lds(uint32_t *out, int iters)
{
    constexpr int N = kProbeLdsBytes / (int)sizeof(T);
    static_assert(N >= 16 * 64, "16 distinct reads per trip");
    __shared__ T buf[N];
    const int t = threadIdx.x;
    uint32_t *w = reinterpret_cast<uint32_t *>(buf);
    for (int i = t; i < kProbeLdsBytes / 4; i += 256) w[i] = (uint32_t)i * 0x9E3779B9u;
    __syncthreads();
    uint32_t acc = 0;
    int lane = t & 63;
    for (int it = 0; it < iters; ++it) {
        asm volatile("" : "+v"(lane));   // the reads are not loop-invariant
#pragma unroll
        for (int k = 0; k < 16; ++k) acc ^= fold(buf[lane + 64 * k]);
    }
    out[blockIdx.x * blockDim.x + t] = acc;
}

static int probe_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// Best of `reps` timed launches (after one warm-up), in ms.
template <typename L>
static int probe_time(hipStream_t s, int reps, L launch, float *best_ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        set_error("event creation failed");
        return XZZX_EDEVICE;
    }
    launch();
    float best = 1e30f;
    int rc = XZZX_OK;
    for (int r = 0; r < reps && !rc; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = XZZX_EDEVICE;
        launch();
        if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = XZZX_EDEVICE;
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = XZZX_EDEVICE;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = XZZX_EDEVICE;
        if (!rc) best = std::min(best, ms);
    }
    if (!rc && hipGetLastError() != hipSuccess) rc = XZZX_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) { set_error("probe launch or timing failed"); return rc; }
    *best_ms = best;
    return XZZX_OK;
}

}  // namespace xzzx

using namespace xzzx;

extern "C" {

int xzzx_probe_valu(int kind, int waves_per_simd, int iters, void *stream, double *lane_ops_per_s)
{
    if (kind < 0 || kind > 3 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || iters > (1 << 20) ||
        !lane_ops_per_s) {
        set_error("bad probe arguments");
        return XZZX_EINVAL;
    }
    const int cus = probe_cus();
    if (cus <= 0) { set_error("no device"); return XZZX_EDEVICE; }
    const int blocks = cus * waves_per_simd;   // 4 waves (one per SIMD) per workgroup
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) { set_error("hipMalloc failed"); return XZZX_ENOMEM; }
    hipStream_t s = (hipStream_t)stream;
    auto launch = [&]() {
        switch (kind) {
        case 0: hipLaunchKernelGGL(k_probe_valu<0>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
        case 1: hipLaunchKernelGGL(k_probe_valu<1>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
        case 2: hipLaunchKernelGGL(k_probe_valu<2>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
        default: hipLaunchKernelGGL(k_probe_valu<3>, dim3(blocks), dim3(256), 0, s, out, 7u, iters); break;
        }
    };
    float ms = 0.f;
    const int rc = probe_time(s, 5, launch, &ms);
    (void)hipFree(out);
    if (rc) return rc;
    *lane_ops_per_s = (double)blocks * 256.0 * (double)iters * 128.0 / (ms * 1e-3);
    return XZZX_OK;
}

int xzzx_probe_lds(int bytes_per_read, int waves_per_simd, int iters, void *stream, double *bytes_per_s)
{
    if ((bytes_per_read != 4 && bytes_per_read != 8 && bytes_per_read != 16) || waves_per_simd < 1 ||
        waves_per_simd > 8 || iters < 1 || iters > (1 << 20) || !bytes_per_s) {
        set_error("bad probe arguments");
        return XZZX_EINVAL;
    }
    const int cus = probe_cus();
    if (cus <= 0) { set_error("no device"); return XZZX_EDEVICE; }
    const int blocks = cus * waves_per_simd;
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) { set_error("hipMalloc failed"); return XZZX_ENOMEM; }
    hipStream_t s = (hipStream_t)stream;
    auto launch = [&]() {
        if (bytes_per_read == 4) hipLaunchKernelGGL(k_probe_lds<uint32_t>, dim3(blocks), dim3(256), 0, s, out, iters);
        else if (bytes_per_read == 8) hipLaunchKernelGGL(k_probe_lds<uint2>, dim3(blocks), dim3(256), 0, s, out, iters);
        else hipLaunchKernelGGL(k_probe_lds<uint4>, dim3(blocks), dim3(256), 0, s, out, iters);
    };
    float ms = 0.f;
    const int rc = probe_time(s, 5, launch, &ms);
    (void)hipFree(out);
    if (rc) return rc;
    *bytes_per_s = (double)blocks * 256.0 * (double)iters * 16.0 * bytes_per_read / (ms * 1e-3);
    return XZZX_OK;
}

}  // extern "C"
