// Measurement only: the rate at which the device performs LDS atomic adds at random addresses,
// the ceiling of the vote step, whose work is one LDS atomic add per vote.
//
// Each 1024-thread workgroup holds 64 KiB of u32 counters in LDS (two workgroups fit a
// compute unit, 32 waves) and every lane adds into one of the two 16-bit halves of a
// pseudo-random counter per iteration, as the vote kernel does.  The returning form keeps the
// old values (summed, so the adds stay independent and several are in flight per wave); the
// other form discards them.
#include "rd_host.h"

namespace rd {
namespace {

constexpr int CNT = 1024;
constexpr int CAL_WORDS = 16384;   // 64 KiB

__device__ uint32_t g_sink;          // written only if a checksum takes one given value

template <bool RTN>
__global__ __launch_bounds__(CNT) void k_lds_atomic_rate(int iters) {
    __shared__ uint32_t s[CAL_WORDS];
    for (int i = threadIdx.x; i < CAL_WORDS; i += CNT) s[i] = 0u;
    __syncthreads();
    uint32_t x = (blockIdx.x * CNT + threadIdx.x) * 2654435761u + 12345u;
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        x = x * 1664525u + 1013904223u;                 // LCG step
        const uint32_t idx = x >> 18;                    // 14 bits: 0 .. CAL_WORDS - 1
        const uint32_t inc = 1u << ((x >> 4) & 16u);     // low or high half
        if (RTN)
            acc += atomicAdd(&s[idx], inc);
        else
            atomicAdd(&s[idx], inc);
    }
    __syncthreads();
    acc += s[threadIdx.x];
    if (acc == 0x9e3779b9u) g_sink = acc;               // keeps the counters live
}

}  // namespace
}  // namespace rd

using namespace rd;

extern "C" rd_status rd_measure_lds_atomics(int32_t device, int32_t with_return, double* atomics_per_s,
                                            double* ms) {
    if (!atomics_per_s || (with_return != 0 && with_return != 1)) return RD_E_INVALID;
    *atomics_per_s = 0.0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RD_E_DEVICE;
    RD_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    RD_HIP(hipGetDeviceProperties(&prop, device));
    const int blocks = 8 * prop.multiProcessorCount;   // four rounds of two workgroups per CU
    const int iters = 2048;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RD_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return RD_E_DEVICE;
    }
    hipError_t err = hipSuccess;
    float best = 0.f;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        (void)hipEventRecord(e0, nullptr);
        if (with_return)
            hipLaunchKernelGGL(k_lds_atomic_rate<true>, dim3(blocks), dim3(CNT), 0, nullptr, iters);
        else
            hipLaunchKernelGGL(k_lds_atomic_rate<false>, dim3(blocks), dim3(CNT), 0, nullptr, iters);
        err = hipGetLastError();
        (void)hipEventRecord(e1, nullptr);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (rep > 0 && (best == 0.f || t < best)) best = t;   // the first launch warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess || best <= 0.f) return RD_E_DEVICE;
    const double n = static_cast<double>(blocks) * CNT * iters;
    *atomics_per_s = n / (best * 1e-3);
    if (ms) *ms = best;
    return RD_OK;
}
