// Measurement support: the sustained issue rate of the XOR + population
// count instruction pair that the plain search is built from, used as the
// ALU roofline of that kernel. Sixteen independent accumulator chains per
// lane, each step exactly v_xor_b32 (one SGPR operand) + v_bcnt_u32_b32 with
// accumulate, as in the search's inner loop; 16 workgroups of 256 threads
// per compute unit.
#include "internal.h"

namespace homs {
namespace {

constexpr int kChains = 16;

__global__ __launch_bounds__(256) void xor_popcount_rate_kernel(uint32_t* __restrict__ out,
                                                                uint32_t seed, int iters)
{
    uint32_t acc[kChains], q[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        acc[c] = 0u;
        q[c] = (seed + threadIdx.x) * (uint32_t)(c + 1);
    }
    const uint32_t w = __builtin_amdgcn_readfirstlane(seed * 2654435761u);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            uint32_t t;
            asm volatile("v_xor_b32 %0, %1, %2" : "=v"(t) : "s"(w), "v"(q[c]));
            asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc[c]) : "v"(t));
        }
    }
    uint32_t r = 0u;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r += acc[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace
}  // namespace homs

extern "C" homs_status homs_measure_xor_popcount_rate(int32_t device, double* lane_ops_per_s)
{
    if (!lane_ops_per_s) return HOMS_E_INVALID;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return HOMS_E_INVALID;
    hipDeviceProp_t prop;
    homs_status st = HOMS_OK;
    uint32_t* out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    do {
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) { st = HOMS_E_DEVICE; break; }
        const int blocks = prop.multiProcessorCount * 16;
        const int iters = 4096;
        if (homs::dev_malloc(&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) {
            st = HOMS_E_OOM;
            break;
        }
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            st = HOMS_E_DEVICE;
            break;
        }
        homs::xor_popcount_rate_kernel<<<blocks, 256>>>(out, 1u, 64);  // warm-up
        float best = 1e30f;
        for (int rep = 0; rep < 3 && st == HOMS_OK; ++rep) {
            if (hipEventRecord(a, nullptr) != hipSuccess) st = HOMS_E_DEVICE;
            homs::xor_popcount_rate_kernel<<<blocks, 256>>>(out, 1u, iters);
            if (hipEventRecord(b, nullptr) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
                st = HOMS_E_DEVICE;
            float ms = 0.f;
            if (st == HOMS_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess) st = HOMS_E_DEVICE;
            if (ms > 0.f && ms < best) best = ms;
        }
        if (st != HOMS_OK) break;
        const double ops = (double)blocks * 256.0 * iters * homs::kChains * 2.0;
        *lane_ops_per_s = ops / (best * 1e-3);
    } while (0);
    if (out) (void)hipFree(out);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
}
