// sw_probe.hip -- VALU issue-rate probe for gfx950: the instruction rates the
// sweep's roofline assumes (packed 16-bit add, packed three-way maximum,
// 32-bit three-way maximum, 32-bit add), measured with HIP events on a grid
// that fills the device.  Used to confirm the peak the roofline divides by.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swprobe.h"

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

constexpr int kChains = 8;   // independent dependency chains per thread

template <int KIND>
__device__ __forceinline__ uint32_t step(uint32_t x, uint32_t y, uint32_t z) {
    if constexpr (KIND == SW_PROBE_PK_ADD_U16) {
        return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, x) + __builtin_bit_cast(u16x2, y));
    } else if constexpr (KIND == SW_PROBE_PK_MAX3_F16) {
        const f16x2 a = __builtin_bit_cast(f16x2, x), b = __builtin_bit_cast(f16x2, y),
                    c = __builtin_bit_cast(f16x2, z);
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c));
    } else if constexpr (KIND == SW_PROBE_MAX3_U32) {
        const uint32_t m = x > y ? x : y;
        return m > z ? m : z;
    } else {
        return x + y;
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void probe_kernel(uint32_t* out, int iters, uint32_t seed) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[kChains];
    // positive normal half-precision patterns in both halves (0x0400..0x3BFF)
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (((t * 7u + k * 13u + seed) & 0x37FFu) + 0x400u) * 0x10001u;
    const uint32_t y = ((seed & 0x1Fu) + 0x400u) * 0x10001u;
    const uint32_t z = ((seed & 0x3Fu) + 0x401u) * 0x10001u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = step<KIND>(a[k], y, z);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc ^= a[k];
    out[t] = acc;
}

}  // namespace

extern "C" int sw_probe_valu(int device, int kind, int iters, int blocks, double* instr_per_s) {
    if (!instr_per_s || iters < 1 || blocks < 1 || kind < 0 || kind > 3) return -1;
    if (hipSetDevice(device) != hipSuccess) return -4;
    uint32_t* out = nullptr;
    const size_t threads = (size_t)blocks * 256;
    if (hipMalloc(&out, threads * 4) != hipSuccess) return -2;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {   // the first launch warms up
        (void)hipEventRecord(e0, nullptr);
        switch (kind) {
            case SW_PROBE_PK_ADD_U16: hipLaunchKernelGGL(probe_kernel<SW_PROBE_PK_ADD_U16>, dim3(blocks), dim3(256), 0, nullptr, out, iters, 7u); break;
            case SW_PROBE_PK_MAX3_F16: hipLaunchKernelGGL(probe_kernel<SW_PROBE_PK_MAX3_F16>, dim3(blocks), dim3(256), 0, nullptr, out, iters, 7u); break;
            case SW_PROBE_MAX3_U32: hipLaunchKernelGGL(probe_kernel<SW_PROBE_MAX3_U32>, dim3(blocks), dim3(256), 0, nullptr, out, iters, 7u); break;
            default: hipLaunchKernelGGL(probe_kernel<SW_PROBE_ADD_U32>, dim3(blocks), dim3(256), 0, nullptr, out, iters, 7u); break;
        }
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    const hipError_t err = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (err != hipSuccess || ms <= 0.f) return -4;
    // one instruction per chain step per thread; a 64-lane wavefront
    // instruction counts as 64 lane-instructions
    *instr_per_s = (double)threads * (double)iters * kChains / (ms / 1e3);
    return 0;
}
