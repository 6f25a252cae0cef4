// Measurement helpers for the matrix cores the fused product runs on:
//  - the sustained MFMA rate of the device on its own (operands in
//    registers, no memory traffic), the ceiling the fused kernel is compared
//    with besides the vendor peak;
//  - one MFMA instruction on chosen inputs, to read off how the matrix
//    cores sum their products into the accumulator (the reason the fused
//    kernel never adds small split products to a sum that holds large ones).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sdc_internal.h"

namespace sdc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kPeakAcc = 4;    // independent accumulators per wave
constexpr int kPeakOps = 4;    // operand sets cycled through (data that toggles)

__device__ inline uint32_t rand_bits(uint32_t lane, uint32_t k, uint64_t seed) {
    uint32_t c[4] = {lane, k, 0x51u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return c[0];
}

// Two 16-bit floats in [-1, 1) from random bits (bf16 or f16 layout), or the
// constant 0.5 for both.
template <int FORM>
__device__ inline uint32_t pair_bits(uint32_t r, int random) {
    const uint32_t one_half = FORM == SDC_MFMA_BF16 ? 0x3F00u : 0x3800u;
    if (!random) return one_half | (one_half << 16);
    uint32_t out = 0;
    for (int h = 0; h < 2; ++h) {
        const uint32_t b = (r >> (16 * h)) & 0xFFFFu;
        uint32_t v;
        if (FORM == SDC_MFMA_BF16) v = (b & 0x807Fu) | (((b >> 7) % 8u + 119u) << 7);  // |v| in [2^-8, 1)
        else v = (b & 0x83FFu) | (((b >> 10) % 8u + 7u) << 10);                        // |v| in [2^-8, 1)
        out |= v << (16 * h);
    }
    return out;
}

template <int FORM>
__global__ __launch_bounds__(256, 2) void mfma_peak_kernel(int64_t iters, int random, uint64_t seed,
                                                           float* __restrict__ sink) {
    const uint32_t gl = blockIdx.x * blockDim.x + threadIdx.x;
    f32x16 acc[kPeakAcc];
#pragma unroll
    for (int k = 0; k < kPeakAcc; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.0f;
    if constexpr (FORM == SDC_MFMA_F32) {
        float a[kPeakOps], b[kPeakOps];
#pragma unroll
        for (int s = 0; s < kPeakOps; ++s) {
            const uint32_t r0 = rand_bits(gl, 2 * s, seed), r1 = rand_bits(gl, 2 * s + 1, seed);
            a[s] = random ? (float)(int32_t)r0 * 0x1p-31f : 0.5f;
            b[s] = random ? (float)(int32_t)r1 * 0x1p-31f : 0.5f;
        }
        for (int64_t it = 0; it < iters; ++it)
#pragma unroll
            for (int s = 0; s < kPeakOps; ++s)
#pragma unroll
                for (int k = 0; k < kPeakAcc; ++k)
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[(s + k) % kPeakOps], acc[k], 0, 0, 0);
    } else {
        uint4 a[kPeakOps], b[kPeakOps];
#pragma unroll
        for (int s = 0; s < kPeakOps; ++s) {
            uint32_t w[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = pair_bits<FORM>(rand_bits(gl, 8 * s + e, seed), random);
            a[s] = make_uint4(w[0], w[1], w[2], w[3]);
            b[s] = make_uint4(w[4], w[5], w[6], w[7]);
        }
        for (int64_t it = 0; it < iters; ++it)
#pragma unroll
            for (int s = 0; s < kPeakOps; ++s)
#pragma unroll
                for (int k = 0; k < kPeakAcc; ++k) {
                    if constexpr (FORM == SDC_MFMA_BF16)
                        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[s]),
                                                                         __builtin_bit_cast(bf16x8, b[(s + k) % kPeakOps]),
                                                                         acc[k], 0, 0, 0);
                    else
                        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[s]),
                                                                        __builtin_bit_cast(f16x8, b[(s + k) % kPeakOps]),
                                                                        acc[k], 0, 0, 0);
                }
    }
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < kPeakAcc; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) t += acc[k][r];
    sink[gl] = t;  // keeps the products alive
}

// One MFMA of the chosen form on one wave: element (0, 0) of the 32x32
// output gets c plus the products a[k] b[k] (k = 0..n-1: lane (0, h) holds
// k = 8h .. 8h + 7 of row 0 and column 0 for the 16-bit forms; lanes 0 and
// 32 hold k = 0 and 1 for the FP32 form); every other input is zero.
__global__ void mfma_probe_kernel(int form, float c, const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                  float* __restrict__ out) {
    const int lane = threadIdx.x;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    if (lane == 0) acc[0] = c;
    const uint4 av = make_uint4(a[4 * lane], a[4 * lane + 1], a[4 * lane + 2], a[4 * lane + 3]);
    const uint4 bv = make_uint4(b[4 * lane], b[4 * lane + 1], b[4 * lane + 2], b[4 * lane + 3]);
    if (form == SDC_MFMA_BF16)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                      acc, 0, 0, 0);
    else if (form == SDC_MFMA_F16)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av), __builtin_bit_cast(f16x8, bv),
                                                     acc, 0, 0, 0);
    else
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(av.x), __uint_as_float(bv.x), acc, 0, 0, 0);
    if (lane == 0) out[0] = acc[0];
}

bool exact16(float x, int form, uint16_t* bits) {
    if (form == SDC_MFMA_BF16) {
        uint32_t u;
        std::memcpy(&u, &x, 4);
        if (u & 0xFFFFu) return false;
        *bits = (uint16_t)(u >> 16);
        return true;
    }
    const _Float16 h = (_Float16)x;
    if ((float)h != x) return false;
    std::memcpy(bits, &h, 2);
    return true;
}

}  // namespace
}  // namespace sdc

extern "C" {

sdc_status sdc_mfma_peak(int32_t form, int32_t random_operands, int64_t iterations, int32_t workgroups_per_cu,
                         int device, double* ms, double* tflops) {
    if (!ms || !tflops) return sdc::set_error(SDC_ERR_INVALID_ARG, "null output");
    if (form < SDC_MFMA_BF16 || form > SDC_MFMA_F32) return sdc::set_error(SDC_ERR_INVALID_ARG, "unknown form");
    if (iterations < 1 || iterations > ((int64_t)1 << 32))
        return sdc::set_error(SDC_ERR_INVALID_ARG, "iterations must be in [1, 2^32]");
    if (workgroups_per_cu < 1 || workgroups_per_cu > 2)
        return sdc::set_error(SDC_ERR_INVALID_ARG, "workgroups_per_cu must be 1 or 2");
    if (hipSetDevice(device) != hipSuccess) return sdc::set_error(SDC_ERR_NO_DEVICE, "hipSetDevice failed");
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return sdc::set_error(SDC_ERR_HIP, "device attribute");
    const int grid = n_cu * workgroups_per_cu;
    float* sink = nullptr;
    if (hipMalloc((void**)&sink, (size_t)grid * 256 * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return sdc::set_error(SDC_ERR_OOM, "hipMalloc failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const uint64_t seed = 0x5DC0F1A5ull;
    auto launch = [&](int64_t it) {
        if (form == SDC_MFMA_BF16)
            hipLaunchKernelGGL(sdc::mfma_peak_kernel<SDC_MFMA_BF16>, dim3(grid), dim3(256), 0, 0, it, random_operands,
                               seed, sink);
        else if (form == SDC_MFMA_F16)
            hipLaunchKernelGGL(sdc::mfma_peak_kernel<SDC_MFMA_F16>, dim3(grid), dim3(256), 0, 0, it, random_operands,
                               seed, sink);
        else
            hipLaunchKernelGGL(sdc::mfma_peak_kernel<SDC_MFMA_F32>, dim3(grid), dim3(256), 0, 0, it, random_operands,
                               seed, sink);
        return hipGetLastError();
    };
    if (he == hipSuccess) he = launch(std::min<int64_t>(iterations, 64));  // warm-up
    if (he == hipSuccess) he = hipEventRecord(e0, 0);
    if (he == hipSuccess) he = launch(iterations);
    if (he == hipSuccess) he = hipEventRecord(e1, 0);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (he != hipSuccess) return sdc::set_error(SDC_ERR_HIP, std::string("MFMA rate kernel: ") + hipGetErrorString(he));
    const double per_mfma = form == SDC_MFMA_F32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
    const double flops = per_mfma * (double)grid * 4 /* waves */ * (double)iterations * sdc::kPeakOps * sdc::kPeakAcc;
    *ms = t;
    *tflops = flops / (t * 1e-3) / 1e12;
    sdc::set_error(SDC_OK, "");
    return SDC_OK;
}

sdc_status sdc_mfma_probe(int32_t form, float c, const float* a, const float* b, int32_t n_products, int device,
                          float* out) {
    if (!a || !b || !out) return sdc::set_error(SDC_ERR_INVALID_ARG, "null pointer");
    if (form < SDC_MFMA_BF16 || form > SDC_MFMA_F32) return sdc::set_error(SDC_ERR_INVALID_ARG, "unknown form");
    const int kmax = form == SDC_MFMA_F32 ? 2 : 16;
    if (n_products < 0 || n_products > kmax) return sdc::set_error(SDC_ERR_INVALID_ARG, "too many products");
    std::vector<uint32_t> ha(64 * 4, 0u), hb(64 * 4, 0u);
    for (int k = 0; k < n_products; ++k) {
        if (form == SDC_MFMA_F32) {
            uint32_t ua, ub;
            std::memcpy(&ua, &a[k], 4);
            std::memcpy(&ub, &b[k], 4);
            ha[4 * (32 * k)] = ua;
            hb[4 * (32 * k)] = ub;
        } else {
            uint16_t xa, xb;
            if (!sdc::exact16(a[k], form, &xa) || !sdc::exact16(b[k], form, &xb))
                return sdc::set_error(SDC_ERR_INVALID_ARG, "an operand is not exact in the form's 16-bit type");
            const int lane = 32 * (k / 8), e = k % 8;
            uint32_t* wa = &ha[4 * lane + e / 2];
            uint32_t* wb = &hb[4 * lane + e / 2];
            *wa |= (uint32_t)xa << (16 * (e % 2));
            *wb |= (uint32_t)xb << (16 * (e % 2));
        }
    }
    if (hipSetDevice(device) != hipSuccess) return sdc::set_error(SDC_ERR_NO_DEVICE, "hipSetDevice failed");
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, (2 * 64 * 4 + 1) * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return sdc::set_error(SDC_ERR_OOM, "hipMalloc failed");
    }
    hipError_t he = hipMemcpy(d, ha.data(), 64 * 4 * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(d + 64 * 4, hb.data(), 64 * 4 * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (he == hipSuccess) {
        hipLaunchKernelGGL(sdc::mfma_probe_kernel, dim3(1), dim3(64), 0, 0, (int)form, c, d, d + 64 * 4,
                           (float*)(d + 2 * 64 * 4));
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipMemcpy(out, d + 2 * 64 * 4, sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (he != hipSuccess) return sdc::set_error(SDC_ERR_HIP, std::string("MFMA probe: ") + hipGetErrorString(he));
    sdc::set_error(SDC_OK, "");
    return SDC_OK;
}

}  // extern "C"
