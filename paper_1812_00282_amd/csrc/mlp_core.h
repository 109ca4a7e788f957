// Device-side building blocks of the learned VATE estimator shared by the
// training/inference kernels (mlp.hip) and the fused estimate (vate.hip):
// parameter layout, BF16 rounding, GELU, the gfx950 BF16 matrix-core tile
// (v_mfma_f32_16x16x32_bf16) and the per-wavefront forward pass.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vate_mlp.h"

namespace vate {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int F = VATE_MLP_FEATURES;   // 64
constexpr int HD = VATE_MLP_HIDDEN;    // 64
constexpr int LDS_STRIDE = 72;         // bf16 per LDS row (64 + 8 pad)

// Offsets into the flat FP32 parameter vector theta.
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + HD * F;
constexpr int OFF_W2 = OFF_B1 + HD;
constexpr int OFF_B2 = OFF_W2 + HD * HD;
constexpr int OFF_W3 = OFF_B2 + HD;
constexpr int OFF_B3 = OFF_W3 + HD;
static_assert(OFF_B3 + 1 == VATE_MLP_PARAMS, "parameter count");

// The network's training envelope (vate_mlp_envelope) as kept with the
// packed weights.
constexpr uint32_t kEnvMagic = 0x31564E45u;   // set by vate_mlp_set_envelope; anything else: no envelope
struct Envelope {
    uint32_t magic;
    uint32_t k, g, log2_pool, width;
    uint32_t pad[3];
    unsigned long long pad1[2];
    float lo[F], hi[F];
};

// Hosts the envelope sent to the closed form, counted in kFallbackSlots
// counters (a workgroup adds its count to slot blockIdx mod kFallbackSlots,
// so that no counter takes an atomic from every workgroup); the reader sums
// them.
constexpr int kFallbackSlots = 16;

// Packed inference weights (bytes).
struct Packed {
    uint16_t W1b[HD * F];     // bf16, row = hidden unit, col = input
    uint16_t W2b[HD * HD];    // bf16, row = layer-2 unit, col = layer-1 unit
    uint16_t W2bT[HD * HD];   // transpose of W2b
    float b1[HD], b2[HD], w3[HD], b3;
    float pad[63];
    Envelope env;
    unsigned long long fallbacks[kFallbackSlots];
    float pad3[20];
};
static_assert(sizeof(Packed) == VATE_MLP_WEIGHT_BYTES, "packed weight size");

// Whether an envelope is set, and whether it rules the network out for the
// whole sketch (another geometry).
__device__ __forceinline__ bool env_on(const Packed *P) { return P->env.magic == kEnvMagic; }

__device__ __forceinline__ bool env_geometry_off(const Packed *P, uint32_t k, uint32_t g, uint32_t c, uint32_t w)
{
    return env_on(P) && (P->env.k != k || P->env.g != g || P->env.log2_pool != c || P->env.width != w);
}

// The range of feature f ([-inf, inf] without an envelope), read once per
// lane, and whether a feature's BF16 bits xb lie outside it.
struct EnvRange {
    float lo, hi;
};

__device__ __forceinline__ EnvRange env_range(const Packed *P, int f)
{
    if (!env_on(P)) return {-INFINITY, INFINITY};
    return {P->env.lo[f], P->env.hi[f]};
}

__device__ __forceinline__ bool env_outside(const EnvRange &r, uint16_t xb)
{
    const float x = __uint_as_float((uint32_t)xb << 16);
    return !(x >= r.lo && x <= r.hi);
}

// Adds a workgroup's n fallback hosts to its slot (one lane per workgroup).
__device__ __forceinline__ void env_count(const Packed *P, uint32_t n)
{
    if (n) atomicAdd(&const_cast<Packed *>(P)->fallbacks[blockIdx.x % kFallbackSlots], (unsigned long long)n);
}

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_float(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

// erf by the rational approximation of Abramowitz & Stegun 7.1.26 (after
// Hastings): erf(a) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-a^2)
// with t = 1 / (1 + p a) for a >= 0, absolute error at most 1.5e-7, odd in
// x.  Branch-free, with one hardware reciprocal and one hardware 2^x (each
// within 1 ulp); far below the BF16 rounding that follows it.
__device__ __forceinline__ float erf_as(float x)
{
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-(a * a) * 1.4426950408889634f);   // e^(-a^2)
    return copysignf(fmaf(-poly, e, 1.0f), x);
}

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Fragment conventions of v_mfma_f32_16x16x32_bf16 for lane l, q = l / 16:
//   A (16 x 32): row l % 16, columns 8q .. 8q+7
//   B (32 x 16): rows 8q .. 8q+7, column l % 16
//   D (16 x 16): rows 4q .. 4q+3 (element r), column l % 16
// so an A or B fragment is 8 consecutive bf16 of one row of a row-major
// operand whose rows are the fragment's m (for A) or n (for B).  K = 64 takes
// two steps s = 0, 1 at column offset 32 s.
__device__ __forceinline__ bf16x8 frag(const uint16_t *row, int s, int q)
{
    return as_bf16x8(*reinterpret_cast<const uint4 *>(row + 32 * s + 8 * q));
}

// out[16 x 64] (4 D tiles) = A[16 x 64] * Bt[64 x 64]^T, where A's row m is
// arow(m) and Bt's row n (the B column n) is brow(n).
template <class RowA, class RowB>
__device__ __forceinline__ void gemm16x64(RowA arow, RowB brow, f32x4 acc[4])
{
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const bf16x8 a0 = frag(arow(c), 0, q), a1 = frag(arow(c), 1, q);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const uint16_t *br = brow(16 * nt + c);
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        d = mfma(a0, frag(br, 0, q), d);
        d = mfma(a1, frag(br, 1, q), d);
        acc[nt] = d;
    }
}

// Orders a wavefront's LDS writes before its later LDS reads (lanes of one
// wavefront; no other wavefront waits).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront forward pass over 16 samples whose bf16 features are rows of
// xs (16 rows, stride LDS_STRIDE).  Leaves z1, z2 (D layout), writes a1 rows
// into a1s (stride LDS_STRIDE) and returns o for rows 4q .. 4q+3 in o4.
// WG_SYNC: the layer-1 activations are published with a workgroup barrier
// (callers that then read other wavefronts' rows), else with a wavefront one.
template <bool WG_SYNC = true>
__device__ __forceinline__ void forward16(const Packed *__restrict__ P, const uint16_t *xs, uint16_t *a1s,
                                          const float r4[4], f32x4 z1[4], f32x4 z2[4], float a2v[4][4],
                                          float o4[4])
{
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    gemm16x64([&](int m) { return xs + m * LDS_STRIDE; }, [&](int n) { return P->W1b + n * F; }, z1);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = 16 * nt + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            z1[nt][r] += P->b1[n];
            a1s[(4 * q + r) * LDS_STRIDE + n] = bf16_bits(gelu(z1[nt][r]));
        }
    }
    if constexpr (WG_SYNC)
        __syncthreads();
    else
        wave_sync();
    gemm16x64([&](int m) { return a1s + m * LDS_STRIDE; }, [&](int n) { return P->W2b + n * HD; }, z2);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = 16 * nt + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            z2[nt][r] += P->b2[n];
            a2v[nt][r] = bf16_float(bf16_bits(gelu(z2[nt][r])));
            part[r] += a2v[nt][r] * P->w3[n];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) part[r] += __shfl_xor(part[r], off, 64);
        o4[r] = part[r] + P->b3 + r4[r];
    }
}

}  // namespace mlp
}  // namespace vate
