// Learned estimator for VATE on MI355X: a 64 -> 64 -> 64 -> 1 GELU network
// that maps a host's sketch features (distance histogram, live fraction, pool
// occupancy) to the log of its window cardinality, on top of the log of the
// closed-form estimate (a fixed residual branch).  Hand-written training and
// inference kernels on gfx950's BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16: 16x32 by 32x16 tiles, FP32 accumulate).
//
// Numerics (mirrored by the CPU oracle): BF16 round-to-nearest-even of the
// features, W1, W2, a1 = GELU(z1), a2 = GELU(z2), and of the pre-activation
// gradients dz2, dz1 before the products that consume them; every sum, bias,
// GELU, the output layer and Adam in FP32.
//
// Tile organisation: a workgroup of 4 wavefronts owns 64 samples, each
// wavefront 16 of them.  Forward layers are (16 x 64) x (64 x 64) products per
// wavefront; the weight gradients are (64 x 64 samples) x (64 samples x 64)
// products per workgroup, one 16-row slab per wavefront, accumulated across
// workgroups with FP32 atomics.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vate.h"
#include "vate_mlp.h"
#include "mlp_core.h"

namespace vate {
namespace mlp {

// ---------------------------------------------------------------------------
// Pack FP32 parameters into the inference layout.
// ---------------------------------------------------------------------------
__global__ void k_pack(const float *__restrict__ theta, Packed *__restrict__ P)
{
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < HD * F; i += blockDim.x * gridDim.x) {
        P->W1b[i] = bf16_bits(theta[OFF_W1 + i]);
        const int n = i / HD, k = i % HD;
        const uint16_t w2 = bf16_bits(theta[OFF_W2 + i]);
        P->W2b[i] = w2;
        P->W2bT[k * HD + n] = w2;
    }
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < HD; i += blockDim.x) {
            P->b1[i] = theta[OFF_B1 + i];
            P->b2[i] = theta[OFF_B2 + i];
            P->w3[i] = theta[OFF_W3 + i];
        }
        if (threadIdx.x == 0) {
            P->b3 = theta[OFF_B3];
            P->env.magic = 0;         // packing switches the envelope off
        }
        for (int i = threadIdx.x; i < kFallbackSlots; i += blockDim.x) P->fallbacks[i] = 0;
    }
}

// Load 16 feature rows of this wavefront into LDS (zero beyond n).
__device__ __forceinline__ void stage_rows(const uint16_t *__restrict__ X, uint64_t row0, uint64_t n, uint16_t *xs)
{
    const int l = threadIdx.x & 63;
    // 16 rows x 64 bf16 = 16 x 8 uint4; 64 lanes take two each
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int idx = l + 64 * t, m = idx >> 3, part = idx & 7;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row0 + m < n) v = reinterpret_cast<const uint4 *>(X + (row0 + m) * F)[part];
        *reinterpret_cast<uint4 *>(xs + m * LDS_STRIDE + part * 8) = v;
    }
}

// ---------------------------------------------------------------------------
// Inference over a feature matrix: o[i] = network(x_i) + r[i].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_forward(const Packed *__restrict__ P, const uint16_t *__restrict__ X,
                                                 const float *__restrict__ R, uint64_t n, float *__restrict__ O)
{
    __shared__ __attribute__((aligned(16))) uint16_t xs_all[4][16 * LDS_STRIDE];
    __shared__ __attribute__((aligned(16))) uint16_t a1_all[4][16 * LDS_STRIDE];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const uint64_t row0 = (uint64_t)blockIdx.x * 64 + 16 * w;
    stage_rows(X, row0, n, xs_all[w]);
    __syncthreads();
    float r4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) r4[r] = row0 + 4 * q + r < n ? R[row0 + 4 * q + r] : 0.f;
    f32x4 z1[4], z2[4];
    float a2v[4][4], o4[4];
    forward16(P, xs_all[w], a1_all[w], r4, z1, z2, a2v, o4);
    if (c < 4 && row0 + 4 * q + c < n) O[row0 + 4 * q + c] = o4[c];
}

// ---------------------------------------------------------------------------
// One training pass over a minibatch: forward, loss gradient, backward; the
// parameter gradient (FP32, VATE_MLP_PARAMS entries, caller-zeroed) and the
// loss sum are accumulated with atomics.  Loss = mean |exp(o - y) - 1|.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_train(const Packed *__restrict__ P, const uint16_t *__restrict__ X,
                                               const float *__restrict__ R, const float *__restrict__ Y,
                                               uint64_t n, float inv_batch, float *__restrict__ grad,
                                               float *__restrict__ loss)
{
    __shared__ __attribute__((aligned(16))) uint16_t xs[64 * LDS_STRIDE];    // [sample][feature]
    __shared__ __attribute__((aligned(16))) uint16_t xT[64 * LDS_STRIDE];    // [feature][sample]
    __shared__ __attribute__((aligned(16))) uint16_t a1s[64 * LDS_STRIDE];   // [sample][unit]
    __shared__ __attribute__((aligned(16))) uint16_t a1T[64 * LDS_STRIDE];   // [unit][sample]
    __shared__ __attribute__((aligned(16))) uint16_t dz2s[64 * LDS_STRIDE];  // [sample][unit]
    __shared__ __attribute__((aligned(16))) uint16_t dz2T[64 * LDS_STRIDE];  // [unit][sample]
    __shared__ __attribute__((aligned(16))) uint16_t dz1T[64 * LDS_STRIDE];  // [unit][sample]
    __shared__ float gsmall[3 * HD + 1];                                      // db1, db2, dw3, db3
    __shared__ float lsum;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const uint64_t blk0 = (uint64_t)blockIdx.x * 64, row0 = blk0 + 16 * w;
    for (int i = threadIdx.x; i < 3 * HD + 1; i += blockDim.x) gsmall[i] = 0.f;
    if (threadIdx.x == 0) lsum = 0.f;
    uint16_t *xw = xs + 16 * w * LDS_STRIDE;
    stage_rows(X, row0, n, xw);
    __syncthreads();
    // transposed copy of the features for the W1 gradient
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        const int m = i >> 6, f = i & 63;
        xT[f * LDS_STRIDE + m] = xs[m * LDS_STRIDE + f];
    }
    float r4[4], y4[4];
    bool v4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t row = row0 + 4 * q + r;
        v4[r] = row < n;
        r4[r] = v4[r] ? R[row] : 0.f;
        y4[r] = v4[r] ? Y[row] : 0.f;
    }
    f32x4 z1[4], z2[4];
    float a2v[4][4], o4[4];
    forward16(P, xw, a1s + 16 * w * LDS_STRIDE, r4, z1, z2, a2v, o4);

    // loss gradient
    float do4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float e = expf(o4[r] - y4[r]);
        const float d = e - 1.0f;
        do4[r] = v4[r] ? (d > 0.f ? e : (d < 0.f ? -e : 0.f)) * inv_batch : 0.f;
        if (v4[r] && c == 0) atomicAdd(&lsum, fabsf(d));
    }
    // output layer gradients, dz2
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = 16 * nt + c;
        float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            gw3 += do4[r] * a2v[nt][r];
            const float dz = do4[r] * P->w3[n] * gelu_grad(z2[nt][r]);
            gb2 += dz;
            const uint16_t b = bf16_bits(dz);
            const int m = 16 * w + 4 * q + r;
            dz2s[m * LDS_STRIDE + n] = b;
            dz2T[n * LDS_STRIDE + m] = b;
        }
        atomicAdd(&gsmall[2 * HD + n], gw3);
        atomicAdd(&gsmall[HD + n], gb2);
    }
    if (c == 0) {
        float s = do4[0] + do4[1] + do4[2] + do4[3];
        atomicAdd(&gsmall[3 * HD], s);
    }
    // a1 transposed for the W2 gradient
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        const int m = i >> 6, k = i & 63;
        a1T[k * LDS_STRIDE + m] = a1s[m * LDS_STRIDE + k];
    }
    __syncthreads();
    // dW2[n][k] = sum_m dz2[m][n] a1[m][k]: rows n of this wavefront's slab
    {
        f32x4 acc[4];
        gemm16x64([&](int i) { return dz2T + (16 * w + i) * LDS_STRIDE; },
                  [&](int j) { return a1T + j * LDS_STRIDE; }, acc);
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                atomicAdd(&grad[OFF_W2 + (16 * w + 4 * q + r) * HD + 16 * jt + c], acc[jt][r]);
    }
    // da1 = dz2 W2 (this wavefront's 16 samples), dz1 = da1 * gelu'(z1)
    {
        f32x4 acc[4];
        gemm16x64([&](int m) { return dz2s + (16 * w + m) * LDS_STRIDE; },
                  [&](int k) { return P->W2bT + k * HD; }, acc);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int k = 16 * kt + c;
            float gb1 = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dz = acc[kt][r] * gelu_grad(z1[kt][r]);
                gb1 += dz;
                dz1T[k * LDS_STRIDE + 16 * w + 4 * q + r] = bf16_bits(dz);
            }
            atomicAdd(&gsmall[k], gb1);
        }
    }
    __syncthreads();
    // dW1[j][f] = sum_m dz1[m][j] x[m][f]
    {
        f32x4 acc[4];
        gemm16x64([&](int i) { return dz1T + (16 * w + i) * LDS_STRIDE; },
                  [&](int f) { return xT + f * LDS_STRIDE; }, acc);
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                atomicAdd(&grad[OFF_W1 + (16 * w + 4 * q + r) * F + 16 * ft + c], acc[ft][r]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HD; i += blockDim.x) {
        atomicAdd(&grad[OFF_B1 + i], gsmall[i]);
        atomicAdd(&grad[OFF_B2 + i], gsmall[HD + i]);
        atomicAdd(&grad[OFF_W3 + i], gsmall[2 * HD + i]);
    }
    if (threadIdx.x == 0) {
        atomicAdd(&grad[OFF_B3], gsmall[3 * HD]);
        atomicAdd(loss, lsum * inv_batch);
    }
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba), bias-corrected, on FP32 parameters.
// ---------------------------------------------------------------------------
__global__ void k_adam(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int count, float lr, float beta1, float beta2, float eps,
                       float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Features of one host per thread from vate_estimate's histogram output.
__global__ void k_features(const uint32_t *__restrict__ hist, const float *__restrict__ est, uint64_t n,
                           uint32_t k, uint32_t g, float occupancy, uint16_t *__restrict__ X,
                           float *__restrict__ R)
{
    const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    const uint32_t *row = hist + h * (k + 1);
    const float fg = (float)g;
    uint32_t live = 0;
    uint16_t out[F];
    for (int f = 0; f < F; ++f) out[f] = 0;
    for (uint32_t d = 0; d < k; ++d) {
        live += row[d];
        out[d] = bf16_bits((float)row[d] / fg);
    }
    out[k] = bf16_bits((float)live / fg);
    out[k + 1] = bf16_bits(occupancy);
    const float r = logf(fmaxf(est[h], 1.0f));
    out[k + 2] = bf16_bits(r * 0.0625f);
    uint4 *dst = reinterpret_cast<uint4 *>(X + h * F);
    for (int j = 0; j < F / 8; ++j) {
        uint32_t wv[4];
        for (int t = 0; t < 4; ++t) wv[t] = (uint32_t)out[8 * j + 2 * t] | ((uint32_t)out[8 * j + 2 * t + 1] << 16);
        dst[j] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    }
    R[h] = r;
}

__global__ void k_fill(float *__restrict__ p, int count, float value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// Layout self-check of the matrix-core fragments: D = A * B for one 16x32 by
// 32x16 tile, with A and B row-major bf16 and D row-major FP32.
__global__ void k_mfma_selftest(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                float *__restrict__ D)
{
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    uint32_t bw[4];
    for (int j = 0; j < 4; ++j)
        bw[j] = (uint32_t)B[(8 * q + 2 * j) * 16 + c] | ((uint32_t)B[(8 * q + 2 * j + 1) * 16 + c] << 16);
    const bf16x8 a = as_bf16x8(*reinterpret_cast<const uint4 *>(A + c * 32 + 8 * q));
    const bf16x8 b = as_bf16x8(make_uint4(bw[0], bw[1], bw[2], bw[3]));
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
    d = mfma(a, b, d);
    for (int r = 0; r < 4; ++r) D[(4 * q + r) * 16 + c] = d[r];
}

}  // namespace mlp
}  // namespace vate

using namespace vate::mlp;

static int mlp_check(const char *what)
{
    (void)what;
    return hipGetLastError() == hipSuccess ? VATE_OK : VATE_E_DEVICE;
}

extern "C" {

int vate_mlp_pack(const float *theta_dev, void *weights_dev, void *stream)
{
    if (!theta_dev || !weights_dev || (reinterpret_cast<uintptr_t>(weights_dev) & 255u)) return VATE_E_INVAL;
    k_pack<<<16, 256, 0, static_cast<hipStream_t>(stream)>>>(theta_dev, static_cast<Packed *>(weights_dev));
    return mlp_check("pack");
}

int vate_mlp_set_envelope(void *weights_dev, const vate_mlp_envelope *env, void *stream)
{
    if (!weights_dev || (reinterpret_cast<uintptr_t>(weights_dev) & 255u)) return VATE_E_INVAL;
    Envelope e{};
    if (env) {
        for (int f = 0; f < F; ++f)
            if (!(env->lo[f] <= env->hi[f])) return VATE_E_INVAL;
        e.magic = kEnvMagic;
        e.k = env->k;
        e.g = env->g;
        e.log2_pool = env->log2_pool;
        e.width = env->width;
        for (int f = 0; f < F; ++f) e.lo[f] = env->lo[f], e.hi[f] = env->hi[f];
    }
    Packed *P = static_cast<Packed *>(weights_dev);
    const unsigned long long zero[kFallbackSlots] = {};
    hipError_t err = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (err == hipSuccess) err = hipMemcpy(&P->env, &e, sizeof(Envelope), hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(P->fallbacks, zero, sizeof(zero), hipMemcpyHostToDevice);
    return err == hipSuccess ? VATE_OK : VATE_E_DEVICE;
}

int vate_mlp_fallbacks(const void *weights_dev, uint64_t *count, int reset, void *stream)
{
    if (!weights_dev || !count || (reinterpret_cast<uintptr_t>(weights_dev) & 255u)) return VATE_E_INVAL;
    const Packed *P = static_cast<const Packed *>(weights_dev);
    unsigned long long c[kFallbackSlots] = {};
    hipError_t err = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (err == hipSuccess) err = hipMemcpy(c, P->fallbacks, sizeof(c), hipMemcpyDeviceToHost);
    if (err == hipSuccess && reset) {
        const unsigned long long zero[kFallbackSlots] = {};
        err = hipMemcpy(const_cast<unsigned long long *>(P->fallbacks), zero, sizeof(zero), hipMemcpyHostToDevice);
    }
    if (err != hipSuccess) return VATE_E_DEVICE;
    uint64_t sum = 0;
    for (int i = 0; i < kFallbackSlots; ++i) sum += c[i];
    *count = sum;
    return VATE_OK;
}

int vate_mlp_forward(const void *weights_dev, const uint16_t *x_dev, const float *r_dev, size_t n, float *o_dev,
                     void *stream)
{
    if (n == 0) return VATE_OK;
    if (!weights_dev || !x_dev || !r_dev || !o_dev || (reinterpret_cast<uintptr_t>(x_dev) & 15u))
        return VATE_E_INVAL;
    const uint64_t blocks = (n + 63) / 64;
    if (blocks > 0x7FFFFFFFull) return VATE_E_INVAL;
    k_forward<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const Packed *>(weights_dev), x_dev, r_dev, n, o_dev);
    return mlp_check("forward");
}

int vate_mlp_train_step(const void *weights_dev, const uint16_t *x_dev, const float *r_dev, const float *y_dev,
                        size_t n, float *grad_dev, float *loss_dev, void *stream)
{
    if (n == 0) return VATE_OK;
    if (!weights_dev || !x_dev || !r_dev || !y_dev || !grad_dev || !loss_dev ||
        (reinterpret_cast<uintptr_t>(x_dev) & 15u))
        return VATE_E_INVAL;
    const uint64_t blocks = (n + 63) / 64;
    if (blocks > 0x7FFFFFFFull) return VATE_E_INVAL;
    k_train<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const Packed *>(weights_dev), x_dev, r_dev, y_dev, n, 1.0f / (float)n, grad_dev, loss_dev);
    return mlp_check("train");
}

int vate_mlp_adam(float *theta_dev, const float *grad_dev, float *m_dev, float *v_dev, uint32_t step, float lr,
                  float beta1, float beta2, float eps, void *stream)
{
    if (!theta_dev || !grad_dev || !m_dev || !v_dev || step < 1) return VATE_E_INVAL;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    k_adam<<<(VATE_MLP_PARAMS + 255) / 256, 256, 0, static_cast<hipStream_t>(stream)>>>(
        theta_dev, grad_dev, m_dev, v_dev, VATE_MLP_PARAMS, lr, beta1, beta2, eps, c1, c2);
    return mlp_check("adam");
}

int vate_mlp_fill(float *dst_dev, size_t count, float value, void *stream)
{
    if (!dst_dev || count > 0x7FFFFFFFull) return VATE_E_INVAL;
    if (count == 0) return VATE_OK;
    k_fill<<<(unsigned)((count + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(dst_dev, (int)count,
                                                                                            value);
    return mlp_check("fill");
}

int vate_mlp_features(const uint32_t *hist_dev, const float *est_dev, size_t n, uint32_t k, uint32_t g,
                      float pool_active_fraction, uint16_t *x_dev, float *r_dev, void *stream)
{
    if (n == 0) return VATE_OK;
    if (k < 1 || k + 3 > (uint32_t)F) return VATE_E_UNSUPPORTED;
    if (!hist_dev || !est_dev || !x_dev || !r_dev || g < 1 || (reinterpret_cast<uintptr_t>(x_dev) & 15u))
        return VATE_E_INVAL;
    const uint64_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return VATE_E_INVAL;
    k_features<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(
        hist_dev, est_dev, n, k, g, pool_active_fraction, x_dev, r_dev);
    return mlp_check("features");
}

int vate_mlp_mfma_selftest(const uint16_t *a_dev, const uint16_t *b_dev, float *d_dev, void *stream)
{
    if (!a_dev || !b_dev || !d_dev || (reinterpret_cast<uintptr_t>(a_dev) & 15u)) return VATE_E_INVAL;
    k_mfma_selftest<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(a_dev, b_dev, d_dev);
    return mlp_check("selftest");
}

}  // extern "C"
