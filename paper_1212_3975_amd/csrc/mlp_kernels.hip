// HIP kernels of the learned initial weights: a 4 -> 64 -> 64 -> 64 -> 1 MLP
// with tanh-form GELU, BF16 weights and activations as matrix inputs, FP32
// accumulation, FP32 master weights and Adam.  The two 64 x 64 layers (and
// their backward products) run on MFMA 16x16x16 bf16 tiles; one wave owns a
// tile of 64 samples.
//
// Parameter vector (FP32 master copy, BF16 working copy), offsets in floats:
//   W1 [64][4] 0, b1 [64] 256, W2 [64][64] 320, b2 [64] 4416,
//   W3 [64][64] 4480, b3 [64] 8576, W4 [64] 8640, b4 [1] 8704; 8705 total.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_device.h"

namespace muca {

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

constexpr int H = 64;
constexpr int TILE = 64;   // samples per workgroup (one wave)

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu(float z, float *deriv) {
    const float c = 0.7978845608028654f;   // sqrt(2/pi)
    const float u = c * (z + 0.044715f * z * z * z);
    const float t = tanhf(u);
    *deriv = 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
    return 0.5f * z * (1.0f + t);
}

// C tile (16 x 16 at rows m0, cols n0) += A[m0.., k] * B[k, n0..] over k in [0, K).
// Accessors return BF16 bits.  MFMA 16x16x16 lane layout: lane l holds
// A[m0 + l%16][k0 + 4(l/16) + t] and B[k0 + 4(l/16) + t][n0 + l%16], t = 0..3;
// the result acc[j] is C[m0 + 4(l/16) + j][n0 + l%16].
template <class FA, class FB>
__device__ __forceinline__ v4f32 mfma_tile(FA a, FB b, int m0, int n0, int K, v4f32 acc) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kb = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4i16 av, bv;
        av.x = (short)a(m0 + r, k0 + 4 * kb + 0);
        av.y = (short)a(m0 + r, k0 + 4 * kb + 1);
        av.z = (short)a(m0 + r, k0 + 4 * kb + 2);
        av.w = (short)a(m0 + r, k0 + 4 * kb + 3);
        bv.x = (short)b(k0 + 4 * kb + 0, n0 + r);
        bv.y = (short)b(k0 + 4 * kb + 1, n0 + r);
        bv.z = (short)b(k0 + 4 * kb + 2, n0 + r);
        bv.w = (short)b(k0 + 4 * kb + 3, n0 + r);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// Forward pass of one 64-sample tile; stores what the backward pass needs.
//   x [n][4] fp32 inputs, t [n] targets (may be null when predicting)
//   outputs: y [n]; z1..z3 [n][64] fp32 pre-activations; a0 [n][4], a1..a3
//   [n][64] bf16 activations; dy [n] = 2 (y - t) / n; loss_part [tiles]
__global__ void __launch_bounds__(64) mlp_forward_kernel(MlpBuffers b, const float *x, const float *t, int n,
                                                         int train) {
    __shared__ uint16_t A[TILE][H + 2];   // current activation tile (bf16)
    __shared__ uint16_t Wt[H][H + 2];     // weight matrix W[out][in] (bf16)
    __shared__ float red[64];
    const int lane = threadIdx.x;
    const int s0 = blockIdx.x * TILE;
    const int s = s0 + lane;
    const bool valid = s < n;
    const uint16_t *P = b.pbf;

    // layer 1 (K = 4) on the vector units
    float x0[4];
    for (int i = 0; i < 4; ++i) {
        const float v = valid ? x[(int64_t)s * 4 + i] : 0.0f;
        const uint16_t vb = f2bf(v);
        x0[i] = bf2f(vb);
        if (train && valid) b.a0[(int64_t)s * 4 + i] = vb;
    }
    for (int o = 0; o < H; ++o) {
        float z = bf2f(P[256 + o]);
        for (int i = 0; i < 4; ++i) z += bf2f(P[o * 4 + i]) * x0[i];
        float dg;
        const float h = gelu(z, &dg);
        const uint16_t hb = f2bf(h);
        A[lane][o] = hb;
        if (train && valid) {
            b.z1[(int64_t)s * H + o] = z;
            b.a1[(int64_t)s * H + o] = hb;
        }
    }
    // layers 2 and 3 on MFMA
    for (int layer = 0; layer < 2; ++layer) {
        const int woff = layer == 0 ? 320 : 4480;
        const int boff = layer == 0 ? 4416 : 8576;
        float *zout = layer == 0 ? b.z2 : b.z3;
        uint16_t *aout = layer == 0 ? b.a2 : b.a3;
        for (int j = lane; j < H * H; j += 64) Wt[j / H][j % H] = P[woff + j];
        __syncthreads();
        v4f32 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                v4f32 c = {0.f, 0.f, 0.f, 0.f};
                // Z[s][o] = sum_i A[s][i] W[o][i]
                acc[mt][nt] = mfma_tile([&](int r, int k) { return A[r][k]; },
                                        [&](int k, int c2) { return Wt[c2][k]; }, 16 * mt, 16 * nt, H, c);
            }
        __syncthreads();
        const int r = lane & 15, kb = lane >> 4;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * kb + j, col = 16 * nt + r;
                    const float z = acc[mt][nt][j] + bf2f(P[boff + col]);
                    float dg;
                    const uint16_t hb = f2bf(gelu(z, &dg));
                    A[row][col] = hb;
                    const int ss = s0 + row;
                    if (train && ss < n) {
                        zout[(int64_t)ss * H + col] = z;
                        aout[(int64_t)ss * H + col] = hb;
                    }
                }
        __syncthreads();
    }
    // output layer
    float y = bf2f(P[8704]);
    for (int i = 0; i < H; ++i) y += bf2f(P[8640 + i]) * bf2f(A[lane][i]);
    if (valid) b.y[s] = y;
    float l2 = 0.0f;
    if (train) {
        const float d = valid ? y - t[s] : 0.0f;
        if (valid) b.dy[s] = 2.0f * d / (float)n;
        l2 = d * d;
        red[lane] = l2;
        __syncthreads();
        if (lane == 0) {
            float acc = 0.0f;
            for (int j = 0; j < 64; ++j) acc += red[j];
            b.loss_part[blockIdx.x] = acc;
        }
    }
}

// Backward pass of one tile: writes the tile's gradient of every parameter
// (summed over its samples) to grad_part[tile][8705].
__global__ void __launch_bounds__(64) mlp_backward_kernel(MlpBuffers b, int n) {
    __shared__ uint16_t G[TILE][H + 2];     // bf16 gradient w.r.t. pre-activations, [sample][unit]
    __shared__ uint16_t Aprev[TILE][H + 2]; // bf16 activations of the layer below, [sample][unit]
    __shared__ uint16_t Wt[H][H + 2];       // W[out][in] bf16
    __shared__ float dyl[TILE];
    const int lane = threadIdx.x;
    const int s0 = blockIdx.x * TILE;
    const int s = s0 + lane;
    const bool valid = s < n;
    const uint16_t *P = b.pbf;
    float *gp = b.grad_part + (int64_t)blockIdx.x * kMlpParams;

    dyl[lane] = valid ? b.dy[s] : 0.0f;
    // output layer: dW4[i] = sum_s dy a3[s][i]; db4 = sum_s dy
    for (int j = lane; j < TILE * H; j += 64) {
        const int ss = s0 + j / H;
        Aprev[j / H][j % H] = ss < n ? b.a3[(int64_t)ss * H + (j % H)] : (uint16_t)0;
    }
    __syncthreads();
    {
        float g = 0.0f;
        for (int k = 0; k < TILE; ++k) g += dyl[k] * bf2f(Aprev[k][lane]);
        gp[8640 + lane] = g;
        if (lane == 0) {
            float gb = 0.0f;
            for (int k = 0; k < TILE; ++k) gb += dyl[k];
            gp[8704] = gb;
        }
    }
    // dz3 = dy W4 * gelu'(z3)
    for (int o = 0; o < H; ++o) {
        float dz = 0.0f;
        if (valid) {
            float dg;
            gelu(b.z3[(int64_t)s * H + o], &dg);
            dz = dyl[lane] * bf2f(P[8640 + o]) * dg;
        }
        G[lane][o] = f2bf(dz);
    }
    __syncthreads();
    // layers 3 and 2: weight gradients and the gradient of the layer below
    for (int layer = 1; layer >= 0; --layer) {
        const int woff = layer == 0 ? 320 : 4480;
        const int boff = layer == 0 ? 4416 : 8576;
        const uint16_t *abelow = layer == 0 ? b.a1 : b.a2;
        const float *zbelow = layer == 0 ? b.z1 : b.z2;
        for (int j = lane; j < TILE * H; j += 64) {
            const int ss = s0 + j / H;
            Aprev[j / H][j % H] = ss < n ? abelow[(int64_t)ss * H + (j % H)] : (uint16_t)0;
        }
        for (int j = lane; j < H * H; j += 64) Wt[j / H][j % H] = P[woff + j];
        __syncthreads();
        const int r = lane & 15, kb = lane >> 4;
        // dW[o][i] = sum_s G[s][o] Aprev[s][i]
        for (int mt = 0; mt < 4; ++mt)
            for (int nt = 0; nt < 4; ++nt) {
                v4f32 c = {0.f, 0.f, 0.f, 0.f};
                c = mfma_tile([&](int o, int k) { return G[k][o]; }, [&](int k, int i) { return Aprev[k][i]; },
                              16 * mt, 16 * nt, TILE, c);
#pragma unroll
                for (int j = 0; j < 4; ++j) gp[woff + (16 * mt + 4 * kb + j) * H + 16 * nt + r] = c[j];
            }
        // db[o] = sum_s G[s][o]
        {
            float g = 0.0f;
            for (int k = 0; k < TILE; ++k) g += bf2f(G[k][lane]);
            gp[boff + lane] = g;
        }
        // dA[s][i] = sum_o G[s][o] W[o][i], then dz = dA * gelu'(z below)
        v4f32 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                v4f32 c = {0.f, 0.f, 0.f, 0.f};
                acc[mt][nt] = mfma_tile([&](int ss, int o) { return G[ss][o]; }, [&](int o, int i) { return Wt[o][i]; },
                                        16 * mt, 16 * nt, H, c);
            }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * kb + j, col = 16 * nt + r;
                    const int ss = s0 + row;
                    float dz = 0.0f;
                    if (ss < n) {
                        float dg;
                        gelu(zbelow[(int64_t)ss * H + col], &dg);
                        dz = acc[mt][nt][j] * dg;
                    }
                    G[row][col] = f2bf(dz);
                }
        __syncthreads();
    }
    // layer 1: dW1[o][i] = sum_s G[s][o] a0[s][i]; db1[o] = sum_s G[s][o]
    {
        float g[4] = {0.f, 0.f, 0.f, 0.f}, gb = 0.0f;
        for (int k = 0; k < TILE; ++k) {
            const int ss = s0 + k;
            if (ss >= n) break;
            const float gk = bf2f(G[k][lane]);
            gb += gk;
            for (int i = 0; i < 4; ++i) g[i] += gk * bf2f(b.a0[(int64_t)ss * 4 + i]);
        }
        for (int i = 0; i < 4; ++i) gp[lane * 4 + i] = g[i];
        gp[256 + lane] = gb;
    }
}

// Sums the tile gradients in a fixed order and, if step > 0, applies one Adam
// step to the FP32 master weights and refreshes the BF16 copy.
__global__ void mlp_adam_kernel(MlpBuffers b, int n_tiles, int step, float lr, float beta1, float beta2,
                                float eps) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams) return;
    float g = 0.0f;
    for (int t = 0; t < n_tiles; ++t) g += b.grad_part[(int64_t)t * kMlpParams + j];
    b.grad[j] = g;
    if (step <= 0) return;
    const float m = beta1 * b.m[j] + (1.0f - beta1) * g;
    const float v = beta2 * b.v[j] + (1.0f - beta2) * g * g;
    b.m[j] = m;
    b.v[j] = v;
    const float mh = m / (1.0f - powf(beta1, (float)step));
    const float vh = v / (1.0f - powf(beta2, (float)step));
    const float p = b.p[j] - lr * mh / (sqrtf(vh) + eps);
    b.p[j] = p;
    b.pbf[j] = f2bf(p);
}

// Refreshes the BF16 copy from the master weights.
__global__ void mlp_cast_kernel(MlpBuffers b) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kMlpParams) b.pbf[j] = f2bf(b.p[j]);
}

// Sums the tile losses (fixed order) into loss_out[idx].
__global__ void mlp_loss_kernel(MlpBuffers b, int n_tiles, int n, float *loss_out, int idx) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float acc = 0.0f;
    for (int t = 0; t < n_tiles; ++t) acc += b.loss_part[t];
    loss_out[idx] = acc / (float)n;
}

hipError_t mlp_launch_forward(const MlpBuffers &b, const float *x, const float *t, int n, int train, hipStream_t s) {
    const int tiles = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(tiles), dim3(64), 0, s, b, x, t, n, train);
    return hipGetLastError();
}

hipError_t mlp_launch_backward(const MlpBuffers &b, int n, hipStream_t s) {
    const int tiles = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(tiles), dim3(64), 0, s, b, n);
    return hipGetLastError();
}

hipError_t mlp_launch_adam(const MlpBuffers &b, int n, int step, float lr, hipStream_t s) {
    const int tiles = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, b, tiles, step, lr, 0.9f,
                       0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t mlp_launch_cast(const MlpBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(mlp_cast_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t mlp_launch_loss(const MlpBuffers &b, int n, float *loss_out, int idx, hipStream_t s) {
    const int tiles = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(64), 0, s, b, tiles, n, loss_out, idx);
    return hipGetLastError();
}

}  // namespace muca
