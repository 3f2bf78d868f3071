// Device buffers of the MLP that predicts ln Omega / N for initial weights.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

constexpr int kMlpParams = 8705;   // 4*64+64 + 64*64+64 + 64*64+64 + 64+1
constexpr int kMlpIn = 4;
constexpr int kMlpHidden = 64;

struct MlpBuffers {
    float *p;          // [kMlpParams] FP32 master weights
    uint16_t *pbf;     // [kMlpParams] BF16 working copy
    float *m, *v;      // Adam moments
    float *grad;       // [kMlpParams] summed gradient of the last backward pass
    float *grad_part;  // [tiles][kMlpParams] per-tile gradients
    float *loss_part;  // [tiles]
    float *y, *dy;     // [n]
    float *z1, *z2, *z3;            // [n][64] pre-activations
    uint16_t *a0;                   // [n][4] bf16 inputs
    uint16_t *a1, *a2, *a3;         // [n][64] bf16 activations
};

hipError_t mlp_launch_forward(const MlpBuffers &b, const float *x, const float *t, int n, int train, hipStream_t s);
hipError_t mlp_launch_backward(const MlpBuffers &b, int n, hipStream_t s);
hipError_t mlp_launch_adam(const MlpBuffers &b, int n, int step, float lr, hipStream_t s);
hipError_t mlp_launch_cast(const MlpBuffers &b, hipStream_t s);
hipError_t mlp_launch_loss(const MlpBuffers &b, int n, float *loss_out, int idx, hipStream_t s);

}  // namespace muca
