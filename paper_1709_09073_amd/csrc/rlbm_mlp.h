// rlbm_mlp.h -- the small network that supplies the starting point of the
// Fermi-Dirac / Bose-Einstein inversion (n, eps) -> (theta, z).
//
// The inversion is one-dimensional: z solves g_2(z)^3 / g_3(z)^2 = r with
// r = 2 n^3 / (pi eps^2) (theta cancels in Eq. n-eps-eq), so the network maps
// L = ln r to mu = ln z.  Layout of the float weight buffer (RLBM_MLP_FLOATS):
//   [0] a, [1] b      input normalisation   x = (L - a) * b
//   [2] m, [3] s      output scaling        mu = m + s * y
//   [4 .. 4+H)        W1   hidden weights
//   [4+H .. 4+2H)     b1   hidden biases
//   [4+2H .. 4+3H)    W2   output weights
//   [4+3H]            b2   output bias
// y = b2 + sum_h W2_h max(W1_h x + b1_h, 0)   (one hidden layer of H ReLU units).
#pragma once

#include "rlbm.h"

namespace rlbm_mlp {

constexpr int H = RLBM_MLP_HIDDEN;
constexpr int HDR = 4;
constexpr int NTRAIN = 3 * H + 1;          // trainable parameters
constexpr int NFLOAT = HDR + NTRAIN;
static_assert(NFLOAT == RLBM_MLP_FLOATS, "weight layout");

// mu = ln z guess from L = ln r (FP32 arithmetic; every lane reads the same weights)
// The output sum runs in four interleaved partial sums (units h = 4i + j go to sum j)
// so its dependency chain is a quarter as long.
__device__ __forceinline__ float eval(const float *__restrict__ w, float L) {
    static_assert(H % 4 == 0, "four partial sums");
    const float x = (L - w[0]) * w[1];
    float y[4] = {w[HDR + 3 * H], 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const float z = w[HDR + h] * x + w[HDR + H + h];
        y[h & 3] += w[HDR + 2 * H + h] * fmaxf(z, 0.0f);
    }
    return w[2] + w[3] * ((y[0] + y[1]) + (y[2] + y[3]));
}

}  // namespace rlbm_mlp
