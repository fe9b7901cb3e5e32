// mlp.h -- the refinement predictor's network on the GPU: 32 inputs -> 64 -> 64 -> 1 logit
// (ReLU), parameters in one flat vector W1[64][32], b1[64], W2[64][64], b2[64], w3[64], b3.
//
// Two forward forms:
//  * training (k_mlp_fwd_bwd): minibatches of 64 samples per workgroup, the three dense
//    products of the forward pass and the three of the backward pass on the matrix cores
//    (bfloat16 operands rounded to nearest even, float32 accumulation, 16x16x16 tiles);
//  * deployment (mlp_logit_wave): one candidate at a time per wave, one hidden unit per
//    lane, bfloat16 parameters, float32 sums taken in a fixed sequential order with no fused
//    multiply-add, so that every refinement decision is reproducible outside the GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrl {

constexpr int MLP_IN = 32, MLP_H = 64;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN, MLP_OFF_W2 = MLP_OFF_B1 + MLP_H,
              MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H, MLP_OFF_W3 = MLP_OFF_B2 + MLP_H,
              MLP_OFF_B3 = MLP_OFF_W3 + MLP_H, MLP_NPARAM = MLP_OFF_B3 + 1;

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Deployment logit of the feature vector x[0..30] held by lane c of the calling wave; every
// lane of the wave must call it with the same c (wave-uniform) and receives the logit. Lane j
// computes hidden unit j of both layers and the other lanes' values arrive by readlane, so
// each sum keeps the order input 0, 1, ... / hidden 0, 1, ... with one rounding per product
// and per addition (no fused multiply-add).
__device__ inline float bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

__device__ inline float mlp_logit_wave(const uint16_t* __restrict__ w, const float* x, int c, int lane) {
    float a = bf2f(w[MLP_OFF_B1 + lane]);
#pragma unroll
    for (int i = 0; i < MLP_IN - 1; ++i) a = a + bf2f(w[MLP_OFF_W1 + lane * MLP_IN + i]) * bcast(x[i], c);
    const float h1 = a > 0.f ? a : 0.f;
    float h2 = bf2f(w[MLP_OFF_B2 + lane]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) h2 = h2 + bf2f(w[MLP_OFF_W2 + lane * MLP_H + k]) * bcast(h1, k);
    const float t = bf2f(w[MLP_OFF_W3 + lane]) * (h2 > 0.f ? h2 : 0.f);
    float o = bf2f(w[MLP_OFF_B3]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) o = o + bcast(t, k);
    return o;
}

}  // namespace mrl
