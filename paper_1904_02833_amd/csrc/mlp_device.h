// Device pieces of the warm-start network (gfx950), shared by the network
// kernels and the solver's fused warm start: parameter layout, MFMA operand
// types, GELU, and the forward pass of a 16-sample tile on one wave with the
// weights held in registers.
//
// The network is a 32 -> 64 -> 64 -> 3 perceptron with GELU after both
// hidden layers, evaluated with BF16 MFMA (v_mfma_f32_16x16x32_bf16)
// accumulating in FP32; biases and GELU are FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace snake {
namespace mlp {

constexpr int NI = 32, NH = 64, NO = 3;
constexpr int P_W1 = 0, P_B1 = P_W1 + NH * NI, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH;
constexpr int P_W3 = P_B2 + NH, P_B3 = P_W3 + NO * NH, P_COUNT = P_B3 + NO;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// GELU(z) = z Phi(z) with the logistic approximation of the standard normal
// distribution function of Bowling, Khasawneh, Kaewkuekool and Cho, "A
// logistic approximation to the cumulative normal distribution" (J. Ind.
// Eng. Manag. 2, 2009): Phi(z) ~ 1 / (1 + exp(-(1.5976 z + 0.07056 z^3))),
// absolute error at most 1.4e-4, so GELU within 4e-4 of the exact-erf form
// (a fifth of the BF16 half-ulp that rounds every activation).  One
// exponential and one reciprocal; exp(-s) = 2^(-s log2 e) with the constants
// scaled by log2 e.
constexpr float kPhiC1 = -1.5976f * 1.4426950408889634f;
constexpr float kPhiC3 = -0.07056f * 1.4426950408889634f;

__device__ __forceinline__ float phi_logistic(float z)
{
    const float e = __builtin_amdgcn_exp2f(z * fmaf(kPhiC3, z * z, kPhiC1));
    return __builtin_amdgcn_rcpf(1.f + e);
}

__device__ __forceinline__ float gelu(float z) { return z * phi_logistic(z); }

// derivative of the same approximation: Phi + z Phi (1 - Phi) s'(z),
// s(z) = 1.5976 z + 0.07056 z^3 (within 8e-4 of the exact derivative)
__device__ __forceinline__ float gelu_grad(float z)
{
    const float ph = phi_logistic(z);
    const float ds = fmaf(3.f * 0.07056f, z * z, 1.5976f);
    return fmaf(z * ph * (1.f - ph), ds, ph);
}

// Weights of the forward pass as MFMA B operands of one lane (r = lane % 16,
// g = lane / 16): B1[nt] holds W1 rows nt * 16 + r, columns 8 g .. +8; B2 the
// same for both 32-column halves of W2; B3 the rows of W3 (rows >= 3 zero).
struct FwdWeights {
    bf16x8 B1[4], B2[4][2], B3[2];
    float bb1[4], bb2[4], bb3;
};

__device__ __forceinline__ void load_fwd_weights(const float* __restrict__ p, FwdWeights& W)
{
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int o = nt * 16 + r;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            W.B1[nt][j] = (__bf16)p[P_W1 + o * NI + 8 * g + j];
            W.B2[nt][0][j] = (__bf16)p[P_W2 + o * NH + 8 * g + j];
            W.B2[nt][1][j] = (__bf16)p[P_W2 + o * NH + 32 + 8 * g + j];
        }
        W.bb1[nt] = p[P_B1 + o];
        W.bb2[nt] = p[P_B2 + o];
    }
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            W.B3[kt][j] = r < NO ? (__bf16)p[P_W3 + r * NH + kt * 32 + 8 * g + j] : (__bf16)0.f;
    W.bb3 = r < NO ? p[P_B3 + r] : 0.f;
}

constexpr int FW_ROW = NH + 8;   // padded activation row (144 bytes)

// Forward pass of 16 samples on one wave.  `a` is the lane's A operand (the
// normalised inputs of sample r, columns 8 g .. +8, BF16); H is the wave's
// 16 x 64 BF16 buffer in LDS that turns each layer's output (D layout: lane
// l holds rows 4 g .. +4 of column r) into the next layer's A operand.
// Returns output r (r < 3) of samples 4 g .. +4, bias included.
__device__ __forceinline__ f32x4 forward_tile(const FwdWeights& W, bf16x8 a, __bf16 (*H)[FW_ROW])
{
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    // layer 1: h1 = GELU(W1 x + b1)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, W.B1[nt], zero, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) H[4 * g + v][nt * 16 + r] = (__bf16)gelu(acc[v] + W.bb1[nt]);
    }
    // (memcpy: the vector read may not be reordered with the element stores)
    bf16x8 a2[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) __builtin_memcpy(&a2[kt], &H[r][kt * 32 + 8 * g], sizeof(bf16x8));
    // layer 2: h2 = GELU(W2 h1 + b2)
    f32x4 acc2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        acc2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[0], W.B2[nt][0], zero, 0, 0, 0);
        acc2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[1], W.B2[nt][1], acc2[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) H[4 * g + v][nt * 16 + r] = (__bf16)gelu(acc2[nt][v] + W.bb2[nt]);
    bf16x8 a3[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) __builtin_memcpy(&a3[kt], &H[r][kt * 32 + 8 * g], sizeof(bf16x8));
    // layer 3: y = W3 h2 + b3 (columns >= 3 are padding)
    f32x4 acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[0], W.B3[0], zero, 0, 0, 0);
    acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[1], W.B3[1], acc3, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc3[v] += W.bb3;
    return acc3;
}

}  // namespace mlp
}  // namespace snake
