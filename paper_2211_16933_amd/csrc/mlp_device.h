// The learned closure's network layout and the bfloat16 helpers shared by its kernels and
// by the stage kernel's fused form of its inference.
//
// Parameters live in one packed FP32 array (and a bfloat16 copy of the same layout):
//   W1 [64][32] (inputs 12..31 zero), b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64],
//   W4 [16][64] (outputs >= Q_s zero), b4 [16].
// Normalisation block (FP32): in_mean[12], in_std[12], out_mean[16], out_std[16], lo[12],
// hi[12].
#pragma once
#include <hip/hip_runtime.h>

namespace elb {

constexpr int MLP_IN = 12, MLP_K1 = 32, MLP_H = 64, MLP_OUT = 16;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_K1;
constexpr int OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H * MLP_H;
constexpr int OFF_W4 = OFF_B3 + MLP_H, OFF_B4 = OFF_W4 + MLP_OUT * MLP_H;
constexpr int MLP_PARAMS = OFF_B4 + MLP_OUT;  // 11472
constexpr int NRM_IN_MEAN = 0, NRM_IN_STD = 12, NRM_OUT_MEAN = 24, NRM_OUT_STD = 40,
              NRM_LO = 56, NRM_HI = 68, MLP_NORM = 80;

constexpr int MLP_ROWS = 64;       // batch rows per block: 4 waves x 16
constexpr int AS = MLP_H + 8;      // LDS row stride (bf16) of an activation tile
constexpr int WS1 = MLP_K1 + 8;    // LDS row stride of W1
constexpr int WSH = MLP_H + 8;     // LDS row stride of W2, W3, W4 and of transposed weights
constexpr int WGRAD_ROWS = 128;    // batch rows per block of the weight-gradient kernel
constexpr int GS_T = WGRAD_ROWS + 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

// FP32 -> bfloat16, round to nearest even (finite inputs)
__device__ inline unsigned short f2bf(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// SiLU z s(z) and its derivative s (1 + z (1 - s)), with the logistic s(z) = 1 / (1 + 2^(-z
// log2 e)) from the hardware's base-2 exponential and reciprocal (v_exp_f32, v_rcp_f32,
// about 1 ulp each; far below the bfloat16 rounding of the activations that follows).
// Saturates to 0 and z for large |z|.
__device__ inline float sigmoid_hw(float z)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ inline float silu(float z) { return z * sigmoid_hw(z); }
__device__ inline float dsilu(float z)
{
    const float s = sigmoid_hw(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ inline bf16x8 ld8(const unsigned short *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(p));
}

}  // namespace elb
