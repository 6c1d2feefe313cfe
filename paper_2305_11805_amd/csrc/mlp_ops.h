// Activations of Eq. (1) and the FP32 MFMA step shared by the MLP kernels
// (the fused two-hidden-layer kernels and the layer-by-layer path).
#pragma once

#include <math.h>

#include "common.h"

namespace nnp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float act_f(int code, float z) {
  switch (code) {
    case NN_ACT_GAUSSIAN: return __builtin_amdgcn_exp2f(-1.4426950408889634f * z * z);
    case NN_ACT_RELU: return z > 0.f ? z : 0.f;
    case NN_ACT_TANH: return tanhf(z);
    default: return z;
  }
}
__device__ __forceinline__ float act_d(int code, float z, float a) {
  switch (code) {
    case NN_ACT_GAUSSIAN: return -2.0f * z * a;
    case NN_ACT_RELU: return z > 0.f ? 1.f : 0.f;
    case NN_ACT_TANH: return 1.0f - a * a;
    default: return 1.0f;
  }
}

__device__ __forceinline__ float act_d2(int code, float z, float a) {
  switch (code) {
    case NN_ACT_GAUSSIAN: return fmaf(4.0f * z, z, -2.0f) * a;
    case NN_ACT_TANH: return -2.0f * a * (1.0f - a * a);
    default: return 0.0f;
  }
}

// FP32 products use v_mfma_f32_16x16x4_f32 over 16-wide k blocks: lane
// (lm, lk) holds the four k values kb + 4 lk + i (i = 0..3) of its A row and
// B column, and the i-th of four MFMAs takes element i.  The four MFMAs
// together cover the whole block (each product a_k b_k once), so every lane
// fetches its operands as one 16-byte vector.
__device__ __forceinline__ float4 ld4(const float* p, int k, int kmax, bool vec) {
  if (vec && k + 3 < kmax) return *reinterpret_cast<const float4*>(p + k);
  float4 v;
  v.x = k < kmax ? p[k] : 0.f;
  v.y = k + 1 < kmax ? p[k + 1] : 0.f;
  v.z = k + 2 < kmax ? p[k + 2] : 0.f;
  v.w = k + 3 < kmax ? p[k + 3] : 0.f;
  return v;
}

__device__ __forceinline__ floatx4 mma4_f32(floatx4 acc, const float4& a, const float4& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
}

// Products in the MLP run in one of three modes:
//   kFp32  - FP32 operands, v_mfma_f32_16x16x4_f32;
//   kBf16  - operands rounded to BF16, v_mfma_f32_16x16x32_bf16, FP32 sums;
//   kBf16x3 - each operand split x = hi + lo with hi, lo in BF16 and the
//            product taken as hi*hi + hi*lo + lo*hi (three BF16 MFMAs, FP32
//            sums): about 16 significant bits per operand.
enum { kFp32 = 0, kBf16 = 1, kBf16x3 = 2 };

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const __bf16 h = (__bf16)x[q];
    hi[q] = h;
    lo[q] = (__bf16)(x[q] - (float)h);
  }
}

template <int MODE>
__device__ __forceinline__ floatx4 mma_bf16(floatx4 acc, const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                            const bf16x8& bl) {
  if constexpr (MODE == kBf16x3) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

}  // namespace nnp
