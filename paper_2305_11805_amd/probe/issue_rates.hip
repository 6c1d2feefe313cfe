// Issue-rate probe for the rooflines of the FP32 VALU kernels: the rate of
// unpacked v_fma_f32, of v_exp_f32, of the FP32 MFMA shapes the descriptor
// and MLP kernels use, and of MFMA and FMA mixed in one wave, on every CU at
// 1 to 8 waves per SIMD.  Built with packed FP32 disabled, like the library.
//
//   ./paper_2305_11805_amd/probe/issue_rates
//
// Each thread writes only out[its global index]; the buffer holds one float
// per thread of the largest grid.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kIters = 4096;

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

// 32 FMAs per iteration in 8 independent chains
__global__ void __launch_bounds__(256) k_fma(float* out, float a0) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = a0 + c;
  const float m = 0.999f + threadIdx.x * 1e-7f, k = 1e-4f;
  for (int i = 0; i < kIters; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], m, k);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 exp2 per iteration in 8 independent chains
__global__ void __launch_bounds__(256) k_exp(float* out, float a0) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = -1e-3f * (a0 + c + threadIdx.x);
  for (int i = 0; i < kIters; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = -__builtin_amdgcn_exp2f(x[c]) * 1e-3f;
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 independent 4x4x1 (16 blocks) MFMA chains
__global__ void __launch_bounds__(256) k_mfma4(float* out, float a0) {
  floatx4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  const float a = a0 + threadIdx.x * 1e-3f, b = a0 - threadIdx.x * 1e-3f;
  for (int i = 0; i < kIters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_4x4x1f32(b, b, c3, 0, 0, 0);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

// 4 independent 16x16x4 MFMA chains
__global__ void __launch_bounds__(256) k_mfma16(float* out, float a0) {
  floatx4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  const float a = a0 + threadIdx.x * 1e-3f, b = a0 - threadIdx.x * 1e-3f;
  for (int i = 0; i < kIters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, b, c3, 0, 0, 0);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

// both: 4 MFMA 4x4x1 and 32 FMAs per iteration, independent of each other
__global__ void __launch_bounds__(256) k_mix(float* out, float a0) {
  floatx4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  const float a = a0 + threadIdx.x * 1e-3f, b = a0 - threadIdx.x * 1e-3f;
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = a0 + c;
  const float m = 0.999f + threadIdx.x * 1e-7f, k = 1e-4f;
  for (int i = 0; i < kIters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_4x4x1f32(b, b, c3, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], m, k);
  }
  float s = c0[0] + c1[1] + c2[2] + c3[3];
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

struct Probe {
  const char* name;
  void (*kernel)(float*, float);
  double flops_per_wave_iter;  // FMA = 2, exp2 = 1, MFMA = 2 M N K blocks
  int instr_per_wave_iter;
};

}  // namespace

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  const double ghz = prop.clockRate * 1e-6;
  std::printf("%s, %d CUs, peak clock %.2f GHz, LDS per block %zu B\n", prop.gcnArchName, cus, ghz,
              prop.sharedMemPerBlock);
  const Probe probes[] = {
      {"v_fma_f32 (unpacked)", k_fma, 32 * 2 * 64.0, 32},
      {"v_exp_f32", k_exp, 8 * 64.0, 8},
      {"mfma_f32_4x4x1_16b", k_mfma4, 4 * 512.0, 4},
      {"mfma_f32_16x16x4", k_mfma16, 4 * 2048.0, 4},
      {"4 mfma 4x4x1 + 32 fma", k_mix, 4 * 512.0 + 32 * 128.0, 36},
  };
  const int max_blocks = cus * 8;
  float* out;
  CHECK(hipMalloc(&out, (size_t)max_blocks * 256 * sizeof(float)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::printf("%-24s %10s %12s %14s %18s\n", "probe", "waves/SIMD", "ms", "TFLOP/s", "SIMD clocks/instr");
  for (const Probe& pr : probes) {
    for (int wps = 1; wps <= 8; wps *= 2) {
      const int blocks = cus * wps;  // 4 waves per block: wps waves on each of the 4 SIMDs of a CU
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(pr.kernel, dim3(blocks), dim3(256), 0, 0, out, 1.0f);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&ms, e0, e1));
      }
      const double waves = (double)blocks * 4, s = ms * 1e-3;
      const double tflops = waves * kIters * pr.flops_per_wave_iter / s / 1e12;
      // clocks per wave instruction on one SIMD, at the peak clock
      const double cpi = s * ghz * 1e9 / (wps * (double)kIters * pr.instr_per_wave_iter);
      std::printf("%-24s %10d %12.3f %14.1f %18.2f\n", pr.name, wps, ms, tflops, cpi);
    }
  }
  CHECK(hipFree(out));
  return 0;
}
