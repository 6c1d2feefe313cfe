// The training loss of Sec. II.A: energy and force errors with a relative
// weight, each a quadratic or exponential function of the difference, the
// energy error per configuration or per atom:
//   L = w_E / B  sum_c l_E(dE_c)  +  w_F / (3N)  sum_k,a l_F(F_ka - F*_ka),
//   dE_c = E_c - T_c, or (E_c - T_c) / N_c per atom;
//   l(x) = x^2 (quadratic) or exp(x^2) - 1 (exponential).
// Besides L it writes dL/dE_c and dL/dF_ka, the inputs of the gradient
// pass.  Blocks of 256 threads sum their terms in FP64 by a fixed tree; one
// more block adds the block sums in block order, so L is the same on every
// run.
#include "common.h"

namespace nnp {

constexpr int kLossThreads = 256;

__device__ __forceinline__ double loss_term(int kind, double x, double& dx) {
  if (kind == NN_LOSS_EXP) {
    const double e = exp(x * x);
    dx = 2.0 * x * e;
    return e - 1.0;
  }
  dx = 2.0 * x;
  return x * x;
}

// blocks [0, nbE) take structures, [nbE, nbE + nbF) force components
__global__ void __launch_bounds__(kLossThreads) k_loss_terms(nn_loss_params lp, const int64_t* __restrict__ atom_ptr,
                                                            int32_t B, int64_t N, const double* __restrict__ E,
                                                            const double* __restrict__ T, const float* __restrict__ F,
                                                            const float* __restrict__ Fr, double* __restrict__ dL_dE,
                                                            float* __restrict__ dL_dF, unsigned nbE,
                                                            double* __restrict__ partial) {
  __shared__ double sh[kLossThreads];
  double v = 0.0;
  if (blockIdx.x < nbE) {
    const int64_t c = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (c < B) {
      const double n = (double)(atom_ptr[c + 1] - atom_ptr[c]);
      const double scale = lp.per_atom ? 1.0 / (n > 0.0 ? n : 1.0) : 1.0;
      double d;
      v = lp.energy_weight / B * loss_term(lp.energy_kind, (E[c] - T[c]) * scale, d);
      dL_dE[c] = lp.energy_weight / B * d * scale;
    }
  } else {
    const int64_t x = (int64_t)(blockIdx.x - nbE) * kLossThreads + threadIdx.x;
    if (x < 3 * N) {
      double d;
      const double w = lp.force_weight / (3.0 * (double)N);
      v = w * loss_term(lp.force_kind, (double)F[x] - (double)Fr[x], d);
      dL_dF[x] = (float)(w * d);
    }
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kLossThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kLossThreads) k_loss_sum(const double* __restrict__ partial, unsigned n,
                                                          double* __restrict__ L) {
  __shared__ double sh[kLossThreads];
  double v = 0.0;
  for (unsigned b = threadIdx.x; b < n; b += kLossThreads) v += partial[b];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kLossThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *L = sh[0];
}

size_t loss_partial_elems(int64_t N, int32_t B) {
  return (size_t)((B + kLossThreads - 1) / kLossThreads + (3 * N + kLossThreads - 1) / kLossThreads + 1);
}

void launch_loss(const nn_loss_params& lp, const int64_t* atom_ptr, int32_t B, int64_t N, const double* E,
                 const double* T, const float* F, const float* Fr, double* L, double* dL_dE, float* dL_dF,
                 double* partial, hipStream_t s) {
  const unsigned nbE = (unsigned)((B + kLossThreads - 1) / kLossThreads);
  const unsigned nbF = F ? (unsigned)((3 * N + kLossThreads - 1) / kLossThreads) : 0u;
  if (nbE + nbF > 0)
    hipLaunchKernelGGL(k_loss_terms, dim3(nbE + nbF), dim3(kLossThreads), 0, s, lp, atom_ptr, B, N, E, T, F, Fr,
                       dL_dE, dL_dF, nbE, partial);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kLossThreads), 0, s, partial, nbE + nbF, L);
}

}  // namespace nnp
