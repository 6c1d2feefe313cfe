// Gradients of the per-structure energies with respect to the MLP
// parameters and the positions (the loss gradient of Sec. II.A; forces are
// the negative position gradient of the energy, Sec. II).
//
// With w_i = dL/dE of atom i's structure, delta_l,i = dE_i/dz^l and a^0 = G:
//   dL/dW^l = sum_i w_i delta_l,i a_{l-1,i}^T,   dL/db^l = sum_i w_i delta_l,i,
//   dL/dW^3 = sum_i w_i a_2,i,  dL/db^3 = sum_i w_i.
// With a loss on forces as well (L = sum_i (w_i E_i - E_dot_i), E_dot the
// derivative of the MLP along the descriptor tangent u), each hidden layer
// gets a second product, with x_l = w delta_l - eps_l from the tangent pass:
//   dL/dW^1 = sum_i x_1,i G_i^T - delta_1,i u_i^T,
//   dL/dW^2 = sum_i x_2,i a_1,i^T - delta_2,i a1_dot_i^T,
//   dL/db^l = sum_i x_l,i,  dL/dW^3 = sum_i (w_i a_2,i - a2_dot_i).
// The atoms of each species are cut into chunks of kChunk in species order.
// For each chunk, one wave computes one 16 x 64 tile of a weight gradient on
// FP32 MFMA (the atoms are the contraction index), and a second kernel adds
// the bias and output-layer columns.  The chunk partial sums are then
// reduced in chunk order, so the result is the same on every run.
#include "common.h"

namespace nnp {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 512;

struct WgradLayout {
  int D, H1, H2;
  int64_t off_w1, off_w2, off_b1, off_b2, off_w3, off_b3, per_chunk;
};

static WgradLayout wgrad_layout(int D, int H1, int H2) {
  WgradLayout L;
  L.D = D;
  L.H1 = H1;
  L.H2 = H2;
  L.off_w1 = 0;
  L.off_w2 = L.off_w1 + (int64_t)H1 * D;
  L.off_b1 = L.off_w2 + (int64_t)H2 * H1;
  L.off_b2 = L.off_b1 + H1;
  L.off_w3 = L.off_b2 + H2;
  L.off_b3 = L.off_w3 + H2;
  L.per_chunk = (L.off_b3 + 1 + 63) / 64 * 64;
  return L;
}

size_t wgrad_partial_floats(int64_t N, int S, const ModelDev& m) {
  const WgradLayout L = wgrad_layout(m.m[0].width[0], m.m[0].width[1], m.m[0].width[2]);
  const int64_t chunks = N / kChunk + S + 1;
  return (size_t)(chunks * L.per_chunk);
}

// chunk -> (species, first and end position in perm); false if past the end
__device__ __forceinline__ bool chunk_range(const int64_t* sp_start, int S, int64_t c, int& s, int64_t& r0,
                                            int64_t& r1) {
  for (s = 0; s < S; ++s) {
    const int64_t ns = sp_start[s + 1] - sp_start[s];
    const int64_t nc = (ns + kChunk - 1) / kChunk;
    if (c < nc) {
      r0 = sp_start[s] + c * kChunk;
      r1 = min(r0 + kChunk, sp_start[s + 1]);
      return true;
    }
    c -= nc;
  }
  return false;
}

__global__ void k_atom_weights(const double* __restrict__ dL_dE, const int64_t* __restrict__ atom_ptr, int32_t B,
                               int64_t N, float* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (!dL_dE) {
    w[i] = 0.f;
    return;
  }
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (atom_ptr[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  w[i] = (float)dL_dE[lo];
}

__global__ void k_pos_grad(const double* __restrict__ dL_dE, const int64_t* __restrict__ atom_ptr, int32_t B,
                           int64_t N, const float* __restrict__ F, float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (atom_ptr[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const float s = -(float)dL_dE[lo];
  g[3 * i] = s * F[3 * i];
  g[3 * i + 1] = s * F[3 * i + 1];
  g[3 * i + 2] = s * F[3 * i + 2];
}

// out[m][n] (chunk partial) = sum over the chunk's atoms k of w_k X_k[m] Y_k[n]
// job 0: X = delta1 [N][H1], Y = G  [N][D]   -> dW1 [H1][D]
// job 1: X = delta2 [N][H2], Y = a1 [N][H1]  -> dW2 [H2][H1]
// With the force term (src.x1 set) the sum is X'_k[m] Y_k[n] - X_k[m] Y'_k[n]
// instead, X' = x1 / x2 and Y' = u / a1_dot, with no weight w_k.
__global__ void __launch_bounds__(64) k_wgrad_mm(WgradArgs a, WgradLayout L, WgradSrc src) {
  const int job = blockIdx.z;
  const bool fm = src.x1 != nullptr;
  const float* X = job == 0 ? src.d1 : src.d2;
  const float* Y = job == 0 ? src.G : src.a1;
  const float* Xf = job == 0 ? src.x1 : src.x2;
  const float* Yf = job == 0 ? src.U : src.t1;
  const int M = job == 0 ? L.H1 : L.H2;
  const int Nc = job == 0 ? L.D : L.H1;
  const int ldx = M, ldy = Nc;
  const int ntn = (Nc + 63) / 64;
  const int tile = blockIdx.y;
  if (tile >= (M / 16) * ntn) return;
  const int m0 = (tile / ntn) * 16, n0 = (tile % ntn) * 64;
  int s;
  int64_t r0, r1;
  if (!chunk_range(a.sp_start, a.S, blockIdx.x, s, r0, r1)) return;
  const int lane = threadIdx.x, lm = lane & 15, lk = lane >> 4;
  floatx4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = r0; k0 < r1; k0 += 4) {
    const int64_t kk = k0 + lk;
    const bool valid = kk < r1;
    const int64_t atom = valid ? a.perm[kk] : 0;
    if (fm) {
      const float av = valid ? Xf[atom * ldx + m0 + lm] : 0.f;
      const float avn = valid ? -X[atom * ldx + m0 + lm] : 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = n0 + 16 * t + lm;
        const bool in = valid && col < Nc;
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, in ? Y[atom * ldy + col] : 0.f, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(avn, in ? Yf[atom * ldy + col] : 0.f, acc[t], 0, 0, 0);
      }
    } else {
      const float av = valid ? a.w[atom] * X[atom * ldx + m0 + lm] : 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = n0 + 16 * t + lm;
        const float bv = (valid && col < Nc) ? Y[atom * ldy + col] : 0.f;
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  float* out = a.partial + (int64_t)blockIdx.x * L.per_chunk + (job == 0 ? L.off_w1 : L.off_w2);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = n0 + 16 * t + lm;
    if (col < Nc)
#pragma unroll
      for (int j = 0; j < 4; ++j) out[(int64_t)(m0 + 4 * lk + j) * Nc + col] = acc[t][j];
  }
}

// Bias columns and the output layer: sums over the chunk's atoms, one
// thread per output element, atoms in order.  With the force term the
// sources already hold the weighted values (x1, x2, c3 = w a2 - a2_dot).
__global__ void __launch_bounds__(256) k_wgrad_cols(WgradArgs a, WgradLayout L, WgradSrc src) {
  int s;
  int64_t r0, r1;
  if (!chunk_range(a.sp_start, a.S, blockIdx.x, s, r0, r1)) return;
  const bool fm = src.x1 != nullptr;
  float* out = a.partial + (int64_t)blockIdx.x * L.per_chunk;
  const int ncol = L.H1 + 2 * L.H2 + 1;
  for (int t = threadIdx.x; t < ncol; t += blockDim.x) {
    const float* p;
    int ld, col;
    int64_t dst;
    if (t < L.H1) {
      p = fm ? src.x1 : src.d1, ld = L.H1, col = t, dst = L.off_b1 + t;
    } else if (t < L.H1 + L.H2) {
      col = t - L.H1;
      p = fm ? src.x2 : src.d2, ld = L.H2, dst = L.off_b2 + col;
    } else if (t < L.H1 + 2 * L.H2) {
      p = src.a2, ld = L.H2, col = t - L.H1 - L.H2, dst = L.off_w3 + col;
    } else {
      p = nullptr, ld = 0, col = 0, dst = L.off_b3;
    }
    float acc = 0.f;
    for (int64_t k = r0; k < r1; ++k) {
      const int64_t atom = a.perm[k];
      if (!p) acc += a.w[atom];
      else if (fm) acc += p[atom * ld + col];
      else acc = fmaf(a.w[atom], p[atom * ld + col], acc);
    }
    out[dst] = acc;
  }
}

struct GradOut {
  float* W[NN_MAX_SPECIES][3];
  float* b[NN_MAX_SPECIES][3];
};

// Sum of the chunk partials of each species, in chunk order.
__global__ void k_wgrad_reduce(WgradArgs a, WgradLayout L, GradOut out) {
  const int s = blockIdx.y;
  if (s >= a.S) return;
  int64_t c0 = 0;
  for (int q = 0; q < s; ++q) c0 += (a.sp_start[q + 1] - a.sp_start[q] + kChunk - 1) / kChunk;
  const int64_t nc = (a.sp_start[s + 1] - a.sp_start[s] + kChunk - 1) / kChunk;
  const int64_t P = L.off_b3 + 1;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int64_t c = 0; c < nc; ++c) acc += a.partial[(c0 + c) * L.per_chunk + p];
    float* dst = nullptr;
    int64_t o = 0;
    if (p < L.off_w2) dst = out.W[s][0], o = p - L.off_w1;
    else if (p < L.off_b1) dst = out.W[s][1], o = p - L.off_w2;
    else if (p < L.off_b2) dst = out.b[s][0], o = p - L.off_b1;
    else if (p < L.off_w3) dst = out.b[s][1], o = p - L.off_b2;
    else if (p < L.off_b3) dst = out.W[s][2], o = p - L.off_w3;
    else dst = out.b[s][2], o = 0;
    if (dst) dst[o] = acc;
  }
}

void launch_atom_weights(const double* dL_dE, const int64_t* atom_ptr, int32_t B, int64_t N, float* w, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_atom_weights, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, dL_dE, atom_ptr, B, N, w);
}

void launch_pos_grad(const double* dL_dE, const int64_t* atom_ptr, int32_t B, int64_t N, const float* F,
                     float* dL_dpos, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_pos_grad, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, dL_dE, atom_ptr, B, N, F,
                     dL_dpos);
}

void launch_wgrad(const WgradArgs& a, const ModelDev& m, const WgradSrc& src, int D, int64_t N, float* const* dW,
                  float* const* db, hipStream_t s) {
  const WgradLayout L = wgrad_layout(D, m.m[0].width[1], m.m[0].width[2]);
  const int64_t chunks = N / kChunk + a.S + 1;
  const int tiles1 = (L.H1 / 16) * ((L.D + 63) / 64), tiles2 = (L.H2 / 16) * ((L.H1 + 63) / 64);
  const int tiles = tiles1 > tiles2 ? tiles1 : tiles2;
  hipLaunchKernelGGL(k_wgrad_mm, dim3((unsigned)chunks, (unsigned)tiles, 2), dim3(64), 0, s, a, L, src);
  hipLaunchKernelGGL(k_wgrad_cols, dim3((unsigned)chunks), dim3(256), 0, s, a, L, src);
  GradOut out{};
  for (int sp = 0; sp < a.S; ++sp)
    for (int l = 0; l < 3; ++l) {
      out.W[sp][l] = dW ? dW[sp * NN_MAX_LAYERS + l] : nullptr;
      out.b[sp][l] = db ? db[sp * NN_MAX_LAYERS + l] : nullptr;
    }
  const int64_t P = L.off_b3 + 1;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((P + 255) / 256), (unsigned)a.S), dim3(256), 0, s, a, L, out);
}

}  // namespace nnp
