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
// The atoms of each species are cut into fixed chunks in species order; one
// launch computes every chunk's partial sums of all the products above on
// FP32 MFMA (the atoms are the contraction index; biases and the output
// layer are extra columns of the same products), and a second kernel adds
// the chunk partials in chunk order, so the result is the same on every run.
#include "common.h"

namespace nnp {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Atoms per chunk: 128, or more for large N so that there are at most about
// 256 chunks (plus one partial chunk per species) and the partials stay small.
static int64_t chunk_atoms(int64_t N) {
  const int64_t per = (N + 255) / 256;
  const int64_t c = (per + 127) / 128 * 128;
  return c > 128 ? c : 128;
}

struct WgradLayout {
  int D, H1, H2;
  int64_t chunk;  // atoms per chunk
  int64_t off_w1, off_w2, off_b1, off_b2, off_w3, off_b3, per_chunk;
};

static WgradLayout wgrad_layout(int D, int H1, int H2, int64_t N) {
  WgradLayout L;
  L.D = D;
  L.H1 = H1;
  L.H2 = H2;
  L.chunk = chunk_atoms(N);
  L.off_w1 = 0;
  L.off_w2 = L.off_w1 + (int64_t)H1 * D;
  L.off_b1 = L.off_w2 + (int64_t)H2 * H1;
  L.off_b2 = L.off_b1 + H1;
  L.off_w3 = L.off_b2 + H2;
  L.off_b3 = L.off_w3 + H2;
  L.per_chunk = (L.off_b3 + 1 + 63) / 64 * 64;
  return L;
}

static int64_t n_chunks(int64_t N, int S) { return N / chunk_atoms(N) + S + 1; }

size_t wgrad_partial_floats(int64_t N, int S, const ModelDev& m) {
  const WgradLayout L = wgrad_layout(m.m[0].width[0], m.m[0].width[1], m.m[0].width[2], N);
  return (size_t)(n_chunks(N, S) * L.per_chunk);
}

// chunk -> (species, first and end position in perm); false if past the end
__device__ __forceinline__ bool chunk_range(const int64_t* sp_start, int S, int64_t chunk, int64_t c, int& s,
                                            int64_t& r0, int64_t& r1) {
  for (s = 0; s < S; ++s) {
    const int64_t ns = sp_start[s + 1] - sp_start[s];
    const int64_t nc = (ns + chunk - 1) / chunk;
    if (c < nc) {
      r0 = sp_start[s] + c * chunk;
      r1 = min(r0 + chunk, sp_start[s + 1]);
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

// Split-K products over atoms: for chunk c, job j and a 64 x 64 tile of the
// job's output, partial[c] = sum over the chunk's atoms k of A_k[m] B_k[n]:
//   job 0: A = w delta1 [H1], B = (G, 1)  [D + 1]  -> dW1 | db1
//   job 1: A = w delta2 [H2], B = (a1, 1) [H1 + 1] -> dW2 | db2
//   job 2: A = w (one row), B = (a2, 1)   [H2 + 1] -> dW3 | db3
// With the force term (src.x1 set) jobs 0 and 1 take two passes over the
// chunk, (x, (Y, 1)) and (-delta, (Y', 0)), and job 2 is A = 1, B = (c3, w).
// The block's four waves stage 32 atoms of A and B at a time in LDS (one
// atom row is contiguous in HBM) and each wave runs 16 x 64 of the tile on
// FP32 MFMA 16x16x4.  The chunk partials are reduced in chunk order later,
// so every sum is taken in a fixed order.
constexpr int kKB = 32;           // atoms per LDS slab
constexpr int kTile = 64;         // output tile edge
constexpr int kLdsLd = kTile + 16; // padded LDS row: the four k rows of an MFMA read fall in distinct banks

__device__ __forceinline__ void job_shape(int job, const WgradLayout& L, int& M, int& Ncol) {
  M = job == 0 ? L.H1 : job == 1 ? L.H2 : 1;
  Ncol = (job == 0 ? L.D : job == 1 ? L.H1 : L.H2) + 1;
}

// One slab row (an atom) of A or B for this thread: 8 consecutive values
// from column c0 of a row-major source of width `width`, zero past it.
__device__ __forceinline__ void load8(const float* __restrict__ row, int c0, int width, bool vec, float (&v)[8]) {
  if (vec && c0 + 8 <= width) {
    const float4 x = *reinterpret_cast<const float4*>(row + c0);
    const float4 y = *reinterpret_cast<const float4*>(row + c0 + 4);
    v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w, v[4] = y.x, v[5] = y.y, v[6] = y.z, v[7] = y.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = c0 + q < width ? row[c0 + q] : 0.f;
  }
}

__global__ void __launch_bounds__(256) k_wgrad_gemm(WgradArgs a, WgradLayout L, WgradSrc src) {
  __shared__ __align__(16) float As[kKB][kLdsLd];
  __shared__ __align__(16) float Bs[kKB][kLdsLd];
  const int job = blockIdx.z;
  int M, Ncol;
  job_shape(job, L, M, Ncol);
  const int tn = (Ncol + kTile - 1) / kTile;
  const int tiles = ((M + kTile - 1) / kTile) * tn;
  if ((int)blockIdx.y >= tiles) return;
  const int m0 = (blockIdx.y / tn) * kTile, n0 = (blockIdx.y % tn) * kTile;
  int s;
  int64_t r0, r1;
  if (!chunk_range(a.sp_start, a.S, L.chunk, blockIdx.x, s, r0, r1)) return;
  const bool fm = src.x1 != nullptr;
  const int Ny = Ncol - 1;  // columns of the per-atom B source
  const float* Xw = job == 0 ? src.d1 : src.d2;  // delta (energy term: times w)
  const float* Xf = job == 0 ? src.x1 : src.x2;  // x (force term)
  const float* Y = job == 0 ? src.G : job == 1 ? src.a1 : src.a2;
  const float* Yf = job == 0 ? src.U : src.t1;
  const bool vecY = (Ny & 3) == 0;  // rows 16-byte aligned (buffers are)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const int sr = tid >> 3, sc = (tid & 7) * 8;  // staging: slab row (atom) and first of 8 columns
  const int passes = (fm && job < 2) ? 2 : 1;
  const int nslab = (int)((r1 - r0 + kKB - 1) / kKB);
  const int total = passes * nslab;
  // the values this thread stages for slab q (loaded one slab ahead)
  auto fetch = [&](int q, float (&av)[8], float (&bv)[8]) {
    const int pass = q >= nslab ? 1 : 0;
    const int64_t row = r0 + (int64_t)(q - pass * nslab) * kKB + sr;
    const int atom = row < r1 ? a.perm[row] : -1;
#pragma unroll
    for (int k = 0; k < 8; ++k) av[k] = bv[k] = 0.f;
    if (atom < 0) return;
    const float w = a.w[atom];
    if (job == 2) {
      if (m0 + sc == 0) av[0] = fm ? 1.f : w;
    } else {
      const float* X = (fm && pass == 0) ? Xf : Xw;
      load8(X + (int64_t)atom * M, m0 + sc, M, true, av);
      const float scale = fm ? (pass == 0 ? 1.f : -1.f) : w;
#pragma unroll
      for (int k = 0; k < 8; ++k) av[k] *= scale;
    }
    load8((pass == 0 ? Y : Yf) + (int64_t)atom * Ny, n0 + sc, Ny, vecY, bv);
    const int ones = Ny - (n0 + sc);  // the extra column, if it falls in this thread's eight
    if (ones >= 0 && ones < 8) bv[ones] = job == 2 ? (fm ? w : 1.f) : (pass == 0 ? 1.f : 0.f);
  };
  floatx4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float av[8], bv[8];
  if (total > 0) fetch(0, av, bv);
  for (int q = 0; q < total; ++q) {
    *reinterpret_cast<float4*>(&As[sr][sc]) = make_float4(av[0], av[1], av[2], av[3]);
    *reinterpret_cast<float4*>(&As[sr][sc + 4]) = make_float4(av[4], av[5], av[6], av[7]);
    *reinterpret_cast<float4*>(&Bs[sr][sc]) = make_float4(bv[0], bv[1], bv[2], bv[3]);
    *reinterpret_cast<float4*>(&Bs[sr][sc + 4]) = make_float4(bv[4], bv[5], bv[6], bv[7]);
    __syncthreads();
    if (q + 1 < total) fetch(q + 1, av, bv);  // in flight during the products below
    if (m0 + 16 * wv < M) {
#pragma unroll
      for (int k = 0; k < kKB; k += 4) {
        const float x = As[k + lk][16 * wv + lm];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, Bs[k + lk][16 * t + lm], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* out = a.partial + (int64_t)blockIdx.x * L.per_chunk;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int n = n0 + 16 * t + lm;
    if (n >= Ncol) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + 16 * wv + 4 * lk + j;
      if (m >= M) continue;
      int64_t dst;
      if (job == 0) dst = n < Ny ? L.off_w1 + (int64_t)m * Ny + n : L.off_b1 + m;
      else if (job == 1) dst = n < Ny ? L.off_w2 + (int64_t)m * Ny + n : L.off_b2 + m;
      else dst = n < Ny ? L.off_w3 + n : L.off_b3;
      out[dst] = acc[t][j];
    }
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
  for (int q = 0; q < s; ++q) c0 += (a.sp_start[q + 1] - a.sp_start[q] + L.chunk - 1) / L.chunk;
  const int64_t nc = (a.sp_start[s + 1] - a.sp_start[s] + L.chunk - 1) / L.chunk;
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
  const WgradLayout L = wgrad_layout(D, m.m[0].width[1], m.m[0].width[2], N);
  const int64_t chunks = n_chunks(N, a.S);
  int tiles = 0;
  for (int job = 0; job < 3; ++job) {
    const int M = job == 0 ? L.H1 : job == 1 ? L.H2 : 1;
    const int Ncol = (job == 0 ? L.D : job == 1 ? L.H1 : L.H2) + 1;
    const int t = ((M + kTile - 1) / kTile) * ((Ncol + kTile - 1) / kTile);
    tiles = t > tiles ? t : tiles;
  }
  hipLaunchKernelGGL(k_wgrad_gemm, dim3((unsigned)chunks, (unsigned)tiles, 3), dim3(256), 0, s, a, L, src);
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
