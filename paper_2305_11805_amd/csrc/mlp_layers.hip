// Per-species MLPs of any depth and width (Eq. (1); Sec. II.A gives every
// species its own network), layer by layer on FP32 MFMA.
//
// The fused kernels of mlp.hip cover two hidden layers of a few widths shared
// by all species.  Everything else -- one to three hidden layers, any widths,
// different architectures per species (for instance the 64-32, 256-128 and
// 1024-512-256 networks of Table II) -- runs here, one launch per layer for
// all species at once:
//   forward   z^h = W^h a^(h-1) + b^h,  a^h = act(z^h)  (a^0 = G),
//             stashing a^h and act'(z^h) per atom;
//   output    E = w . a^(L-1) + b  and  delta^(L-1) = w * act'(z^(L-1));
//   backward  delta^(h-1) = (W^h^T delta^h) * act'(z^(h-1)),
//             lambda = dE/dG = W^1^T delta^1;
//   weights   dL/dW^h = sum_i x^h_i a^(h-1)_i^T (split over atom chunks,
//             partial sums added in chunk order).
// With a loss on forces the forward pass also carries the tangent along the
// descriptor tangent u (a_dot^h = act'(z^h) W^h a_dot^(h-1), a_dot^0 = u),
// and the reverse pass of  w E - E_dot  runs two adjoints per layer:
//   z_bar^h = a_bar^h act'(z^h) + a_dot_bar^h act''(z^h) z_dot^h,
//   z_dot_bar^h = a_dot_bar^h act'(z^h),
//   a_bar^(h-1) = W^h^T z_bar^h,  a_dot_bar^(h-1) = W^h^T z_dot_bar^h,
//   dL/dW^h = sum_i z_bar^h a^(h-1)^T + z_dot_bar^h a_dot^(h-1)^T,
// starting from z_bar = w, z_dot_bar = -1 at the linear output.
//
// Rows are atoms in species order (slot r is atom perm[r]).  A block computes
// 16 rows x 64 columns as four 16x16x4 FP32 MFMA tiles, its four waves each
// taking every fourth 16-wide block of the contraction and adding their sums
// in wave order through LDS at the end (a 16-atom cell gives few tiles, so
// the contraction is what there is to spread); the k order inside each
// 16-wide block is permuted identically for both operands, so every lane
// loads its A row as 16-byte vectors.  Per-hidden-layer stashes are
// [rows][ld] with ld the largest width of that layer rounded up to 16.
#include <algorithm>

#include "common.h"
#include "mlp_ops.h"

namespace nnp {

constexpr int kLayRows = 16;   // rows of one species per tile
constexpr int kLayWaves = 4;   // waves per block: they split the contraction of one 16 x 64 tile

// Row tile t of a launch -> its species and rows [r0, r1) in slot order;
// false past the last tile.
__device__ __forceinline__ bool lay_tile(const int64_t* __restrict__ sp_start, int S, int64_t t, int& s, int64_t& r0,
                                         int64_t& r1) {
  for (s = 0; s < S; ++s) {
    const int64_t ns = sp_start[s + 1] - sp_start[s];
    const int64_t nt = (ns + kLayRows - 1) / kLayRows;
    if (t < nt) {
      r0 = sp_start[s] + t * kLayRows;
      r1 = min(r0 + kLayRows, sp_start[s + 1]);
      return true;
    }
    t -= nt;
  }
  return false;
}

__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------------------------
// forward of hidden layer h (weights W[h-1]), with the tangent when TAN
// ---------------------------------------------------------------------------

template <bool TAN>
__global__ void __launch_bounds__(64 * kLayWaves) k_lay_fwd(LayArgs A, int h) {
  __shared__ float red[TAN ? 2 : 1][kLayWaves][4][4][64];  // per wave: its partial sums over its k blocks
  int s;
  int64_t r0, r1;
  if (!lay_tile(A.sp_start, A.model.S, blockIdx.x, s, r0, r1)) return;
  const MlpDev& M = A.model.m[s];
  if (M.n_layers <= h) return;  // no hidden layer h in this species
  const int K = M.width[h - 1], Nout = M.width[h];
  const int c0 = (int)blockIdx.y * 64;
  if (c0 >= Nout) return;  // block-uniform
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
  // this lane's A row (rows past the tile read row r0: their sums are never stored)
  const int64_t r = (r0 + lm < r1) ? r0 + lm : r0;
  const float *xr, *ur = nullptr;
  bool vx;
  if (h == 1) {
    const int64_t atom = A.perm[r];
    xr = A.G + atom * A.D;
    if (TAN) ur = A.U + atom * A.D;
    vx = (A.D & 3) == 0 && aligned16(A.G) && (!TAN || aligned16(A.U));
  } else {
    xr = A.buf.a[h - 1] + r * A.buf.ld[h - 1];
    if (TAN) ur = A.buf.at[h - 1] + r * A.buf.ld[h - 1];
    vx = true;
  }
  const float* W = M.W[h - 1];
  const bool vw = (K & 3) == 0 && aligned16(W);
  floatx4 acc[4], acct[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = acct[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  // the waves split the contraction: wave w takes the 16-wide blocks w, w + 4, ...
  for (int k0 = 16 * wv; k0 < K; k0 += 16 * kLayWaves) {
    const int k = k0 + 4 * lk;
    const float4 a = ld4(xr, k, K, vx);
    float4 at{};
    if constexpr (TAN) at = ld4(ur, k, K, vx);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = c0 + 16 * t + lm;
      const float4 b = n < Nout ? ld4(W + (int64_t)n * K, k, K, vw) : float4{0.f, 0.f, 0.f, 0.f};
      acc[t] = mma4_f32(acc[t], a, b);
      if constexpr (TAN) acct[t] = mma4_f32(acct[t], at, b);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      red[0][wv][t][j][lane] = acc[t][j];
      if constexpr (TAN) red[TAN ? 1 : 0][wv][t][j][lane] = acct[t][j];
    }
  __syncthreads();
  // wave w finishes column tile t = w: the four waves' sums in wave order
  // (the same order on every run); lane (lm, lk) holds rows 4 lk + j, column
  // c0 + 16 w + lm
  const int t = wv;
  const int n = c0 + 16 * t + lm;
  if (n >= Nout) return;
  const int act = M.act[h - 1];
  const int ld = A.buf.ld[h];
  const float bn = M.b[h - 1][n];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t rr = r0 + 4 * lk + j;
    if (rr >= r1) continue;
    float zs = 0.f, zts = 0.f;
#pragma unroll
    for (int q = 0; q < kLayWaves; ++q) {
      zs += red[0][q][t][j][lane];
      if constexpr (TAN) zts += red[TAN ? 1 : 0][q][t][j][lane];
    }
    const float z = zs + bn;
    const float a = act_f(act, z);
    const float d = act_d(act, z, a);
    A.buf.a[h][rr * ld + n] = a;
    A.buf.s[h][rr * ld + n] = d;
    if constexpr (TAN) {
      A.buf.at[h][rr * ld + n] = d * zts;
      A.buf.q[h][rr * ld + n] = act_d2(act, z, a) * zts;
    }
  }
}

// ---------------------------------------------------------------------------
// linear output layer: the atom's outputs, and the adjoints of the last
// hidden layer
//   mode 0: E only;  1: delta = w_out * act';
//   2 (loss on forces, per-atom weight w): z_bar = w_out (w act' - act'' z_dot),
//     z_dot_bar = -w_out act';
//   3: the n_out outputs into out [N][n_out] (no adjoint);
//   4: delta = (sum_o seed_o w_out[o]) * act'  (seeded outputs, no output write).
// 16 lanes per row; fixed shuffle tree, so the outputs are the same on every run.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_lay_out(LayArgs A, int mode) {
  const int64_t r = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int sub = threadIdx.x & 15;
  const int S = A.model.S;
  const bool valid = r < A.sp_start[S];
  int s = 0;
  if (valid)
    while (s + 1 < S && A.sp_start[s + 1] <= r) ++s;
  const MlpDev& M = A.model.m[s];
  const int L = M.n_layers, hl = L - 1;  // the last hidden layer
  const int K = M.width[hl];
  const float* w = M.W[L - 1];           // [n_out][K]
  const int ld = A.buf.ld[hl];
  const int64_t atom = valid ? A.perm[r] : 0;
  if (mode != 4) {
    for (int o = 0; o < A.n_out; ++o) {
      float e = 0.f;
      if (valid) {
        const float* ar = A.buf.a[hl] + r * ld;
        for (int k = sub; k < K; k += 16) e = fmaf(w[(int64_t)o * K + k], ar[k], e);
      }
#pragma unroll
      for (int x = 8; x > 0; x >>= 1) e += __shfl_xor(e, x, 16);
      if (valid && sub == 0) {
        if (mode == 3) A.out[atom * A.n_out + o] = e + M.b[L - 1][o];
        else A.E_atom[atom] = e + M.b[L - 1][0];
      }
    }
  }
  if (!valid || mode == 0 || mode == 3) return;
  const float* sr = A.buf.s[hl] + r * ld;
  float* dr = A.buf.d[hl] + r * ld;
  if (mode == 1) {
    for (int k = sub; k < K; k += 16) dr[k] = w[k] * sr[k];
  } else if (mode == 4) {
    const float* sd = A.seed + atom * A.n_out;
    for (int k = sub; k < K; k += 16) {
      float g = 0.f;
      for (int o = 0; o < A.n_out; ++o) g = fmaf(sd[o], w[(int64_t)o * K + k], g);
      dr[k] = g * sr[k];
    }
  } else {
    const float wa = A.w_atom[atom];
    const float* qr = A.buf.q[hl] + r * ld;
    float* tr = A.buf.dt[hl] + r * ld;
    for (int k = sub; k < K; k += 16) {
      dr[k] = w[k] * fmaf(wa, sr[k], -qr[k]);
      tr[k] = -w[k] * sr[k];
    }
  }
}

// ---------------------------------------------------------------------------
// backward through W[h-1] from hidden layer h: C = delta^h W^h (the
// contraction runs over the rows of W^h)
//   h >= 2: delta^(h-1) = C * act'(z^(h-1))          (TAN: the two adjoints)
//   h == 1: lambda of the atom = C                   (energy path only)
// ---------------------------------------------------------------------------

template <bool TAN>
__global__ void __launch_bounds__(64 * kLayWaves) k_lay_bwd(LayArgs A, int h) {
  __shared__ float red[TAN ? 2 : 1][kLayWaves][4][4][64];
  int s;
  int64_t r0, r1;
  if (!lay_tile(A.sp_start, A.model.S, blockIdx.x, s, r0, r1)) return;
  const MlpDev& M = A.model.m[s];
  if (M.n_layers - 1 < h) return;  // h is not a hidden layer of this species
  const int K = M.width[h], Nout = M.width[h - 1];
  const int c0 = (int)blockIdx.y * 64;
  if (c0 >= Nout) return;  // block-uniform
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
  const int64_t r = (r0 + lm < r1) ? r0 + lm : r0;
  const int ldh = A.buf.ld[h];
  const float* dr = A.buf.d[h] + r * ldh;
  const float* tr = TAN ? A.buf.dt[h] + r * ldh : nullptr;
  const float* W = M.W[h - 1];  // [K rows][Nout columns]
  floatx4 acc[4], acct[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = acct[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 16 * wv; k0 < K; k0 += 16 * kLayWaves) {
    const int k = k0 + 4 * lk;
    const float4 a = ld4(dr, k, K, true);
    float4 at{};
    if constexpr (TAN) at = ld4(tr, k, K, true);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = c0 + 16 * t + lm;
      float4 b{0.f, 0.f, 0.f, 0.f};
      if (n < Nout) {  // column n of rows k .. k + 3 of W^h: coalesced over the lanes lm
        const float* wc = W + (int64_t)k * Nout + n;
        b.x = k < K ? wc[0] : 0.f;
        b.y = k + 1 < K ? wc[Nout] : 0.f;
        b.z = k + 2 < K ? wc[2 * Nout] : 0.f;
        b.w = k + 3 < K ? wc[3 * Nout] : 0.f;
      }
      acc[t] = mma4_f32(acc[t], a, b);
      if constexpr (TAN) acct[t] = mma4_f32(acct[t], at, b);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      red[0][wv][t][j][lane] = acc[t][j];
      if constexpr (TAN) red[TAN ? 1 : 0][wv][t][j][lane] = acct[t][j];
    }
  __syncthreads();
  const int t = wv;
  const int n = c0 + 16 * t + lm;
  if (n >= Nout) return;
  const int ldp = A.buf.ld[h - 1];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t rr = r0 + 4 * lk + j;
    if (rr >= r1) continue;
    float cs = 0.f, cts = 0.f;
#pragma unroll
    for (int q = 0; q < kLayWaves; ++q) {
      cs += red[0][q][t][j][lane];
      if constexpr (TAN) cts += red[TAN ? 1 : 0][q][t][j][lane];
    }
    if (h == 1) {
      A.lambda[(int64_t)A.perm[rr] * A.D + n] = cs;
    } else if constexpr (TAN) {
      const float sp = A.buf.s[h - 1][rr * ldp + n], qp = A.buf.q[h - 1][rr * ldp + n];
      A.buf.d[h - 1][rr * ldp + n] = fmaf(cs, sp, cts * qp);
      A.buf.dt[h - 1][rr * ldp + n] = cts * sp;
    } else {
      A.buf.d[h - 1][rr * ldp + n] = cs * A.buf.s[h - 1][rr * ldp + n];
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: per chunk of one species' rows, per weight layer j and per
// 64 x 64 tile of [dW^(j+1) | db^(j+1)] (the bias is column Kin, whose
// operand is 1 for the first product and 0 for the tangent one):
//   partial = sum_rows  Zb[r][o] X[r][k]  (+ Zt[r][o] Xt[r][k] with TAN)
// Zb: w * delta (energy path) or z_bar (TAN) of layer j+1, and at the output
// w (Zt = -1); X: G (via perm) for j = 0, else a^j; Xt: u, a_dot^j.
// ---------------------------------------------------------------------------

// atoms per chunk: at least 128, and at most about 256 chunks
__host__ __device__ inline int64_t lay_chunk_rows(int64_t N) {
  const int64_t per = (N + 255) / 256;
  const int64_t c = (per + 127) / 128 * 128;
  return c > 128 ? c : 128;
}

// offset of layer j's [dW | db] inside a species' block of parameters
__device__ __forceinline__ int64_t lay_param_off(const MlpDev& M, int j) {
  int64_t o = 0;
  for (int q = 0; q < j; ++q) o += (int64_t)M.width[q + 1] * (M.width[q] + 1);
  return o;
}

__device__ __forceinline__ bool lay_chunk(const int64_t* __restrict__ sp_start, int S, int64_t chunk, int64_t c,
                                          int& s, int64_t& r0, int64_t& r1, int64_t& c_first) {
  int64_t first = 0;
  for (s = 0; s < S; ++s) {
    const int64_t ns = sp_start[s + 1] - sp_start[s];
    const int64_t nc = (ns + chunk - 1) / chunk;
    if (c < first + nc) {
      r0 = sp_start[s] + (c - first) * chunk;
      r1 = min(r0 + chunk, sp_start[s + 1]);
      c_first = first;
      return true;
    }
    first += nc;
  }
  return false;
}

template <bool TAN>
__global__ void __launch_bounds__(64 * kLayWaves) k_lay_wgrad(LayArgs A, int64_t chunk, int64_t per_chunk,
                                                              float* __restrict__ partial) {
  int s;
  int64_t r0, r1, cf;
  if (!lay_chunk(A.sp_start, A.model.S, chunk, blockIdx.x, s, r0, r1, cf)) return;
  const MlpDev& M = A.model.m[s];
  const int j = blockIdx.y;
  if (j >= M.n_layers) return;
  const int Kin = M.width[j], Nout = M.width[j + 1];
  const bool out_layer = j == M.n_layers - 1;
  const int nkt = (Kin + 1 + 63) / 64;  // k tiles, bias column included
  const int ot = (int)blockIdx.z / nkt, kt = (int)blockIdx.z % nkt;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
  const int o = ot * 64 + wv * 16 + lm;  // this lane's A row (output unit)
  if (ot * 64 + wv * 16 >= Nout) return;
  const int kc0 = kt * 64;
  const int h = j + 1;  // the layer whose adjoint is contracted
  const int ldh = out_layer ? 0 : A.buf.ld[h];
  floatx4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int64_t rb = r0; rb < r1; rb += 16) {
    float za[4], zt[4];
    float x[4][4], xt[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t rr = rb + 4 * lk + i;
      const bool rv = rr < r1;
      const int64_t atom = rv ? A.perm[rr] : 0;
      // A operand: Zb[rr][o] (and Zt)
      float zb = 0.f, zq = 0.f;
      if (rv && o < Nout) {
        if (out_layer) {
          zb = A.seed ? A.w_atom[atom] * A.seed[(int64_t)atom * A.n_out + o] : A.w_atom[atom];
          zq = -1.f;
        } else if constexpr (TAN) {
          zb = A.buf.d[h][rr * ldh + o];
          zq = A.buf.dt[h][rr * ldh + o];
        } else {
          zb = A.w_atom[atom] * A.buf.d[h][rr * ldh + o];
        }
      }
      za[i] = zb;
      zt[i] = zq;
      // B operands: X[rr][k] and Xt[rr][k] for the four column tiles
      const float *xrow = nullptr, *trow = nullptr;
      if (rv) {
        if (j == 0) {
          xrow = A.G + (int64_t)atom * A.D;
          if (TAN) trow = A.U + (int64_t)atom * A.D;
        } else {
          xrow = A.buf.a[j] + rr * A.buf.ld[j];
          if (TAN) trow = A.buf.at[j] + rr * A.buf.ld[j];
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = kc0 + 16 * t + lm;
        float xv = 0.f, tv = 0.f;
        if (rv) {
          if (k < Kin) {
            xv = xrow[k];
            if (TAN) tv = trow[k];
          } else if (k == Kin) {
            xv = 1.f;  // the bias column
          }
        }
        x[t][i] = xv;
        xt[t][i] = tv;
      }
    }
    const float4 a = make_float4(za[0], za[1], za[2], za[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mma4_f32(acc[t], a, make_float4(x[t][0], x[t][1], x[t][2], x[t][3]));
    if constexpr (TAN) {
      const float4 b = make_float4(zt[0], zt[1], zt[2], zt[3]);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mma4_f32(acc[t], b, make_float4(xt[t][0], xt[t][1], xt[t][2], xt[t][3]));
    }
  }
  // lane (lm, lk) holds output units ot*64 + wv*16 + 4 lk + q, column kc0 + 16 t + lm
  float* P = partial + (int64_t)blockIdx.x * per_chunk + lay_param_off(M, j);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kc0 + 16 * t + lm;
    if (k > Kin) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int oo = ot * 64 + wv * 16 + 4 * lk + q;
      if (oo >= Nout) continue;
      if (k < Kin) P[(int64_t)oo * Kin + k] = acc[t][q];
      else P[(int64_t)Nout * Kin + oo] = acc[t][q];
    }
  }
}

// dW, db of every species and layer: the chunk partials of the species added
// in chunk order (one thread per parameter), so the sums are reproducible.
__global__ void k_lay_wreduce(LayArgs A, int64_t chunk, int64_t per_chunk, const float* __restrict__ partial,
                              LayGradOut out) {
  const int s = blockIdx.y;
  if (s >= A.model.S) return;
  const MlpDev& M = A.model.m[s];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // this species' chunks: the ones before it are those of the species before it
  int64_t first = 0;
  for (int q = 0; q < s; ++q) first += (A.sp_start[q + 1] - A.sp_start[q] + chunk - 1) / chunk;
  const int64_t nc = (A.sp_start[s + 1] - A.sp_start[s] + chunk - 1) / chunk;
  int j = 0;
  for (; j < M.n_layers; ++j) {
    const int64_t n = (int64_t)M.width[j + 1] * (M.width[j] + 1);
    if (e < n) break;
    e -= n;
  }
  if (j >= M.n_layers) return;
  const int Kin = M.width[j], Nout = M.width[j + 1];
  const int64_t off = lay_param_off(M, j) + e;
  float acc = 0.f;
  for (int64_t c = 0; c < nc; ++c) acc += partial[(first + c) * per_chunk + off];
  float* dW = out.dW[s * NN_MAX_LAYERS + j];
  float* db = out.db[s * NN_MAX_LAYERS + j];
  if (e < (int64_t)Nout * Kin) {
    if (dW) dW[e] = acc;
  } else if (db) {
    db[e - (int64_t)Nout * Kin] = acc;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int max_hidden(const ModelDev& m) {
  int h = 0;
  for (int s = 0; s < m.S; ++s) h = std::max(h, m.m[s].n_layers - 1);
  return h;
}

// largest output width of weight layer j (j = h - 1 for hidden layer h) over the species that have it
static int max_width(const ModelDev& m, int l) {
  int w = 0;
  for (int s = 0; s < m.S; ++s)
    if (l <= m.m[s].n_layers) w = std::max(w, m.m[s].width[l]);
  return w;
}

void lay_stash_widths(const ModelDev& m, int ld[NN_MAX_LAYERS]) {
  for (int h = 0; h < NN_MAX_LAYERS; ++h) ld[h] = 0;
  const int H = max_hidden(m);
  for (int h = 1; h <= H; ++h) {
    int w = 0;
    for (int s = 0; s < m.S; ++s)
      if (h < m.m[s].n_layers) w = std::max(w, m.m[s].width[h]);
    ld[h] = (w + 15) / 16 * 16;
  }
}

int64_t lay_params_max(const ModelDev& m) {
  int64_t best = 0;
  for (int s = 0; s < m.S; ++s) {
    int64_t n = 0;
    for (int j = 0; j < m.m[s].n_layers; ++j) n += (int64_t)m.m[s].width[j + 1] * (m.m[s].width[j] + 1);
    best = std::max(best, n);
  }
  return (best + 63) / 64 * 64;
}

size_t lay_partial_floats(int64_t N, const ModelDev& m) {
  const int64_t chunks = N / lay_chunk_rows(N) + m.S + 1;
  return (size_t)(chunks * lay_params_max(m));
}

static unsigned lay_row_tiles(int64_t N, int S) { return (unsigned)((N + kLayRows - 1) / kLayRows + S); }

void launch_mlp_layers(const LayArgs& a, int64_t N, bool lambda, hipStream_t s) {
  if (N == 0) return;
  const int H = max_hidden(a.model);
  const unsigned rt = lay_row_tiles(N, a.model.S);
  for (int h = 1; h <= H; ++h) {
    const unsigned ct = (unsigned)((max_width(a.model, h) + 63) / 64);
    hipLaunchKernelGGL(k_lay_fwd<false>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
  hipLaunchKernelGGL(k_lay_out, dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, a, lambda ? 1 : 0);
  if (!lambda) return;
  for (int h = H; h >= 1; --h) {
    const unsigned ct = (unsigned)((max_width(a.model, h - 1) + 63) / 64);
    hipLaunchKernelGGL(k_lay_bwd<false>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
}

void launch_mlp_layers_outputs(const LayArgs& a, int64_t N, hipStream_t s) {
  if (N == 0) return;
  const int H = max_hidden(a.model);
  const unsigned rt = lay_row_tiles(N, a.model.S);
  for (int h = 1; h <= H; ++h) {
    const unsigned ct = (unsigned)((max_width(a.model, h) + 63) / 64);
    hipLaunchKernelGGL(k_lay_fwd<false>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
  hipLaunchKernelGGL(k_lay_out, dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, a, 3);
}

void launch_mlp_layers_seeded_backward(const LayArgs& a, int64_t N, bool lambda, hipStream_t s) {
  if (N == 0) return;
  const int H = max_hidden(a.model);
  const unsigned rt = lay_row_tiles(N, a.model.S);
  hipLaunchKernelGGL(k_lay_out, dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, a, 4);
  for (int h = H; h >= (lambda ? 1 : 2); --h) {
    const unsigned ct = (unsigned)((max_width(a.model, h - 1) + 63) / 64);
    hipLaunchKernelGGL(k_lay_bwd<false>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
}

void launch_mlp_layers_tangent(const LayArgs& a, int64_t N, hipStream_t s) {
  if (N == 0) return;
  const int H = max_hidden(a.model);
  const unsigned rt = lay_row_tiles(N, a.model.S);
  for (int h = 1; h <= H; ++h) {
    const unsigned ct = (unsigned)((max_width(a.model, h) + 63) / 64);
    hipLaunchKernelGGL(k_lay_fwd<true>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
  hipLaunchKernelGGL(k_lay_out, dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, a, 2);
  for (int h = H; h >= 2; --h) {
    const unsigned ct = (unsigned)((max_width(a.model, h - 1) + 63) / 64);
    hipLaunchKernelGGL(k_lay_bwd<true>, dim3(rt, ct), dim3(64 * kLayWaves), 0, s, a, h);
  }
}

void launch_lay_wgrad(const LayArgs& a, int64_t N, bool tangent, float* partial, const LayGradOut& out, hipStream_t s) {
  if (N == 0) return;
  const int64_t chunk = lay_chunk_rows(N);
  const int64_t per_chunk = lay_params_max(a.model);
  const unsigned chunks = (unsigned)(N / chunk + a.model.S + 1);
  int L = 0, tiles = 0;
  for (int sp = 0; sp < a.model.S; ++sp) {
    const MlpDev& M = a.model.m[sp];
    L = std::max(L, M.n_layers);
    for (int j = 0; j < M.n_layers; ++j)
      tiles = std::max(tiles, ((M.width[j + 1] + 63) / 64) * ((M.width[j] + 1 + 63) / 64));
  }
  const dim3 g(chunks, (unsigned)L, (unsigned)tiles);
  if (tangent) hipLaunchKernelGGL(k_lay_wgrad<true>, g, dim3(64 * kLayWaves), 0, s, a, chunk, per_chunk, partial);
  else hipLaunchKernelGGL(k_lay_wgrad<false>, g, dim3(64 * kLayWaves), 0, s, a, chunk, per_chunk, partial);
  const unsigned rb = (unsigned)((per_chunk + 255) / 256);
  hipLaunchKernelGGL(k_lay_wreduce, dim3(rb, (unsigned)a.model.S), dim3(256), 0, s, a, chunk, per_chunk, partial, out);
}

}  // namespace nnp
