// Per-species MLP of Eq. (1) (Sec. II.A) on MFMA, fused forward + backward.
//
// Atoms are grouped by species (stable counting sort), then one wave takes a
// tile of 16 atoms of one species through
//   z1 = W1 G + b1, a1 = act(z1);  z2 = W2 a1 + b2, a2 = act(z2);
//   E = w3 . a2 + b3;
//   delta2 = w3 * act'(z2);  delta1 = (W2^T delta2) * act'(z1);
//   lambda = W1^T delta1 = dE/dG.
// The two hidden layers run on 16x16 MFMA tiles (FP32: 16x16x4, BF16:
// 16x16x32 with FP32 accumulation); the width-1 output layer is a dot
// product.  act'(z) stays in registers in the MFMA output layout, where the
// backward pass needs it elementwise; activations and deltas pass through
// LDS to become the next product's row operand.
#include <math.h>

#include "common.h"
#include "mlp_ops.h"

namespace nnp {

constexpr int kTile = 16;

// ---------------------------------------------------------------------------
// species grouping: perm lists atoms species by species, in atom order
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(64) k_sp_count(const int32_t* __restrict__ species, int64_t N, int S, int64_t nblk,
                                                 int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int sp = i < N ? species[i] : -1;
  for (int s = 0; s < S; ++s) {
    uint64_t m = __ballot(sp == s);
    if (threadIdx.x == 0) cnt[(int64_t)s * nblk + blockIdx.x] = __popcll(m);
  }
}

__global__ void __launch_bounds__(64) k_sp_scatter(const int32_t* __restrict__ species, int64_t N, int S, int64_t nblk,
                                                   const int64_t* __restrict__ off, int32_t* __restrict__ perm,
                                                   int64_t* __restrict__ sp_start) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int sp = i < N ? species[i] : -1;
  const int lane = threadIdx.x;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int s = 0; s < S; ++s) {
    uint64_t m = __ballot(sp == s);
    if (sp == s) perm[off[(int64_t)s * nblk + blockIdx.x] + __popcll(m & lt)] = (int32_t)i;
  }
  if (blockIdx.x == 0 && lane <= S) sp_start[lane] = off[(int64_t)lane * nblk];
}

// The same grouping in one block for N <= kSpSmall: each thread counts the
// species of a contiguous run of atoms, the runs' counts are scanned per
// species, and each thread then places its run.
constexpr int kSpThreads = 1024;
constexpr int64_t kSpSmall = 64 * 1024;

__global__ void __launch_bounds__(kSpThreads) k_sp_group_small(const int32_t* __restrict__ species, int64_t N, int S,
                                                               int32_t* __restrict__ perm,
                                                               int64_t* __restrict__ sp_start) {
  constexpr int NW = kSpThreads / 64;
  __shared__ int wtot[NW][NN_MAX_SPECIES];
  __shared__ int64_t start[NN_MAX_SPECIES + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t per = (N + kSpThreads - 1) / kSpThreads;
  const int64_t b = (int64_t)t * per, e = min(b + per, N);
  int cnt[NN_MAX_SPECIES], incl[NN_MAX_SPECIES];
#pragma unroll
  for (int q = 0; q < NN_MAX_SPECIES; ++q) cnt[q] = 0;
  for (int64_t k = b; k < e; ++k) {
    const int sp = species[k];
#pragma unroll
    for (int q = 0; q < NN_MAX_SPECIES; ++q) cnt[q] += (sp == q && q < S) ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < NN_MAX_SPECIES; ++q) {
    int x = cnt[q];
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(x, off);
      if (lane >= off) x += v;
    }
    incl[q] = x;
    if (lane == 63) wtot[w][q] = x;
  }
  __syncthreads();
  if (t < NN_MAX_SPECIES) {  // thread q: exclusive scan of species q over the waves
    int run = 0;
    for (int v = 0; v < NW; ++v) {
      const int x = wtot[v][t];
      wtot[v][t] = run;
      run += x;
    }
    start[t + 1] = run;  // species total for now
  }
  __syncthreads();
  if (t == 0) {
    start[0] = 0;
    for (int q = 0; q < NN_MAX_SPECIES; ++q) start[q + 1] = start[q] + (q < S ? start[q + 1] : 0);
  }
  __syncthreads();
  int64_t at[NN_MAX_SPECIES];
#pragma unroll
  for (int q = 0; q < NN_MAX_SPECIES; ++q) at[q] = start[q] + wtot[w][q] + incl[q] - cnt[q];
  for (int64_t k = b; k < e; ++k) {
    const int sp = species[k];
#pragma unroll
    for (int q = 0; q < NN_MAX_SPECIES; ++q)
      if (sp == q && q < S) perm[at[q]++] = (int32_t)k;
  }
  if (t <= S) sp_start[t] = start[t];
}

// ---------------------------------------------------------------------------
// fused MLP tile kernel
// ---------------------------------------------------------------------------


// A fragment (row lm, 8 consecutive k from kb) of a row-major FP32 LDS buffer.
template <int MODE>
__device__ __forceinline__ void a_frag_lds(const float* buf, int ld, int lm, int kb, bf16x8& hi, bf16x8& lo) {
  float x[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) x[q] = buf[lm * ld + kb + q];
  if constexpr (MODE == kBf16x3) split8(x, hi, lo);
  else
#pragma unroll
    for (int q = 0; q < 8; ++q) hi[q] = (__bf16)x[q];
}

// B fragment: 8 consecutive BF16 values at p (hi) and p_lo (lo), zero past n.
template <int MODE>
__device__ __forceinline__ void b_frag(const __bf16* p, const __bf16* p_lo, int avail, bf16x8& hi, bf16x8& lo) {
  if (avail >= 8) {
    hi = *reinterpret_cast<const bf16x8*>(p);
    if constexpr (MODE == kBf16x3) lo = *reinterpret_cast<const bf16x8*>(p_lo);
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      hi[q] = q < avail ? p[q] : (__bf16)0.f;
      if constexpr (MODE == kBf16x3) lo[q] = q < avail ? p_lo[q] : (__bf16)0.f;
    }
  }
}

// One 16-atom tile per block of NW waves.  Wave w owns the 16-column
// output tiles n = w, w + NW, ... of every product, so act'(z) of its
// layer-1 and layer-2 tiles stays in its registers; activations and deltas
// are exchanged through two LDS buffers.
template <int H1T, int H2T, int MODE, int NW>
__global__ void __launch_bounds__(64 * NW) k_mlp(MlpArgs args) {
  constexpr int kWaves = NW;
  constexpr int H1 = H1T * 16, H2 = H2T * 16;
  constexpr int HM = H1 > H2 ? H1 : H2;
  constexpr bool BF = MODE != kFp32;
  constexpr int LD = HM + 4;
  constexpr int T1 = (H1T + kWaves - 1) / kWaves, T2 = (H2T + kWaves - 1) / kWaves;
  __shared__ __align__(16) float buf[2][kTile * LD];
  __shared__ float epart[kWaves][kTile];
  __shared__ int32_t rows[kTile];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile tests become scalar branches
  const int S = args.model.S;
  // which species / tile
  int64_t t = blockIdx.x;
  int s = 0;
  int64_t r0 = 0, ns = 0;
  for (; s < S; ++s) {
    ns = args.sp_start[s + 1] - args.sp_start[s];
    const int64_t nt = (ns + kTile - 1) / kTile;
    if (t < nt) break;
    t -= nt;
  }
  if (s >= S) return;
  r0 = args.sp_start[s] + t * kTile;
  const int nrows = (int)min<int64_t>(kTile, args.sp_start[s] + ns - r0);
  if (tid < kTile) rows[tid] = tid < nrows ? args.perm[r0 + tid] : -1;
  __syncthreads();
  const MlpDev& M = args.model.m[s];
  const int D = args.D;
  const int lm = lane & 15;   // row (A operand) / column (B, C)
  const int lk = lane >> 4;   // k group (A, B) / row group (C)
  const int arow = rows[lm];
  const float* Grow = args.G + (int64_t)(arow < 0 ? 0 : arow) * D;
  const int act1 = M.act[0], act2 = M.act[1];
  bf16x8 ah{}, al{}, bh{}, bl{};
  float* bufA = buf[0];
  float* bufB = buf[1];
  // FP32 with 16-byte aligned G and weights and D a multiple of 32: every
  // operand load is an unguarded vector or scalar load, so each product
  // can issue all of its weight loads before its first MFMA
  // (shapes whose prefetch buffers fit in 192 registers per lane)
  constexpr int kPre = (H1 / 16) * T2 * 4 + (H2 / 16) * T1 * 4 + 2 * (H1 / 16) * 4;
  constexpr bool kFastOK = !BF && kPre <= 192;
  const bool fast = kFastOK && D % 32 == 0 &&
                    ((((uintptr_t)args.G) | ((uintptr_t)M.W[0]) | ((uintptr_t)M.W[1])) & 15) == 0;
  constexpr int KB1 = kFastOK ? H1 / 16 : 1, KB2 = kFastOK ? H2 / 16 : 1;
  float4 w2f[KB1][T2];     // layer 2: B fragments of W2 [H2][H1] (rows n, 4 consecutive k)
  float w2t[KB2][T1][4];   // delta1: B fragments of W2 read by columns
  float w1t[2][KB1][4];    // lambda: B fragments of W1 read by columns, two column tiles
  auto prefetch_w2 = [&]() {
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
      for (int u = 0; u < T2; ++u) {
        const int n = wv + kWaves * u;
        w2f[kb][u] = *reinterpret_cast<const float4*>(M.W[1] + (int64_t)((n < H2T ? n : 0) * 16 + lm) * H1 +
                                                      16 * kb + 4 * lk);
      }
  };
  auto prefetch_w2t = [&]() {
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb) {
      const float* w = M.W[1] + (int64_t)(16 * kb + 4 * lk) * H1 + lm;
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + kWaves * u;
        const int c = (n < H1T ? n : 0) * 16;
#pragma unroll
        for (int i = 0; i < 4; ++i) w2t[kb][u][i] = w[i * H1 + c];
      }
    }
  };
  auto prefetch_w1t = [&](int tile, int slot) {  // column tile `tile` of lambda (tile < D / 16)
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      const float* w = M.W[0] + (int64_t)(16 * kb + 4 * lk) * D + tile * 16 + lm;
#pragma unroll
      for (int i = 0; i < 4; ++i) w1t[slot][kb][i] = w[i * D];
    }
  };

  // ---- layer 1: z1 = G W1^T + b1 (this wave's tiles n = wv + kWaves * u) ----
  floatx4 acc1[T1];
#pragma unroll
  for (int u = 0; u < T1; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
    for (int k0 = 0; k0 < D; k0 += 32) {
      const int kb = k0 + 8 * lk;
      float x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = (arow >= 0 && kb + q < D) ? Grow[kb + q] : 0.f;
      if constexpr (MODE == kBf16x3) split8(x, ah, al);
      else
#pragma unroll
        for (int q = 0; q < 8; ++q) ah[q] = (__bf16)x[q];
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + kWaves * u;
        if (n < H1T) {
          const int64_t off = (int64_t)(n * 16 + lm) * D + kb;
          b_frag<MODE>(M.Wb[0] + off, M.Wl[0] + off, D - kb, bh, bl);
          acc1[u] = mma_bf16<MODE>(acc1[u], ah, al, bh, bl);
        }
      }
    }
  } else if (fast) {
    // weights of the next two products are requested now and arrive while
    // this one runs; the k steps of this one are double-buffered
    prefetch_w2();
    // rows past the tile's atoms read row 0 of G (Grow): every product is
    // row by row and such rows are never stored, so their values do not matter
    const float* w1row[T1];
#pragma unroll
    for (int u = 0; u < T1; ++u) {
      const int n = wv + kWaves * u;
      w1row[u] = M.W[0] + (int64_t)((n < H1T ? n : 0) * 16 + lm) * D;
    }
    float4 xa[2], xb[2][T1], ya[2], yb[2][T1];  // two k steps in flight
    auto fetch = [&](int k0, float4(&a)[2], float4(&b)[2][T1]) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = k0 + 16 * q + 4 * lk;
        a[q] = *reinterpret_cast<const float4*>(Grow + k);
#pragma unroll
        for (int u = 0; u < T1; ++u) b[q][u] = *reinterpret_cast<const float4*>(w1row[u] + k);
      }
    };
    auto step = [&](const float4(&a)[2], const float4(&b)[2][T1]) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < T1; ++u)
          if (H1T % kWaves == 0 || wv + kWaves * u < H1T) acc1[u] = mma4_f32(acc1[u], a[q], b[q][u]);
    };
    fetch(0, xa, xb);
    for (int k0 = 0; k0 < D; k0 += 64) {
      if (k0 + 32 < D) fetch(k0 + 32, ya, yb);
      step(xa, xb);
      if (k0 + 32 >= D) break;
      if (k0 + 64 < D) fetch(k0 + 64, xa, xb);
      step(ya, yb);
    }
  } else {
    const float* W1 = M.W[0];
    const bool vec = ((((uintptr_t)W1) | ((uintptr_t)args.G)) & 15) == 0 && (D & 3) == 0;
    for (int k0 = 0; k0 < D; k0 += 32) {
      float4 a[2], b[2][T1];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = k0 + 16 * q + 4 * lk;
        a[q] = ld4(Grow, k, arow >= 0 ? D : 0, vec);
#pragma unroll
        for (int u = 0; u < T1; ++u) {
          const int n = wv + kWaves * u;
          b[q][u] = ld4(W1 + (int64_t)(n < H1T ? n * 16 + lm : 0) * D, k, n < H1T ? D : 0, vec);
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < T1; ++u)
          if (wv + kWaves * u < H1T) acc1[u] = mma4_f32(acc1[u], a[q], b[q][u]);
    }
  }
  float d1[T1][4];  // act'(z1) in C layout: row 4*lk + j, column n*16 + lm
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    const int n = wv + kWaves * u;
    if (n >= H1T) continue;
    const float bias = M.b[0][n * 16 + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc1[u][j] + bias;
      const float a = act_f(act1, z);
      d1[u][j] = act_d(act1, z, a);
      bufA[(4 * lk + j) * LD + n * 16 + lm] = a;
      if (args.st_a1) {
        const int r = rows[4 * lk + j];
        if (r >= 0) args.st_a1[(int64_t)r * H1 + n * 16 + lm] = a;
      }
    }
  }
  __syncthreads();

  // ---- layer 2: z2 = a1 W2^T + b2 ----
  floatx4 acc2[T2];
#pragma unroll
  for (int u = 0; u < T2; ++u) acc2[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
    for (int k0 = 0; k0 < H1; k0 += 32) {
      const int kb = k0 + 8 * lk;
      a_frag_lds<MODE>(bufA, LD, lm, kb, ah, al);
#pragma unroll
      for (int u = 0; u < T2; ++u) {
        const int n = wv + kWaves * u;
        if (n < H2T) {
          const int64_t off = (int64_t)(n * 16 + lm) * H1 + kb;
          b_frag<MODE>(M.Wb[1] + off, M.Wl[1] + off, 8, bh, bl);
          acc2[u] = mma_bf16<MODE>(acc2[u], ah, al, bh, bl);
        }
      }
    }
  } else if (fast) {
    if (args.lambda != nullptr || args.st_d1 != nullptr) prefetch_w2t();
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
      const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + 16 * kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < T2; ++u)
        if (H2T % kWaves == 0 || wv + kWaves * u < H2T) acc2[u] = mma4_f32(acc2[u], a, w2f[kb][u]);
    }
  } else {
    const float* W2 = M.W[1];
    const bool vec = (((uintptr_t)W2) & 15) == 0;
#pragma unroll
    for (int kb = 0; kb < H1; kb += 16) {
      const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < T2; ++u) {
        const int n = wv + kWaves * u;
        if (n < H2T) acc2[u] = mma4_f32(acc2[u], a, ld4(W2 + (int64_t)(n * 16 + lm) * H1, kb + 4 * lk, H1, vec));
      }
    }
  }
  // ---- output E = w3 . a2 + b3, delta2 = w3 * act'(z2) ----
  const float* w3 = M.W[2];
  float e[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < T2; ++u) {
    const int n = wv + kWaves * u;
    if (n >= H2T) continue;
    const float bias = M.b[1][n * 16 + lm];
    const float w = w3[n * 16 + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc2[u][j] + bias;
      const float a = act_f(act2, z);
      e[j] = fmaf(a, w, e[j]);
      const float dl2 = w * act_d(act2, z, a);
      bufB[(4 * lk + j) * LD + n * 16 + lm] = dl2;
      if (args.st_a2) {
        const int r = rows[4 * lk + j];
        if (r >= 0) {
          args.st_a2[(int64_t)r * H2 + n * 16 + lm] = a;
          args.st_d2[(int64_t)r * H2 + n * 16 + lm] = dl2;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = e[j];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    e[j] = v;
  }
  if (lm == 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) epart[wv][4 * lk + j] = e[j];
  __syncthreads();
  if (tid < kTile) {
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += epart[w][tid];
    const int r = rows[tid];
    if (r >= 0) args.E_atom[r] = v + M.b[2][0];
  }
  if (args.lambda == nullptr && args.st_d1 == nullptr) return;
  // ---- delta1 = (delta2 W2) * act'(z1), this wave's layer-1 tiles ----
#pragma unroll
  for (int u = 0; u < T1; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
    for (int k0 = 0; k0 < H2; k0 += 32) {  // B = W2 [H2][H1] read through W2^T [H1][H2]
      const int kb = k0 + 8 * lk;
      a_frag_lds<MODE>(bufB, LD, lm, kb, ah, al);
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + kWaves * u;
        if (n < H1T) {
          const int64_t off = (int64_t)(n * 16 + lm) * H2 + kb;
          b_frag<MODE>(M.WbT[1] + off, M.WlT[1] + off, 8, bh, bl);
          acc1[u] = mma_bf16<MODE>(acc1[u], ah, al, bh, bl);
        }
      }
    }
  } else if (fast) {
    if (args.lambda != nullptr && wv < D / 16) prefetch_w1t(wv, 0);
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb) {
      const float4 a = *reinterpret_cast<const float4*>(bufB + lm * LD + 16 * kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < T1; ++u)
        if (H1T % kWaves == 0 || wv + kWaves * u < H1T)
          acc1[u] = mma4_f32(acc1[u], a, make_float4(w2t[kb][u][0], w2t[kb][u][1], w2t[kb][u][2], w2t[kb][u][3]));
    }
  } else {
    const float* W2 = M.W[1];  // [H2][H1]: B[k][n] = W2[k][n]
#pragma unroll
    for (int kb = 0; kb < H2; kb += 16) {
      const float4 a = *reinterpret_cast<const float4*>(bufB + lm * LD + kb + 4 * lk);
      const float* w = W2 + (int64_t)(kb + 4 * lk) * H1 + lm;
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + kWaves * u;
        if (n < H1T) {
          float4 b;
          b.x = w[n * 16];
          b.y = w[H1 + n * 16];
          b.z = w[2 * H1 + n * 16];
          b.w = w[3 * H1 + n * 16];
          acc1[u] = mma4_f32(acc1[u], a, b);
        }
      }
    }
  }
  // bufA (a1) is no longer read by anyone after the layer-2 products, which
  // every wave finished before the barrier above
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    const int n = wv + kWaves * u;
    if (n >= H1T) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dd = acc1[u][j] * d1[u][j];
      bufA[(4 * lk + j) * LD + n * 16 + lm] = dd;
      if (args.st_d1) {
        const int r = rows[4 * lk + j];
        if (r >= 0) args.st_d1[(int64_t)r * H1 + n * 16 + lm] = dd;
      }
    }
  }
  if (args.lambda == nullptr) return;
  __syncthreads();
  // ---- lambda = delta1 W1: D columns, 16-column tiles dealt to the waves ----
  const int DT = (D + 15) / 16;
  if constexpr (!BF) {
    if (fast) {
      // tile wv was requested before the delta1 products; each tile's
      // loads are issued before the previous tile's products
      for (int tile = wv; tile < DT; tile += kWaves) {
        const bool more = tile + kWaves < DT;
        if (more) prefetch_w1t(tile + kWaves, 1);
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
          const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + 16 * kb + 4 * lk);
          acc = mma4_f32(acc, a, make_float4(w1t[0][kb][0], w1t[0][kb][1], w1t[0][kb][2], w1t[0][kb][3]));
        }
        const int col = tile * 16 + lm;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rows[4 * lk + j];
          if (r >= 0) args.lambda[(int64_t)r * D + col] = acc[j];
        }
        if (more)
#pragma unroll
          for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) w1t[0][kb][i] = w1t[1][kb][i];
      }
      return;
    }
  }
  constexpr int CH = 4;
  for (int c0 = wv; c0 < DT; c0 += kWaves * CH) {
    floatx4 acc[CH];
#pragma unroll
    for (int n = 0; n < CH; ++n) acc[n] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (BF) {
      for (int k0 = 0; k0 < H1; k0 += 32) {  // B = W1 [H1][D] read through W1^T [D][H1]
        const int kb = k0 + 8 * lk;
        a_frag_lds<MODE>(bufA, LD, lm, kb, ah, al);
#pragma unroll
        for (int n = 0; n < CH; ++n) {
          if (c0 + n * kWaves >= DT) continue;  // no column tile here (the same for the whole wave)
          const int col = (c0 + n * kWaves) * 16 + lm;
          const int64_t off = (int64_t)(col < D ? col : 0) * H1 + kb;
          b_frag<MODE>(M.WbT[0] + off, M.WlT[0] + off, col < D ? 8 : 0, bh, bl);
          acc[n] = mma_bf16<MODE>(acc[n], ah, al, bh, bl);
        }
      }
    } else {
      const float* W1 = M.W[0];  // [H1][D]: B[k][n] = W1[k][n]
#pragma unroll
      for (int kb = 0; kb < H1; kb += 16) {
        const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + kb + 4 * lk);
        const float* w = W1 + (int64_t)(kb + 4 * lk) * D;
#pragma unroll
        for (int n = 0; n < CH; ++n) {
          if (c0 + n * kWaves >= DT) continue;  // no column tile here (the same for the whole wave)
          const int col = (c0 + n * kWaves) * 16 + lm;
          float4 b = {0.f, 0.f, 0.f, 0.f};
          if (col < D) {
            b.x = w[col];
            b.y = w[D + col];
            b.z = w[2 * D + col];
            b.w = w[3 * D + col];
          }
          acc[n] = mma4_f32(acc[n], a, b);
        }
      }
    }
#pragma unroll
    for (int n = 0; n < CH; ++n) {
      const int col = (c0 + n * kWaves) * 16 + lm;
      if (col < D) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rows[4 * lk + j];
          if (r >= 0) args.lambda[(int64_t)r * D + col] = acc[n][j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// MLP with its tangent, for the weight gradient of a loss on forces
// ---------------------------------------------------------------------------

// With the per-atom weight w = dL/dE of the atom's structure and the
// descriptor tangent u (the derivative of G along dL/dF), the loss is
// L = sum_i (w_i E_i - E_dot_i) where E_dot = lambda . u is the forward-mode
// derivative of the MLP along u.  One 16-atom tile per block of NW waves
// (FP32 MFMA) computes
//   z1 = W1 G + b1, z1_dot = W1 u, a1 = act(z1), a1_dot = act'(z1) z1_dot,
//   z2 = W2 a1 + b2, z2_dot = W2 a1_dot, a2, a2_dot likewise, E = w3 . a2 + b3,
// then the reverse pass of w E - E_dot:
//   delta2 = w3 act'(z2),  eps2 = w3 act''(z2) z2_dot,
//   delta1 = act'(z1) (W2^T delta2),
//   eps1 = act''(z1) z1_dot (W2^T delta2) + act'(z1) (W2^T eps2),
// and stashes per atom what the weight-gradient sums contract:
//   x1 = w delta1 - eps1 (with G), delta1 (with -u), a1 and a1_dot,
//   x2 = w delta2 - eps2 (with a1), delta2 (with -a1_dot),
//   c3 = w a2 - a2_dot (the output-layer column).
template <int H1T, int H2T, int NW>
__global__ void __launch_bounds__(64 * NW) k_mlp_fm(MlpFmArgs args) {
  constexpr int H1 = H1T * 16, H2 = H2T * 16;
  constexpr int HM = H1 > H2 ? H1 : H2;
  constexpr int LD = HM + 4;
  constexpr int T1 = (H1T + NW - 1) / NW, T2 = (H2T + NW - 1) / NW;
  __shared__ __align__(16) float buf[2][kTile * LD];
  __shared__ float epart[NW][kTile];
  __shared__ int32_t rows[kTile];
  __shared__ float wrow[kTile];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int S = args.model.S;
  int64_t t = blockIdx.x;
  int s = 0;
  int64_t ns = 0;
  for (; s < S; ++s) {
    ns = args.sp_start[s + 1] - args.sp_start[s];
    const int64_t nt = (ns + kTile - 1) / kTile;
    if (t < nt) break;
    t -= nt;
  }
  if (s >= S) return;
  const int64_t r0 = args.sp_start[s] + t * kTile;
  const int nrows = (int)min<int64_t>(kTile, args.sp_start[s] + ns - r0);
  if (tid < kTile) {
    const int r = tid < nrows ? args.perm[r0 + tid] : -1;
    rows[tid] = r;
    wrow[tid] = r >= 0 ? args.w[r] : 0.f;
  }
  __syncthreads();
  const MlpDev& M = args.model.m[s];
  const int D = args.D;
  const int lm = lane & 15, lk = lane >> 4;
  const int arow = rows[lm];
  const float* Grow = args.G + (int64_t)(arow < 0 ? 0 : arow) * D;
  const float* Urow = args.U + (int64_t)(arow < 0 ? 0 : arow) * D;
  const int act1 = M.act[0], act2 = M.act[1];
  float* bufA = buf[0];
  float* bufB = buf[1];
  auto stash = [&](float* dst, int ld, int col, int j, float v) {
    const int r = rows[4 * lk + j];
    if (r >= 0) dst[(int64_t)r * ld + col] = v;
  };

  // ---- layer 1: z1 = G W1^T, z1_dot = u W1^T (shared B fragments) ----
  floatx4 acc[T1], acct[T1];
#pragma unroll
  for (int u = 0; u < T1; ++u) acc[u] = acct[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  {
    const float* W1 = M.W[0];
    const bool vec = ((((uintptr_t)W1) | ((uintptr_t)args.G) | ((uintptr_t)args.U)) & 15) == 0 && (D & 3) == 0;
    for (int k0 = 0; k0 < D; k0 += 16) {
      const int k = k0 + 4 * lk;
      const float4 a = ld4(Grow, k, arow >= 0 ? D : 0, vec);
      const float4 at = ld4(Urow, k, arow >= 0 ? D : 0, vec);
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + NW * u;
        if (n < H1T) {
          const float4 b = ld4(W1 + (int64_t)(n * 16 + lm) * D, k, D, vec);
          acc[u] = mma4_f32(acc[u], a, b);
          acct[u] = mma4_f32(acct[u], at, b);
        }
      }
    }
  }
  float p1[T1][4], q1[T1][4];  // act'(z1) and act''(z1) z1_dot in C layout
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    const int n = wv + NW * u;
    if (n >= H1T) continue;
    const int col = n * 16 + lm;
    const float bias = M.b[0][col];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc[u][j] + bias, zt = acct[u][j];
      const float a = act_f(act1, z);
      const float d = act_d(act1, z, a);
      p1[u][j] = d;
      q1[u][j] = act_d2(act1, z, a) * zt;
      bufA[(4 * lk + j) * LD + col] = a;
      bufB[(4 * lk + j) * LD + col] = d * zt;
      stash(args.a1, H1, col, j, a);
      stash(args.t1, H1, col, j, d * zt);
    }
  }
  __syncthreads();

  // ---- layer 2: z2 = a1 W2^T, z2_dot = a1_dot W2^T ----
  floatx4 acc2[T2], acc2t[T2];
#pragma unroll
  for (int u = 0; u < T2; ++u) acc2[u] = acc2t[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  {
    const float* W2 = M.W[1];
    const bool vec = (((uintptr_t)W2) & 15) == 0;
#pragma unroll
    for (int kb = 0; kb < H1; kb += 16) {
      const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + kb + 4 * lk);
      const float4 at = *reinterpret_cast<const float4*>(bufB + lm * LD + kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < T2; ++u) {
        const int n = wv + NW * u;
        if (n < H2T) {
          const float4 b = ld4(W2 + (int64_t)(n * 16 + lm) * H1, kb + 4 * lk, H1, vec);
          acc2[u] = mma4_f32(acc2[u], a, b);
          acc2t[u] = mma4_f32(acc2t[u], at, b);
        }
      }
    }
  }
  __syncthreads();  // every wave is done reading a1 and a1_dot
  const float* w3 = M.W[2];
  float e[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < T2; ++u) {
    const int n = wv + NW * u;
    if (n >= H2T) continue;
    const int col = n * 16 + lm;
    const float bias = M.b[1][col];
    const float w = w3[col];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc2[u][j] + bias, zt = acc2t[u][j];
      const float a = act_f(act2, z);
      const float d = act_d(act2, z, a);
      const float wi = wrow[4 * lk + j];
      e[j] = fmaf(a, w, e[j]);
      const float dl2 = w * d;
      const float ep2 = w * act_d2(act2, z, a) * zt;
      bufA[(4 * lk + j) * LD + col] = dl2;
      bufB[(4 * lk + j) * LD + col] = ep2;
      stash(args.d2, H2, col, j, dl2);
      stash(args.x2, H2, col, j, fmaf(wi, dl2, -ep2));
      stash(args.c3, H2, col, j, fmaf(wi, a, -d * zt));
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = e[j];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    e[j] = v;
  }
  if (lm == 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) epart[wv][4 * lk + j] = e[j];
  __syncthreads();
  if (tid < kTile) {
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += epart[w][tid];
    const int r = rows[tid];
    if (r >= 0) args.E_atom[r] = v + M.b[2][0];
  }

  // ---- W2^T delta2 and W2^T eps2 (shared B fragments) ----
#pragma unroll
  for (int u = 0; u < T1; ++u) acc[u] = acct[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  {
    const float* W2 = M.W[1];  // [H2][H1]: B[k][n] = W2[k][n]
#pragma unroll
    for (int kb = 0; kb < H2; kb += 16) {
      const float4 a = *reinterpret_cast<const float4*>(bufA + lm * LD + kb + 4 * lk);
      const float4 at = *reinterpret_cast<const float4*>(bufB + lm * LD + kb + 4 * lk);
      const float* w = W2 + (int64_t)(kb + 4 * lk) * H1 + lm;
#pragma unroll
      for (int u = 0; u < T1; ++u) {
        const int n = wv + NW * u;
        if (n < H1T) {
          float4 b;
          b.x = w[n * 16];
          b.y = w[H1 + n * 16];
          b.z = w[2 * H1 + n * 16];
          b.w = w[3 * H1 + n * 16];
          acc[u] = mma4_f32(acc[u], a, b);
          acct[u] = mma4_f32(acct[u], at, b);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    const int n = wv + NW * u;
    if (n >= H1T) continue;
    const int col = n * 16 + lm;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float tv = acc[u][j];
      const float dl1 = p1[u][j] * tv;
      const float ep1 = fmaf(q1[u][j], tv, p1[u][j] * acct[u][j]);
      stash(args.d1, H1, col, j, dl1);
      stash(args.x1, H1, col, j, fmaf(wrow[4 * lk + j], dl1, -ep1));
    }
  }
}

template <int A, int B>
static void launch_mlp_fm_t(const MlpFmArgs& a, int64_t n_tiles, int waves, hipStream_t s) {
  if constexpr (A >= 8) {
    if (waves != 4) {
      hipLaunchKernelGGL((k_mlp_fm<A, B, 8>), dim3((unsigned)n_tiles), dim3(512), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_mlp_fm<A, B, 4>), dim3((unsigned)n_tiles), dim3(256), 0, s, a);
}

void launch_mlp_fm(const MlpFmArgs& a, int h1, int h2, int64_t N, int waves, hipStream_t s) {
  const int64_t n_tiles = (N + kTile - 1) / kTile + a.model.S;
  if (N == 0) return;
  if (h1 == 64 && h2 == 32) launch_mlp_fm_t<4, 2>(a, n_tiles, waves, s);
  else if (h1 == 128 && h2 == 128) launch_mlp_fm_t<8, 8>(a, n_tiles, waves, s);
  else if (h1 == 256 && h2 == 128) launch_mlp_fm_t<16, 8>(a, n_tiles, waves, s);
}

// ---------------------------------------------------------------------------
// BF16 weight copies: hi = bf16(W), lo = bf16(W - hi), each also transposed;
// one launch for all species and layers
// ---------------------------------------------------------------------------

__global__ void k_convert_bf16(ConvJob job) {
  for (int m = 0; m < job.n; ++m) {
    const int R = job.rows[m], Cc = job.cols[m];
    const int64_t total = (int64_t)R * Cc;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
      const int r = (int)(idx / Cc), c = (int)(idx % Cc);
      const float w = job.src[m][idx];
      const __bf16 h = (__bf16)w;
      const __bf16 l = (__bf16)(w - (float)h);
      job.hi[m][idx] = h;
      job.lo[m][idx] = l;
      job.hiT[m][(int64_t)c * R + r] = h;
      job.loT[m][(int64_t)c * R + r] = l;
    }
  }
}

// ---------------------------------------------------------------------------
// per-structure energy, FP64, fixed-order tree
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_energy_reduce(const float* __restrict__ E_atom,
                                                       const int64_t* __restrict__ atom_ptr, int64_t N,
                                                       double* __restrict__ E_struct) {
  energy_block_sum(E_atom, atom_ptr, N, blockIdx.x, E_struct);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_species_group(const int32_t* species, int64_t N, int S, int64_t* cnt, int64_t* off, int64_t* scan_tmp,
                          int32_t* perm, int64_t* sp_start, hipStream_t s) {
  if (N <= kSpSmall) {
    hipLaunchKernelGGL(k_sp_group_small, dim3(1), dim3(kSpThreads), 0, s, species, N, S, perm, sp_start);
    return;
  }
  const int64_t nblk = (N + 63) / 64 > 0 ? (N + 63) / 64 : 1;
  hipLaunchKernelGGL(k_sp_count, dim3((unsigned)nblk), dim3(64), 0, s, species, N, S, nblk, cnt);
  exclusive_scan_i64(cnt, off, (int64_t)S * nblk, scan_tmp, s, nullptr);
  hipLaunchKernelGGL(k_sp_scatter, dim3((unsigned)nblk), dim3(64), 0, s, species, N, S, nblk, off, perm, sp_start);
}

bool mlp_supported(int h1, int h2) {
  return (h1 == 64 && h2 == 32) || (h1 == 128 && h2 == 128) || (h1 == 256 && h2 == 128);
}

template <int A, int B, int NW>
static void launch_mlp_w(const MlpArgs& a, int mode, int64_t n_tiles, hipStream_t s) {
  const dim3 g((unsigned)n_tiles), b(64 * NW);
  if (mode == kBf16x3) hipLaunchKernelGGL((k_mlp<A, B, kBf16x3, NW>), g, b, 0, s, a);
  else if (mode == kBf16) hipLaunchKernelGGL((k_mlp<A, B, kBf16, NW>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_mlp<A, B, kFp32, NW>), g, b, 0, s, a);
}

// waves per tile: 4, or 8 when layer 1 has at least 8 tiles of 16 units
// (the default)
template <int A, int B>
static void launch_mlp_t(const MlpArgs& a, int mode, int64_t n_tiles, int waves, hipStream_t s) {
  if constexpr (A >= 8) {
    if (waves != 4) {
      launch_mlp_w<A, B, 8>(a, mode, n_tiles, s);
      return;
    }
  }
  launch_mlp_w<A, B, 4>(a, mode, n_tiles, s);
}

void launch_mlp(const MlpArgs& a, int h1, int h2, int mode, int64_t N, int waves, hipStream_t s) {
  const int64_t n_tiles = (N + kTile - 1) / kTile + a.model.S;
  if (N == 0) return;
  if (h1 == 64 && h2 == 32) launch_mlp_t<4, 2>(a, mode, n_tiles, waves, s);
  else if (h1 == 128 && h2 == 128) launch_mlp_t<8, 8>(a, mode, n_tiles, waves, s);
  else if (h1 == 256 && h2 == 128) launch_mlp_t<16, 8>(a, mode, n_tiles, waves, s);
}

void launch_convert_bf16(const ConvJob& job, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_bf16, dim3(256), dim3(256), 0, s, job);
}

void launch_energy_reduce(const float* E_atom, const int64_t* atom_ptr, int32_t B, int64_t N, double* E_struct,
                          hipStream_t s) {
  if (B == 0) return;
  hipLaunchKernelGGL(k_energy_reduce, dim3((unsigned)B), dim3(256), 0, s, E_atom, atom_ptr, N, E_struct);
}

}  // namespace nnp
