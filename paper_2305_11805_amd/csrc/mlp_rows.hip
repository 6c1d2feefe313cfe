// Per-species MLP of Eq. (1) (Sec. II.A), FP32, in row blocks: one block of
// four waves takes 64 atoms of one species and each wave carries 16 of them
// through the whole network (both hidden layers, the output, and the
// backward pass to lambda = dE/dG).  Every weight block a product needs is
// staged in LDS once per block and read by the four waves, so the weights
// are fetched once per 64 atoms; the tile kernel (mlp.hip) splits the
// hidden units over its waves and fetches them once per 16.
//
// Products (16x16x4 FP32 MFMA in the k-permuted form of mma4_f32; C layout:
// lane (lm, lk) holds rows 4 lk + j, column lm of a 16x16 tile):
//   P1  z1 = G W1^T       A: G rows (global), B: W1[:, k0:k0+KC] staged as [n][k]
//   P2  z2 = a1 W2^T      A: a1 (the wave's LDS rows), B: W2[:, k0:k0+KC] as [n][k]
//   P3  g1 = delta2 W2    A: delta2 (LDS rows), B: W2[k0:k0+KC, :] staged transposed as [n][k]
//   P4  lambda = delta1 W1  A: delta1 (LDS rows), B: W1[:, c0:c0+NC] staged transposed as [n][k]
// with delta2 = w3 act'(z2), delta1 = g1 act'(z1); E = w3 . a2 + b3.  Sums
// have a fixed order (k in increasing chunks), so results are the same on
// every run.
#include <math.h>

#include "common.h"
#include "mlp_ops.h"

namespace nnp {

constexpr int kRwWaves = 4;
constexpr int kRwAtoms = 16 * kRwWaves;

__device__ __forceinline__ void rw_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int H1T, int H2T>
struct RowsShape {
  static constexpr int H1 = 16 * H1T, H2 = 16 * H2T;
  static constexpr int HM = H1 > H2 ? H1 : H2;
  static constexpr int KC = 32;   // k (P1-P3) or column (P4) chunk of a staged block (LDS <= 64 KB)
  static constexpr int LDW = KC + 4;               // staged [n][k] rows of P1-P3
  static constexpr int LDT = H1 + 4;               // staged [n][k] rows of P4 (k over H1)
  static constexpr int LDA = HM + 4;               // the wave's activation rows
  static constexpr int WS1 = HM * LDW, WS4 = KC * LDT;
  static constexpr int WS = WS1 > WS4 ? WS1 : WS4;  // floats of the staging buffer
  static constexpr size_t lds = sizeof(float) * ((size_t)WS + (size_t)kRwWaves * 16 * LDA);
};

template <int H1T, int H2T>
__global__ void __launch_bounds__(64 * kRwWaves) k_mlp_rows(MlpArgs args) {
  using Sh = RowsShape<H1T, H2T>;
  constexpr int H1 = Sh::H1, H2 = Sh::H2, KC = Sh::KC, LDW = Sh::LDW, LDT = Sh::LDT, LDA = Sh::LDA;
  extern __shared__ float4 rw_lds4[];
  float* ws = reinterpret_cast<float*>(rw_lds4);
  __shared__ int32_t rows[kRwAtoms];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  float* abuf = ws + Sh::WS + wv * 16 * LDA;  // this wave's rows
  const int lm = lane & 15, lk = lane >> 4;
  // which species / block of 64 atoms
  const int S = args.model.S;
  int64_t t = blockIdx.x;
  int s = 0;
  int64_t ns = 0;
  for (; s < S; ++s) {
    ns = args.sp_start[s + 1] - args.sp_start[s];
    const int64_t nt = (ns + kRwAtoms - 1) / kRwAtoms;
    if (t < nt) break;
    t -= nt;
  }
  if (s >= S) return;
  const int64_t r0 = args.sp_start[s] + t * kRwAtoms;
  const int nrows = (int)min<int64_t>(kRwAtoms, args.sp_start[s] + ns - r0);
  if (tid < kRwAtoms) rows[tid] = tid < nrows ? args.perm[r0 + tid] : -1;
  __syncthreads();
  const MlpDev& M = args.model.m[s];
  const int D = args.D;
  const int act1 = M.act[0], act2 = M.act[1];
  // rows past the block's atoms compute on row 0 of G and are never stored
  const int arow = rows[16 * wv + lm];
  const float* Grow = args.G + (int64_t)(arow < 0 ? 0 : arow) * D;
  const float* W1 = M.W[0];
  const float* W2 = M.W[1];

  // ---- P1: z1 = G W1^T ----
  // Each chunk W1[0:H1][k0:k0+KC] is staged as [n][k] (zero past D; D is a
  // multiple of 4); the next chunk and its G fragments are requested into
  // registers before this chunk's products, so their loads overlap them.
  constexpr int NT = 64 * kRwWaves;
  constexpr int NS1 = H1 * KC / 4 / NT;
  static_assert(H1 * KC / 4 % NT == 0, "whole float4 per thread");
  float4 wpre[NS1], apre[KC / 16];
  auto fetch1 = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NS1; ++q) {
      const int x = tid + q * NT, n = x / (KC / 4), k = k0 + 4 * (x - n * (KC / 4));
      wpre[q] = k < D ? *reinterpret_cast<const float4*>(W1 + (int64_t)n * D + k) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int kb = 0; kb < KC / 16; ++kb) {
      const int k = k0 + 16 * kb + 4 * lk;
      apre[kb] = k < D ? *reinterpret_cast<const float4*>(Grow + k) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  floatx4 acc1[H1T];
#pragma unroll
  for (int u = 0; u < H1T; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  fetch1(0);
  for (int k0 = 0; k0 < D; k0 += KC) {
#pragma unroll
    for (int q = 0; q < NS1; ++q) {
      const int x = tid + q * NT, n = x / (KC / 4);
      *reinterpret_cast<float4*>(ws + n * LDW + 4 * (x - n * (KC / 4))) = wpre[q];
    }
    float4 a[KC / 16];
#pragma unroll
    for (int kb = 0; kb < KC / 16; ++kb) a[kb] = apre[kb];
    __syncthreads();
    if (k0 + KC < D) fetch1(k0 + KC);
#pragma unroll
    for (int kb = 0; kb < KC / 16; ++kb)
#pragma unroll
      for (int u = 0; u < H1T; ++u)
        acc1[u] = mma4_f32(acc1[u], a[kb], *reinterpret_cast<const float4*>(ws + (16 * u + lm) * LDW + 16 * kb + 4 * lk));
    __syncthreads();
  }
  float d1[H1T][4];  // act'(z1) in C layout
#pragma unroll
  for (int u = 0; u < H1T; ++u) {
    const float bias = M.b[0][16 * u + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc1[u][j] + bias;
      const float av = act_f(act1, z);
      d1[u][j] = act_d(act1, z, av);
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = av;
      if (args.st_a1) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) args.st_a1[(int64_t)r * H1 + 16 * u + lm] = av;
      }
    }
  }
  rw_wave_sync();

  // ---- P2: z2 = a1 W2^T ----
  floatx4 acc2[H2T];
#pragma unroll
  for (int u = 0; u < H2T; ++u) acc2[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < H1; k0 += KC) {
    for (int x = tid; x < H2 * KC / 4; x += 64 * kRwWaves) {
      const int n = x / (KC / 4), k4 = x - n * (KC / 4);
      const int k = k0 + 4 * k4;
      const float4 v = k < H1 ? *reinterpret_cast<const float4*>(W2 + (int64_t)n * H1 + k) : make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(ws + n * LDW + 4 * k4) = v;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < KC / 16; ++kb) {
      if (k0 + 16 * kb >= H1) break;
      const float4 a = *reinterpret_cast<const float4*>(abuf + lm * LDA + k0 + 16 * kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < H2T; ++u)
        acc2[u] = mma4_f32(acc2[u], a, *reinterpret_cast<const float4*>(ws + (16 * u + lm) * LDW + 16 * kb + 4 * lk));
    }
    __syncthreads();
  }
  // ---- output E = w3 . a2 + b3 and delta2 = w3 act'(z2) (over a1 in abuf) ----
  // (every wave's reads of a1 ended before the last barrier of P2)
  const float* w3 = M.W[2];
  float e[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < H2T; ++u) {
    const float bias = M.b[1][16 * u + lm];
    const float w = w3[16 * u + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc2[u][j] + bias;
      const float av = act_f(act2, z);
      e[j] = fmaf(av, w, e[j]);
      const float dl2 = w * act_d(act2, z, av);
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = dl2;
      if (args.st_a2) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) {
          args.st_a2[(int64_t)r * H2 + 16 * u + lm] = av;
          args.st_d2[(int64_t)r * H2 + 16 * u + lm] = dl2;
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
    for (int j = 0; j < 4; ++j) {
      const int r = rows[16 * wv + 4 * lk + j];
      if (r >= 0) args.E_atom[r] = e[j] + M.b[2][0];
    }
  if (args.lambda == nullptr && args.st_d1 == nullptr) return;  // the same for the whole block
  rw_wave_sync();

  // ---- P3: g1 = delta2 W2, delta1 = g1 act'(z1) ----
#pragma unroll
  for (int u = 0; u < H1T; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < H2; k0 += KC) {
    // stage W2[k0:k0+KC][0:H1] transposed: ws[n][k] = W2[k0 + k][n], four k
    // per thread (each load coalesced over n) as one 16-byte LDS store: a
    // thread per value would put lanes n and n + 16 on one bank
    for (int x = tid; x < KC / 4 * H1; x += 64 * kRwWaves) {
      const int kq = x / H1, n = x - kq * H1, k = k0 + 4 * kq;
      float4 v;
      v.x = k < H2 ? W2[(int64_t)k * H1 + n] : 0.f;
      v.y = k + 1 < H2 ? W2[(int64_t)(k + 1) * H1 + n] : 0.f;
      v.z = k + 2 < H2 ? W2[(int64_t)(k + 2) * H1 + n] : 0.f;
      v.w = k + 3 < H2 ? W2[(int64_t)(k + 3) * H1 + n] : 0.f;
      *reinterpret_cast<float4*>(ws + n * LDW + 4 * kq) = v;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < KC / 16; ++kb) {
      if (k0 + 16 * kb >= H2) break;
      const float4 a = *reinterpret_cast<const float4*>(abuf + lm * LDA + k0 + 16 * kb + 4 * lk);
#pragma unroll
      for (int u = 0; u < H1T; ++u)
        acc1[u] = mma4_f32(acc1[u], a, *reinterpret_cast<const float4*>(ws + (16 * u + lm) * LDW + 16 * kb + 4 * lk));
    }
    __syncthreads();
  }
  rw_wave_sync();  // every lane's delta2 reads are done before delta1 overwrites them
#pragma unroll
  for (int u = 0; u < H1T; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dd = acc1[u][j] * d1[u][j];
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = dd;
      if (args.st_d1) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) args.st_d1[(int64_t)r * H1 + 16 * u + lm] = dd;
      }
    }
  if (args.lambda == nullptr) return;
  rw_wave_sync();

  // ---- P4: lambda = delta1 W1, column chunks of KC ----
  float4 a4[H1T];  // this wave's delta1 rows as A fragments (k over H1)
#pragma unroll
  for (int kb = 0; kb < H1T; ++kb) a4[kb] = *reinterpret_cast<const float4*>(abuf + lm * LDA + 16 * kb + 4 * lk);
  int orow[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) orow[j] = rows[16 * wv + 4 * lk + j];
  // each chunk W1[0:H1][c0:c0+KC] staged transposed, ws[n][k] = W1[k][c0 + n],
  // four k per thread as one 16-byte LDS store (as in P3), the next chunk
  // requested before this one's products
  constexpr int NS4 = H1 * KC / (4 * NT);
  static_assert(H1 * KC % (4 * NT) == 0, "whole groups of four values per thread");
  float4 wp4[NS4];
  auto fetch4 = [&](int c0) {
#pragma unroll
    for (int q = 0; q < NS4; ++q) {
      const int x = tid + q * NT, kq = x / KC, n = x - kq * KC;
      const bool in = c0 + n < D;
      const float* w = W1 + (int64_t)(4 * kq) * D + c0 + n;
      wp4[q] = in ? make_float4(w[0], w[D], w[2 * D], w[3 * D]) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  fetch4(0);
  for (int c0 = 0; c0 < D; c0 += KC) {
#pragma unroll
    for (int q = 0; q < NS4; ++q) {
      const int x = tid + q * NT, kq = x / KC;
      *reinterpret_cast<float4*>(ws + (x - kq * KC) * LDT + 4 * kq) = wp4[q];
    }
    __syncthreads();
    if (c0 + KC < D) fetch4(c0 + KC);
#pragma unroll
    for (int ct = 0; ct < KC / 16; ++ct) {
      if (c0 + 16 * ct >= D) break;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < H1T; ++kb)
        acc = mma4_f32(acc, a4[kb], *reinterpret_cast<const float4*>(ws + (16 * ct + lm) * LDT + 16 * kb + 4 * lk));
      const int col = c0 + 16 * ct + lm;
      if (col < D)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (orow[j] >= 0) args.lambda[(int64_t)orow[j] * D + col] = acc[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BF16 products (MODE kBf16 or kBf16x3, v_mfma_f32_16x16x32_bf16): the same
// row blocks and stages, with every weight block staged from the BF16 hi/lo
// copies of W (rows [n][k]) and W^T (the per-call conversion of both layers),
// so no product transposes while staging.  A wave splits its own rows'
// operands (G, a1, delta2, delta1) once, 8 k per lane per 32-k step; the
// tile kernel instead had every wave of a tile split the whole G tile.
// ---------------------------------------------------------------------------

template <int H1T, int H2T>
struct RowsShapeBf {
  static constexpr int H1 = 16 * H1T, H2 = 16 * H2T;
  static constexpr int HM = H1 > H2 ? H1 : H2;
  static constexpr int KC = 32;                     // k chunk (P1-P3), column chunk (P4)
  static constexpr int LDB = KC + 8;                // staged BF16 [n][k] rows of P1-P3
  static constexpr int LDT = H1 + 8;                // staged BF16 [n][k] rows of P4
  static constexpr int LDA = HM + 4;                // the wave's FP32 rows
  static constexpr int WS1 = HM * LDB, WS4 = KC * LDT;
  static constexpr int WSB = WS1 > WS4 ? WS1 : WS4;  // BF16 values per staged array (hi, lo)
  static constexpr size_t lds = 2 * sizeof(__bf16) * (size_t)WSB + sizeof(float) * (size_t)kRwWaves * 16 * LDA;
};

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int H1T, int H2T, int MODE>
__global__ void __launch_bounds__(64 * kRwWaves) k_mlp_rows_bf(MlpArgs args) {
  using Sh = RowsShapeBf<H1T, H2T>;
  constexpr int H1 = Sh::H1, H2 = Sh::H2, KC = Sh::KC, LDB = Sh::LDB, LDT = Sh::LDT, LDA = Sh::LDA;
  constexpr bool X3 = MODE == kBf16x3;
  constexpr int NT = 64 * kRwWaves;
  extern __shared__ float4 rw_lds4[];
  __bf16* wsh = reinterpret_cast<__bf16*>(rw_lds4);
  __bf16* wsl = wsh + Sh::WSB;
  __shared__ int32_t rows[kRwAtoms];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  float* abuf = reinterpret_cast<float*>(wsl + Sh::WSB) + wv * 16 * LDA;
  const int lm = lane & 15, lk = lane >> 4;
  const int S = args.model.S;
  int64_t t = blockIdx.x;
  int s = 0;
  int64_t ns = 0;
  for (; s < S; ++s) {
    ns = args.sp_start[s + 1] - args.sp_start[s];
    const int64_t nt = (ns + kRwAtoms - 1) / kRwAtoms;
    if (t < nt) break;
    t -= nt;
  }
  if (s >= S) return;
  const int64_t r0 = args.sp_start[s] + t * kRwAtoms;
  const int nrows = (int)min<int64_t>(kRwAtoms, args.sp_start[s] + ns - r0);
  if (tid < kRwAtoms) rows[tid] = tid < nrows ? args.perm[r0 + tid] : -1;
  __syncthreads();
  const MlpDev& M = args.model.m[s];
  const int D = args.D;
  const int act1 = M.act[0], act2 = M.act[1];
  const int arow = rows[16 * wv + lm];
  const float* Grow = args.G + (int64_t)(arow < 0 ? 0 : arow) * D;
  const u32x4 z4 = {0u, 0u, 0u, 0u};
  // rows [n0, n0 + NR) (of nmax, K columns each), k in [k0, k0 + KCH), into
  // LDS rows 0 .. NR - 1 of stride ld, hi and (split mode) lo; zero outside
  auto stage = [&](const __bf16* hi, const __bf16* lo, int K, int nmax, int n0, int NR, int k0, int KCH, int ld) {
    for (int x = tid; x < NR * KCH / 8; x += NT) {
      const int r = x / (KCH / 8), kk = 8 * (x - r * (KCH / 8));
      const int n = n0 + r, k = k0 + kk;
      const bool in = n < nmax && k < K;
      const int64_t off = (int64_t)n * K + k;
      *reinterpret_cast<u32x4*>(wsh + r * ld + kk) = in ? *reinterpret_cast<const u32x4*>(hi + off) : z4;
      if constexpr (X3) *reinterpret_cast<u32x4*>(wsl + r * ld + kk) = in ? *reinterpret_cast<const u32x4*>(lo + off) : z4;
    }
  };
  // an A fragment (8 k from kb of this lane's row lm) of the wave's FP32 rows,
  // split; every width is a multiple of 32, so kb + 7 stays inside the row
  auto afrag = [&](int kb, bf16x8& ah, bf16x8& al) {
    const float4 u = *reinterpret_cast<const float4*>(abuf + lm * LDA + kb);
    const float4 v = *reinterpret_cast<const float4*>(abuf + lm * LDA + kb + 4);
    const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    if constexpr (X3) split8(x, ah, al);
    else
#pragma unroll
      for (int q = 0; q < 8; ++q) ah[q] = (__bf16)x[q];
  };
  auto bfrag = [&](int off, bf16x8& bh, bf16x8& bl) {
    bh = *reinterpret_cast<const bf16x8*>(wsh + off);
    if constexpr (X3) bl = *reinterpret_cast<const bf16x8*>(wsl + off);
  };

  // ---- P1: z1 = G W1^T; the next chunk (weights and G) requested during this one ----
  constexpr int NS1 = H1 * KC / 8 / NT;
  static_assert(H1 * KC / 8 % NT == 0, "whole 16-byte units per thread");
  u32x4 ph[NS1], pl[NS1];
  float4 gp[KC / 32][2];
  const __bf16 *W1h = M.Wb[0], *W1l = M.Wl[0];
  auto fetch1 = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NS1; ++q) {
      const int x = tid + q * NT, n = x / (KC / 8), k = k0 + 8 * (x - n * (KC / 8));
      const int64_t off = (int64_t)n * D + k;
      ph[q] = k < D ? *reinterpret_cast<const u32x4*>(W1h + off) : z4;
      if constexpr (X3) pl[q] = k < D ? *reinterpret_cast<const u32x4*>(W1l + off) : z4;
    }
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
      const int k = k0 + 32 * kk + 8 * lk;
      gp[kk][0] = k < D ? *reinterpret_cast<const float4*>(Grow + k) : make_float4(0.f, 0.f, 0.f, 0.f);
      gp[kk][1] = k < D ? *reinterpret_cast<const float4*>(Grow + k + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  floatx4 acc1[H1T];
#pragma unroll
  for (int u = 0; u < H1T; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  fetch1(0);
  for (int k0 = 0; k0 < D; k0 += KC) {
#pragma unroll
    for (int q = 0; q < NS1; ++q) {
      const int x = tid + q * NT, n = x / (KC / 8), kk = 8 * (x - n * (KC / 8));
      *reinterpret_cast<u32x4*>(wsh + n * LDB + kk) = ph[q];
      if constexpr (X3) *reinterpret_cast<u32x4*>(wsl + n * LDB + kk) = pl[q];
    }
    bf16x8 ah[KC / 32], al[KC / 32];
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
      const float x[8] = {gp[kk][0].x, gp[kk][0].y, gp[kk][0].z, gp[kk][0].w,
                          gp[kk][1].x, gp[kk][1].y, gp[kk][1].z, gp[kk][1].w};
      if constexpr (X3) split8(x, ah[kk], al[kk]);
      else
#pragma unroll
        for (int q = 0; q < 8; ++q) ah[kk][q] = (__bf16)x[q];
    }
    __syncthreads();
    if (k0 + KC < D) fetch1(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk)
#pragma unroll
      for (int u = 0; u < H1T; ++u) {
        bf16x8 bh, bl;
        bfrag((16 * u + lm) * LDB + 32 * kk + 8 * lk, bh, bl);
        acc1[u] = mma_bf16<MODE>(acc1[u], ah[kk], al[kk], bh, bl);
      }
    __syncthreads();
  }
  float d1[H1T][4];
#pragma unroll
  for (int u = 0; u < H1T; ++u) {
    const float bias = M.b[0][16 * u + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc1[u][j] + bias;
      const float av = act_f(act1, z);
      d1[u][j] = act_d(act1, z, av);
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = av;
      if (args.st_a1) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) args.st_a1[(int64_t)r * H1 + 16 * u + lm] = av;
      }
    }
  }
  rw_wave_sync();

  // ---- P2: z2 = a1 W2^T ----
  floatx4 acc2[H2T];
#pragma unroll
  for (int u = 0; u < H2T; ++u) acc2[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < H1; k0 += KC) {
    stage(M.Wb[1], M.Wl[1], H1, H2, 0, H2, k0, KC, LDB);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
      if (k0 + 32 * kk >= H1) break;
      bf16x8 ah, al;
      afrag(k0 + 32 * kk + 8 * lk, ah, al);
#pragma unroll
      for (int u = 0; u < H2T; ++u) {
        bf16x8 bh, bl;
        bfrag((16 * u + lm) * LDB + 32 * kk + 8 * lk, bh, bl);
        acc2[u] = mma_bf16<MODE>(acc2[u], ah, al, bh, bl);
      }
    }
    __syncthreads();
  }
  // ---- output E and delta2 (over a1 in abuf: every read of it ended before P2's last barrier) ----
  const float* w3 = M.W[2];
  float e[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < H2T; ++u) {
    const float bias = M.b[1][16 * u + lm];
    const float w = w3[16 * u + lm];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float z = acc2[u][j] + bias;
      const float av = act_f(act2, z);
      e[j] = fmaf(av, w, e[j]);
      const float dl2 = w * act_d(act2, z, av);
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = dl2;
      if (args.st_a2) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) {
          args.st_a2[(int64_t)r * H2 + 16 * u + lm] = av;
          args.st_d2[(int64_t)r * H2 + 16 * u + lm] = dl2;
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
    for (int j = 0; j < 4; ++j) {
      const int r = rows[16 * wv + 4 * lk + j];
      if (r >= 0) args.E_atom[r] = e[j] + M.b[2][0];
    }
  if (args.lambda == nullptr && args.st_d1 == nullptr) return;
  rw_wave_sync();

  // ---- P3: g1 = delta2 W2 = delta2 (W2^T)^T, staged from W2^T [H1][H2] ----
#pragma unroll
  for (int u = 0; u < H1T; ++u) acc1[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < H2; k0 += KC) {
    stage(M.WbT[1], M.WlT[1], H2, H1, 0, H1, k0, KC, LDB);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
      if (k0 + 32 * kk >= H2) break;
      bf16x8 ah, al;
      afrag(k0 + 32 * kk + 8 * lk, ah, al);
#pragma unroll
      for (int u = 0; u < H1T; ++u) {
        bf16x8 bh, bl;
        bfrag((16 * u + lm) * LDB + 32 * kk + 8 * lk, bh, bl);
        acc1[u] = mma_bf16<MODE>(acc1[u], ah, al, bh, bl);
      }
    }
    __syncthreads();
  }
  rw_wave_sync();
#pragma unroll
  for (int u = 0; u < H1T; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dd = acc1[u][j] * d1[u][j];
      abuf[(4 * lk + j) * LDA + 16 * u + lm] = dd;
      if (args.st_d1) {
        const int r = rows[16 * wv + 4 * lk + j];
        if (r >= 0) args.st_d1[(int64_t)r * H1 + 16 * u + lm] = dd;
      }
    }
  if (args.lambda == nullptr) return;
  rw_wave_sync();

  // ---- P4: lambda = delta1 W1 = delta1 (W1^T)^T, column chunks staged from W1^T [D][H1] ----
  bf16x8 dh[H1 / 32], dl[H1 / 32];
#pragma unroll
  for (int kb = 0; kb < H1 / 32; ++kb) afrag(32 * kb + 8 * lk, dh[kb], dl[kb]);
  int orow[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) orow[j] = rows[16 * wv + 4 * lk + j];
  constexpr int NS4 = KC * H1 / 8 / NT;
  static_assert(KC * H1 / 8 % NT == 0, "whole 16-byte units per thread");
  u32x4 qh[NS4], ql[NS4];
  const __bf16 *W1Th = M.WbT[0], *W1Tl = M.WlT[0];
  auto fetch4 = [&](int c0) {
#pragma unroll
    for (int q = 0; q < NS4; ++q) {
      const int x = tid + q * NT, r = x / (H1 / 8), k = 8 * (x - r * (H1 / 8));
      const bool in = c0 + r < D;
      const int64_t off = (int64_t)(c0 + r) * H1 + k;
      qh[q] = in ? *reinterpret_cast<const u32x4*>(W1Th + off) : z4;
      if constexpr (X3) ql[q] = in ? *reinterpret_cast<const u32x4*>(W1Tl + off) : z4;
    }
  };
  fetch4(0);
  for (int c0 = 0; c0 < D; c0 += KC) {
#pragma unroll
    for (int q = 0; q < NS4; ++q) {
      const int x = tid + q * NT, r = x / (H1 / 8), k = 8 * (x - r * (H1 / 8));
      *reinterpret_cast<u32x4*>(wsh + r * LDT + k) = qh[q];
      if constexpr (X3) *reinterpret_cast<u32x4*>(wsl + r * LDT + k) = ql[q];
    }
    __syncthreads();
    if (c0 + KC < D) fetch4(c0 + KC);
#pragma unroll
    for (int ct = 0; ct < KC / 16; ++ct) {
      if (c0 + 16 * ct >= D) break;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < H1 / 32; ++kb) {
        bf16x8 bh, bl;
        bfrag((16 * ct + lm) * LDT + 32 * kb + 8 * lk, bh, bl);
        acc = mma_bf16<MODE>(acc, dh[kb], dl[kb], bh, bl);
      }
      const int col = c0 + 16 * ct + lm;
      if (col < D)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (orow[j] >= 0) args.lambda[(int64_t)orow[j] * D + col] = acc[j];
    }
    __syncthreads();
  }
}

bool mlp_rows_bf_supported(int h1, int h2, int D) {
  return ((h1 == 64 && h2 == 32) || (h1 == 128 && h2 == 128)) && D % 8 == 0;
}

void launch_mlp_rows_bf(const MlpArgs& a, int h1, int h2, int mode, int64_t N, hipStream_t s) {
  if (N == 0) return;
  const unsigned grid = (unsigned)((N + kRwAtoms - 1) / kRwAtoms + a.model.S);
  const dim3 g(grid), b(64 * kRwWaves);
  if (h1 == 64 && h2 == 32) {
    constexpr size_t lds = RowsShapeBf<4, 2>::lds;
    if (mode == kBf16x3) hipLaunchKernelGGL((k_mlp_rows_bf<4, 2, kBf16x3>), g, b, lds, s, a);
    else hipLaunchKernelGGL((k_mlp_rows_bf<4, 2, kBf16>), g, b, lds, s, a);
  } else if (h1 == 128 && h2 == 128) {
    constexpr size_t lds = RowsShapeBf<8, 8>::lds;
    if (mode == kBf16x3) hipLaunchKernelGGL((k_mlp_rows_bf<8, 8, kBf16x3>), g, b, lds, s, a);
    else hipLaunchKernelGGL((k_mlp_rows_bf<8, 8, kBf16>), g, b, lds, s, a);
  }
}

bool mlp_rows_supported(int h1, int h2, int D) {
  return ((h1 == 64 && h2 == 32) || (h1 == 128 && h2 == 128)) && D % 4 == 0;
}

void launch_mlp_rows(const MlpArgs& a, int h1, int h2, int64_t N, hipStream_t s) {
  if (N == 0) return;
  const unsigned grid = (unsigned)((N + kRwAtoms - 1) / kRwAtoms + a.model.S);
  if (h1 == 64 && h2 == 32) {
    constexpr size_t lds = RowsShape<4, 2>::lds;
    hipLaunchKernelGGL((k_mlp_rows<4, 2>), dim3(grid), dim3(64 * kRwWaves), lds, s, a);
  } else if (h1 == 128 && h2 == 128) {
    constexpr size_t lds = RowsShape<8, 8>::lds;
    hipLaunchKernelGGL((k_mlp_rows<8, 8>), dim3(grid), dim3(64 * kRwWaves), lds, s, a);
  }
}

}  // namespace nnp
