// Neighbor lists on the device: cell binning for large structures,
// all-pairs over lattice images for small ones, canonical row order and
// reverse-entry index.  Locality and cutoff: Sec. I and Sec. III.A.
//
// Every kernel of a (re)build reads a device flag first and exits when the
// skin test decided that the previous list is still valid, so the whole
// build can sit in a captured graph without host decisions.
#include <math.h>

#include <algorithm>

#include "common.h"

namespace nnp {

// ---------------------------------------------------------------------------
// exclusive scan of int64 (n + 1 outputs: out[n] = total)
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

size_t scan_scratch_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_reduce(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ partial,
                              const int32_t* pred) {
  if (pred && !*pred) return;
  __shared__ int64_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) s += (base + k < n) ? in[base + k] : 0;
  int64_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_scan_partials(int64_t* partial, int64_t nb, const int32_t* pred) {
  if (pred && !*pred) return;
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    int64_t idx = base + threadIdx.x;
    int64_t v = idx < nb ? partial[idx] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(v, sh, &tot);
    if (idx < nb) partial[idx] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) partial[nb] = carry;
}

__global__ void k_scan_apply(const int64_t* __restrict__ in, int64_t n, const int64_t* __restrict__ partial,
                             int64_t nb, int64_t* __restrict__ out, const int32_t* pred) {
  if (pred && !*pred) return;
  __shared__ int64_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(s, sh, &tot) + partial[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partial[nb];
}

// Whole scan in one block of 1024 threads (n <= kScanSmall).  Up to
// kScanRun elements per thread, thread t sums its own contiguous run.
// Beyond that, wave w owns the contiguous chunk [w c, (w + 1) c) of the
// input (c a multiple of 512) and takes it 512 elements at a time, lane l
// the kScanRun consecutive elements from 8 l, so that every load of the
// wave covers one contiguous stretch.  Either way: a pass for the run (or
// chunk) sums, wave shuffles and one step across the 16 wave totals, then
// a pass that writes the outputs on top of the running carry.  If n_dev is
// given, only its first min(*n_dev, n) entries are scanned.
constexpr int kScanSmallThreads = 1024;
constexpr int64_t kScanSmall = 64 * 1024;
constexpr int kScanRun = 8;

struct CapacityJob {  // decision taken after the scan of the row counts
  int64_t capacity;
  int64_t* meta;
  int32_t* flag;
};
__device__ void capacity_decision(const CapacityJob& cj, int64_t nnz);

template <bool CAP>
__global__ void __launch_bounds__(kScanSmallThreads) k_scan_small(const int64_t* __restrict__ in, int64_t n,
                                                                  const int64_t* __restrict__ n_dev,
                                                                  int64_t* __restrict__ out, const int32_t* pred,
                                                                  CapacityJob cj) {
  if (pred && !*pred) {
    if (CAP && threadIdx.x == 0) {
      cj.flag[1] = 0;
      cj.meta[kMetaRebuilt] = 0;
    }
    return;
  }
  constexpr int kW = kScanSmallThreads / 64;
  constexpr int kGroup = 64 * kScanRun;
  __shared__ int64_t wsum[kW];
  if (n_dev) n = min(n, max(*n_dev, (int64_t)0));
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (n <= (int64_t)kScanSmallThreads * kScanRun) {
    const int64_t per = (n + kScanSmallThreads - 1) / kScanSmallThreads;
    const int64_t b = min((int64_t)t * per, n), e = min(b + per, n);
    int64_t sum = 0;
    for (int64_t k = b; k < e; ++k) sum += in[k];
    int64_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
      int64_t x = lane < kW ? wsum[lane] : 0;
      for (int off = 1; off < kW; off <<= 1) {
        const int64_t v = __shfl_up(x, off);
        if (lane >= off) x += v;
      }
      if (lane < kW) wsum[lane] = x;  // inclusive wave totals
    }
    __syncthreads();
    int64_t run = incl - sum + (w > 0 ? wsum[w - 1] : 0);
    for (int64_t k = b; k < e; ++k) {
      const int64_t v = in[k];
      out[k] = run;
      run += v;
    }
    if (t == kScanSmallThreads - 1) {
      out[n] = wsum[kW - 1];
      if (CAP) capacity_decision(cj, wsum[kW - 1]);
    }
    return;
  }
  const int64_t chunk = ((n + kW - 1) / kW + kGroup - 1) / kGroup * kGroup;
  const int64_t b = min((int64_t)w * chunk, n), e = min(b + chunk, n);
  int64_t sum = 0;
  for (int64_t k0 = b + kScanRun * lane; k0 < e; k0 += kGroup) {
#pragma unroll
    for (int r = 0; r < kScanRun; ++r) sum += k0 + r < e ? in[k0 + r] : 0;
  }
  for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane == 0) wsum[w] = sum;
  __syncthreads();
  int64_t carry = 0;
  for (int u = 0; u < w; ++u) carry += wsum[u];
  for (int64_t g0 = b; g0 < e; g0 += kGroup) {
    const int64_t k0 = g0 + kScanRun * lane;
    int64_t v[kScanRun];
    int64_t ls = 0;
#pragma unroll
    for (int r = 0; r < kScanRun; ++r) {
      v[r] = k0 + r < e ? in[k0 + r] : 0;
      ls += v[r];
    }
    int64_t incl = ls;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t x = __shfl_up(incl, off);
      if (lane >= off) incl += x;
    }
    int64_t run = carry + incl - ls;
#pragma unroll
    for (int r = 0; r < kScanRun; ++r) {
      if (k0 + r < e) out[k0 + r] = run;
      run += v[r];
    }
    carry += __shfl(incl, 63);
  }
  if (t == kScanSmallThreads - 1) {
    int64_t total = 0;
    for (int u = 0; u < kW; ++u) total += wsum[u];
    out[n] = total;
    if (CAP) capacity_decision(cj, total);
  }
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s,
                        const int32_t* pred, const int64_t* n_dev) {
  if (n <= kScanSmall) {
    hipLaunchKernelGGL(k_scan_small<false>, dim3(1), dim3(kScanSmallThreads), 0, s, in, n, n_dev, out, pred,
                       CapacityJob{});
    return;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, scratch, pred);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBlock), 0, s, scratch, nb, pred);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, scratch, nb, out, pred);
}

// ---------------------------------------------------------------------------
// skin test and build predicate
// ---------------------------------------------------------------------------

// flag[0] = 1 if the list must be (re)built (no valid list yet, or no
// skin); the skin test below may raise it.  atom_ptr must run from 0 to N
// without decreasing; otherwise nothing is built and the list is marked
// invalid, so no later kernel reads it (the skin test only runs on a valid
// list).  Run by every thread of one block.
__device__ void prep_flags(const int64_t* __restrict__ atom_ptr, int32_t B, int64_t N, int64_t* meta, int32_t* flag,
                           int64_t* cursor, int use_skin) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = (atom_ptr[0] != 0 || atom_ptr[B] != N);
  __syncthreads();
  for (int c = threadIdx.x; c < B; c += blockDim.x)
    if (atom_ptr[c + 1] < atom_ptr[c]) bad = 1;
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (bad) {
    atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrPtr);
    meta[kMetaValid] = 0;
    flag[0] = 0;
    flag[1] = 0;
  } else {
    flag[0] = (use_skin && meta[kMetaValid] == 1) ? 0 : 1;
  }
  flag[2] = 0;  // the generic passes' predicate when the cluster passes are tried (set by k_cl_count)
  flag[3] = 0;  // structures the cluster passes could not take
  *cursor = 0;  // overflow area of the counting pass's row keys
}

__global__ void k_nb_prep(const int64_t* __restrict__ atom_ptr, int32_t B, int64_t N, int64_t* meta, int32_t* flag,
                          int64_t* cursor, int use_skin) {
  prep_flags(atom_ptr, B, N, meta, flag, cursor, use_skin);
}

__global__ void k_skin_check(const double* __restrict__ pos, const double* __restrict__ ref, int64_t n,
                             double half_skin2, const int64_t* meta, int32_t* flag, int use_skin) {
  if (!use_skin || meta[kMetaValid] != 1) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool move = false;
  if (i < n) {
#pragma clang fp contract(off)
    double dx = pos[3 * i] - ref[3 * i], dy = pos[3 * i + 1] - ref[3 * i + 1], dz = pos[3 * i + 2] - ref[3 * i + 2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    move = !(d2 <= half_skin2);  // also catches NaN
  }
  if (__any(move) && lane_id() == 0) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// per-structure geometry
// ---------------------------------------------------------------------------

__device__ void inverse3(const double h[9], double inv[9]) {
  double c00 = h[4] * h[8] - h[5] * h[7];
  double c01 = h[5] * h[6] - h[3] * h[8];
  double c02 = h[3] * h[7] - h[4] * h[6];
  double det = h[0] * c00 + h[1] * c01 + h[2] * c02;
  double id = 1.0 / det;
  inv[0] = c00 * id;
  inv[1] = (h[2] * h[7] - h[1] * h[8]) * id;
  inv[2] = (h[1] * h[5] - h[2] * h[4]) * id;
  inv[3] = c01 * id;
  inv[4] = (h[0] * h[8] - h[2] * h[6]) * id;
  inv[5] = (h[2] * h[3] - h[0] * h[5]) * id;
  inv[6] = c02 * id;
  inv[7] = (h[1] * h[6] - h[0] * h[7]) * id;
  inv[8] = (h[0] * h[4] - h[1] * h[3]) * id;
}

__device__ void perp_widths(const double* h, double w[3]) {
  const double *a = h, *b = h + 3, *c = h + 6;
  double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
  double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  double vol = fabs(a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]);
  w[0] = vol / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  w[1] = vol / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
  w[2] = vol / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
}

__device__ __forceinline__ void frac(const double* inv, const double* x, double s[3]) {
  for (int d = 0; d < 3; ++d) s[d] = x[0] * inv[d] + x[1] * inv[3 + d] + x[2] * inv[6 + d];
}

// Geometry of one structure of nc atoms with cell h (inverse inv): the
// all-pairs path with image bounds K_d = floor(radius/w_d + spread_d) + 1
// on periodic directions (l, u: range of the fractional coordinates) for
// small structures, else bins at least radius wide, merged while there are
// more than 8 nc + 64 of them.  Errors go to meta.
__device__ __forceinline__ StructGeom make_geom(const double h[9], const double inv[9], const uint8_t* pbc3, int64_t nc,
                                                const double l[3], const double u[3], double radius, int64_t* meta) {
  double w[3];
  perp_widths(h, w);
  StructGeom g;
  for (int k = 0; k < 9; ++k) {
    g.h[k] = h[k];
    g.inv[k] = inv[k];
  }
  const bool small = nc <= kSmallMax;
  g.small = small ? 1 : 0;
  int64_t nbins = 0;
  if (small) {
    nbins = nc > 0 ? 1 : 0;  // the whole structure is one group of the row passes
    for (int d = 0; d < 3; ++d) {
      double K = pbc3[d] && nc > 0 ? floor(radius / w[d] + (u[d] - l[d])) + 1.0 : 0.0;
      if (!(K <= 127.0)) {
        atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrShift);
        K = 0.0;
      }
      g.nb[d] = (int)K;
    }
  } else {
    int minb[3];
    for (int d = 0; d < 3; ++d) {
      double k = floor(w[d] / (radius * (1.0 + 1e-6)));
      if (!(k >= 1.0)) k = 1.0;
      if (k > 1024.0) k = 1024.0;
      g.nb[d] = (int)k;
      minb[d] = pbc3[d] ? 3 : 1;
      if (g.nb[d] < minb[d]) {
        atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrCell);
        g.nb[d] = minb[d];
      }
    }
    // keep the bin count near the atom count (dilute boxes): halve the
    // direction with the most bins above its minimum (the first on ties)
    // while there are too many
    const int64_t cap = 8 * nc + 64;
    int n0 = g.nb[0], n1 = g.nb[1], n2 = g.nb[2];
    for (int it = 0; it < 64 && (int64_t)n0 * n1 * n2 > cap; ++it) {
      const int e0 = n0 - minb[0], e1 = n1 - minb[1], e2 = n2 - minb[2];
      const int d = e1 > e0 ? (e2 > e1 ? 2 : 1) : (e2 > e0 ? 2 : 0);
      const int nd = d == 0 ? n0 : (d == 1 ? n1 : n2), md = d == 0 ? minb[0] : (d == 1 ? minb[1] : minb[2]);
      if (nd <= md) break;
      const int half = max(md, (nd + 1) / 2);
      n0 = d == 0 ? half : n0;
      n1 = d == 1 ? half : n1;
      n2 = d == 2 ? half : n2;
    }
    g.nb[0] = n0;
    g.nb[1] = n1;
    g.nb[2] = n2;
    nbins = (int64_t)n0 * n1 * n2;
  }
  g.n_bins = nbins;
  g.bin_base = 0;
  return g;
}

// One 64-thread block per structure.  Small structures (<= kSmallMax atoms)
// take the all-pairs path with an image bound K_d = floor(radius/w_d +
// spread_d) + 1 on periodic directions (spread of the fractional
// coordinates) and form a single bin; larger ones are binned with bins >=
// radius wide.
// Every block of the grid (B or more) also clears its share of the bin
// counts [0, n_zero).  With one structure, bin_base is written here too.
__global__ void k_nb_geom(const double* __restrict__ pos, const int64_t* __restrict__ atom_ptr,
                          const double* __restrict__ cell, const uint8_t* __restrict__ pbc, int32_t B,
                          double radius, StructGeom* __restrict__ geom, int64_t* __restrict__ n_bins,
                          int64_t* __restrict__ bin_count, int64_t n_zero, int64_t* __restrict__ bin_base_one,
                          int64_t N, int64_t* meta, int32_t* flag, int64_t* cursor, int prep) {
  // prep: no skin test, so this launch also checks atom_ptr and sets the
  // build flags (block 0); the other blocks read atom_ptr clamped to [0, N],
  // and nothing after this launch runs if it was invalid
  if (prep) {
    if (blockIdx.x == 0) prep_flags(atom_ptr, B, N, meta, flag, cursor, 0);
  } else if (!*flag) {
    return;
  }
  for (int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x; k < n_zero; k += (int64_t)gridDim.x * 64)
    bin_count[k] = 0;
  const int c = blockIdx.x;
  if (c >= B) return;
  __shared__ double h[9], inv[9];
  if (threadIdx.x < 9) h[threadIdx.x] = cell[9 * (int64_t)c + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) inverse3(h, inv);
  __syncthreads();
  const int64_t a0 = min(max(atom_ptr[c], (int64_t)0), N), a1 = min(max(atom_ptr[c + 1], a0), N);
  const int64_t nc = a1 - a0;
  const bool small = nc <= kSmallMax;
  double l[3] = {1e300, 1e300, 1e300}, u[3] = {-1e300, -1e300, -1e300};
  if (small) {
    for (int64_t a = a0 + threadIdx.x; a < a1; a += 64) {
      double s[3];
      frac(inv, pos + 3 * a, s);
      for (int d = 0; d < 3; ++d) {
        l[d] = fmin(l[d], s[d]);
        u[d] = fmax(u[d], s[d]);
      }
    }
  }
  if (small) {  // range of the fractional coordinates (wave reduction)
    for (int d = 0; d < 3; ++d)
      for (int off = 32; off > 0; off >>= 1) {
        l[d] = fmin(l[d], __shfl_xor(l[d], off));
        u[d] = fmax(u[d], __shfl_xor(u[d], off));
      }
  }
  if (threadIdx.x != 0) return;
  const StructGeom g = make_geom(h, inv, pbc + 3 * c, nc, l, u, radius, meta);
  const int64_t nbins = g.n_bins;
  geom[c] = g;
  n_bins[c] = nbins;
  if (bin_base_one) {
    bin_base_one[0] = 0;
    bin_base_one[1] = nbins;
  }
}


// The largest c < n with a[c] <= x, for a non-decreasing a with a[0] <= x,
// found by the whole wave: each round its 64 lanes probe 64 evenly spaced
// positions of the remaining range and one ballot keeps the stretch after the
// last probe at or below x (two dependent rounds for 4096 entries instead
// of twelve).  Every lane of the wave must call it with the same x.
__device__ __forceinline__ int wave_search_le(const int64_t* a, int n, int64_t x) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int step = (hi - lo + 63) / 64;
    const int p = lo + lane * step;
    const uint64_t le = __ballot(p < hi && a[p] <= x);
    lo += (__popcll(le) - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

__device__ __forceinline__ int struct_of(const int64_t* atom_ptr, int32_t B, int64_t i) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (atom_ptr[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Bin coordinates of an atom of a binned structure; m is the whole-cell
// offset removed on periodic directions.
__device__ __forceinline__ void bin_coords(const StructGeom& g, const uint8_t* pbc3, const double* x, int b3[3],
                                           int m[3]) {
  double s[3];
  frac(g.inv, x, s);
  for (int d = 0; d < 3; ++d) {
    double t = s[d];
    m[d] = 0;
    if (pbc3[d]) {
      double f = floor(t);
      m[d] = (int)fmin(fmax(f, -1073741824.0), 1073741824.0);
      t = t - f;
    }
    double kf = fmin(fmax(floor(t * g.nb[d]), 0.0), (double)(g.nb[d] - 1));
    b3[d] = (int)kf;
  }
}

// Bin of every atom (the single bin of its structure for small ones) and
// its rank inside the bin.  Atoms with non-finite coordinates are left out
// (row count 0) and flagged.
__global__ void k_nb_bin(const double* __restrict__ pos, const int64_t* __restrict__ atom_ptr,
                         const uint8_t* __restrict__ pbc, int32_t B, int64_t N, const StructGeom* __restrict__ geom,
                         const int64_t* __restrict__ bin_base, int64_t* __restrict__ bin_count,
                         int32_t* __restrict__ atom_bin, int32_t* __restrict__ bin_rank,
                         int64_t* __restrict__ row_count, int64_t* meta, const int32_t* flag) {
  if (!*flag) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* x = pos + 3 * i;
  if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
    atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrNonFinite);
    atom_bin[4 * i] = -1;
    row_count[i] = 0;
    return;
  }
  int c = struct_of(atom_ptr, B, i);
  const StructGeom& g = geom[c];
  int b3[3] = {0, 0, 0}, m[3] = {0, 0, 0};
  if (!g.small) bin_coords(g, pbc + 3 * c, x, b3, m);
  int64_t bin = bin_base[c] + ((int64_t)b3[0] * g.nb[1] + b3[1]) * g.nb[2] + b3[2];
  if (g.small) bin = bin_base[c];
  atom_bin[4 * i + 0] = (int32_t)bin;
  atom_bin[4 * i + 1] = m[0];
  atom_bin[4 * i + 2] = m[1];
  atom_bin[4 * i + 3] = m[2];
  bin_rank[i] = (int32_t)atomicAdd((unsigned long long*)&bin_count[bin], 1ull);
}

// Atoms into bin order, with a copy of each atom's position and whole-cell
// offsets in the same order, so that the row passes read the candidates of
// a bin as contiguous memory.  The order inside a bin is the order in which
// the binning pass's atomics ran (rows are sorted afterwards).
__global__ void k_nb_scatter(int64_t N, const double* __restrict__ pos, const int32_t* __restrict__ atom_bin,
                             const int32_t* __restrict__ bin_rank, const int64_t* __restrict__ bin_start,
                             int4* __restrict__ bin_m, double4* __restrict__ bin_x, int32_t* __restrict__ order,
                             const int32_t* flag) {
  if (!*flag) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int32_t bin = atom_bin[4 * i];
  if (bin < 0) return;
  const int64_t k = bin_start[bin] + bin_rank[i];
  bin_m[k] = make_int4((int)i, atom_bin[4 * i + 1], atom_bin[4 * i + 2], atom_bin[4 * i + 3]);
  bin_x[k] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.0);
  if (order) order[k] = (int32_t)i;
}

// The geometry, binning, bin-start scan and scatter passes of a single
// structure of at most kOneAtoms atoms in one block of 1024 threads (one
// launch in place of four).  Bin counts and starts never exceed the atom
// count, so they are kept in LDS as the two 16-bit halves of 32-bit words;
// the geometry allows at most 8 N + 64 bins, which kOneWords covers.  The
// positions are loaded before the geometry is known; each atom's index and
// position go to LDS at its place in bin order (the positions over the bin
// counts, which are no longer needed), and the bin-ordered outputs are then
// written k = t, t + 1024, ... so that the stores of a wave are contiguous.  The
// outputs are those of the four passes: geom[0], n_bins[0], bin_base[0..1],
// bin_start[0..n_bins], bin_m / bin_x / order in bin order, and a zero row
// count for atoms with non-finite coordinates.
constexpr int kOneThreads = 1024;
constexpr int kOnePer = 4;
constexpr int64_t kOneAtoms = (int64_t)kOneThreads * kOnePer;
constexpr int kOneWords = (int)((8 * kOneAtoms + 64 + 1) / 2);

__global__ void __launch_bounds__(kOneThreads) k_nb_one(const double* __restrict__ pos,
                                                        const int64_t* __restrict__ atom_ptr,
                                                        const double* __restrict__ cell,
                                                        const uint8_t* __restrict__ pbc, double radius,
                                                        StructGeom* __restrict__ geom, int64_t* __restrict__ n_bins,
                                                        int64_t* __restrict__ bin_base, int64_t* __restrict__ bin_start,
                                                        int4* __restrict__ bin_m, double4* __restrict__ bin_x,
                                                        int32_t* __restrict__ order, int64_t* __restrict__ row_count,
                                                        int64_t N, int64_t* meta, int32_t* flag, int64_t* cursor,
                                                        int prep) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double hc = t < 9 ? cell[t] : 0.0;
  // prep: no skin test ran, so this launch checks atom_ptr (for one
  // structure: atom_ptr = {0, N}) and sets the build flags itself
  if (prep) prep_flags(atom_ptr, 1, N, meta, flag, cursor, 0);
  const bool go = prep ? (atom_ptr[0] == 0 && atom_ptr[1] == N) : (*flag != 0);
  if (!go) return;
  // this thread's atoms i = t + 1024 r, in flight while the geometry is formed
  double x[kOnePer][3];
#pragma unroll
  for (int r = 0; r < kOnePer; ++r) {
    const int64_t i = t + (int64_t)kOneThreads * r;
    for (int d = 0; d < 3; ++d) x[r][d] = i < N ? pos[3 * i + d] : 0.0;
  }
  constexpr int kW = kOneThreads / 64;
  __shared__ union {
    uint32_t cnt[kOneWords];    // bin counts, then bin starts
    double px[3][kOneAtoms];    // then the positions in bin order
  } lds;
  uint32_t* cnt = lds.cnt;
  __shared__ int32_t slot_atom[kOneAtoms];
  __shared__ double h[9], inv[9];
  __shared__ double ext[2][3][kW];
  __shared__ int64_t wsum[kW];
  __shared__ StructGeom gs;
  if (t < 9) h[t] = hc;
  __syncthreads();
  if (t == 0) inverse3(h, inv);
  __syncthreads();
  const bool small = N <= kSmallMax;
  double l[3] = {1e300, 1e300, 1e300}, u[3] = {-1e300, -1e300, -1e300};
  if (small) {  // range of the fractional coordinates (block reduction; N <= 1024: one atom per thread)
    if (t < N) {
      double f[3];
      frac(inv, x[0], f);
      for (int d = 0; d < 3; ++d) {
        l[d] = f[d];
        u[d] = f[d];
      }
    }
    for (int d = 0; d < 3; ++d) {
      for (int off = 32; off > 0; off >>= 1) {
        l[d] = fmin(l[d], __shfl_xor(l[d], off));
        u[d] = fmax(u[d], __shfl_xor(u[d], off));
      }
      if (lane == 0) {
        ext[0][d][w] = l[d];
        ext[1][d][w] = u[d];
      }
    }
    __syncthreads();
    if (t == 0)
      for (int d = 0; d < 3; ++d)
        for (int v = 1; v < kW; ++v) {
          l[d] = fmin(l[d], ext[0][d][v]);
          u[d] = fmax(u[d], ext[1][d][v]);
        }
  }
  if (t == 0) {
    gs = make_geom(h, inv, pbc, N, l, u, radius, meta);
    geom[0] = gs;
    n_bins[0] = gs.n_bins;
    bin_base[0] = 0;
    bin_base[1] = gs.n_bins;
  }
  __syncthreads();
  const StructGeom& g = gs;
  const int64_t nbins = g.n_bins;
  const int nw = (int)((nbins + 1) / 2);
  for (int k = t; k < nw; k += kOneThreads) cnt[k] = 0;
  __syncthreads();
  // bin and rank of each of this thread's atoms (i = t + 1024 r)
  int bin[kOnePer], rank[kOnePer];
#pragma unroll
  for (int r = 0; r < kOnePer; ++r) {
    const int64_t i = t + (int64_t)kOneThreads * r;
    bin[r] = -1;
    if (i >= N) continue;
    if (!(isfinite(x[r][0]) && isfinite(x[r][1]) && isfinite(x[r][2]))) {
      atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrNonFinite);
      row_count[i] = 0;
      continue;
    }
    int b3[3] = {0, 0, 0}, m[3];
    if (!g.small) bin_coords(g, pbc, x[r], b3, m);
    bin[r] = g.small ? 0 : (b3[0] * g.nb[1] + b3[1]) * g.nb[2] + b3[2];
    const int sh = 16 * (bin[r] & 1);
    rank[r] = (int)((atomicAdd(&cnt[bin[r] >> 1], 1u << sh) >> sh) & 0xffffu);
  }
  __syncthreads();
  // exclusive scan of the counts: thread t takes a contiguous run of words
  const int per = (nw + kOneThreads - 1) / kOneThreads;
  const int w0 = min(t * per, nw), w1 = min(w0 + per, nw);
  int64_t sum = 0;
  for (int k = w0; k < w1; ++k) sum += (cnt[k] & 0xffffu) + (cnt[k] >> 16);
  int64_t incl = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    int64_t v = lane < kW ? wsum[lane] : 0;
    for (int off = 1; off < kW; off <<= 1) {
      const int64_t y = __shfl_up(v, off);
      if (lane >= off) v += y;
    }
    if (lane < kW) wsum[lane] = v;  // inclusive wave totals
  }
  __syncthreads();
  int64_t run = incl - sum + (w > 0 ? wsum[w - 1] : 0);
  for (int k = w0; k < w1; ++k) {
    const uint32_t v = cnt[k];
    const int64_t s0 = run, s1 = run + (v & 0xffffu);
    run = s1 + (v >> 16);
    bin_start[2 * k] = s0;
    if (2 * k + 1 < nbins) bin_start[2 * k + 1] = s1;
    cnt[k] = (uint32_t)s0 | ((uint32_t)s1 << 16);
  }
  const int total = (int)wsum[kW - 1];  // atoms with finite coordinates
  if (t == kOneThreads - 1) bin_start[nbins] = total;
  __syncthreads();
  int slot[kOnePer];
#pragma unroll
  for (int r = 0; r < kOnePer; ++r) {
    const int sh = 16 * (bin[r] & 1);
    slot[r] = bin[r] < 0 ? -1 : (int)((cnt[bin[r] >> 1] >> sh) & 0xffffu) + rank[r];
  }
  __syncthreads();  // every start is read before the positions take the counts' place
#pragma unroll
  for (int r = 0; r < kOnePer; ++r) {
    if (slot[r] < 0) continue;
    slot_atom[slot[r]] = t + kOneThreads * r;
    for (int d = 0; d < 3; ++d) lds.px[d][slot[r]] = x[r][d];
  }
  __syncthreads();
  for (int k = t; k < total; k += kOneThreads) {
    const int i = slot_atom[k];
    const double y[3] = {lds.px[0][k], lds.px[1][k], lds.px[2][k]};
    int b3[3], m[3] = {0, 0, 0};
    if (!g.small) bin_coords(g, pbc, y, b3, m);
    bin_m[k] = make_int4(i, m[0], m[1], m[2]);
    bin_x[k] = make_double4(y[0], y[1], y[2], 0.0);
    if (order) order[k] = i;
  }
}

__device__ __forceinline__ uint64_t entry_key(int32_t j, int na, int nb, int nc) {
  return ((uint64_t)(uint32_t)j << 24) | ((uint64_t)(uint8_t)(na + 128) << 16) | ((uint64_t)(uint8_t)(nb + 128) << 8) |
         (uint64_t)(uint8_t)(nc + 128);
}

// Row passes, one block per group of atoms that share their candidates: a
// bin of a binned structure (candidates: the atoms of the 27 bins around
// it, with the image implied by the bin wrap and the whole-cell offsets of
// both atoms), or a whole small structure (candidates: every atom of the
// structure in every image with |n_d| <= K_d).  The candidates are staged
// in LDS once per group (of a binned group the first kCandMax; the steps
// past them read bin_m / bin_x from HBM); each wave then takes the group's
// atoms one at a time, 64 candidates per step, with the FP64 inclusion test.
//   kRowsCount: row_count[i] = number of entries.
//   kRowsKeys : also the row's keys (j, n_a, n_b, n_c), collected in LDS and
//               put in order by each key's rank among them, go to the
//               atom's slab of kslot keys, or (a longer row) to a range of
//               the overflow area reserved with one atomic; key_loc[i] says
//               where.
constexpr int kGrpWaves = 4;
constexpr int kGrpThreads = 64 * kGrpWaves;
// Blocks sharing one group (blockIdx.y), each with every gridDim.y-th set of
// kGrpWaves atoms: four while the groups are few (up to a few hundred bins
// of a cell of some thousand atoms), so that the grid still fills the chip;
// two from 16384 atoms on, where the groups alone are enough and each block
// stages its candidates for more atoms.
static int grp_split(int64_t n_atoms) { return n_atoms >= 16384 ? 2 : 4; }
constexpr int kCandMax = 768;   // a binned group's candidates past this many are read from HBM
constexpr int kKeyLds = 256;    // row keys kept in LDS; longer rows take a second pass through HBM

// Orders this wave's LDS writes before its later LDS reads of other lanes'
// data (and keeps the compiler from moving accesses across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

enum { kRowsCount = 0, kRowsKeys = 1 };

template <int MODE>
__global__ void __launch_bounds__(kGrpThreads) k_nb_rows(const int64_t* __restrict__ atom_ptr,
                                                         const uint8_t* __restrict__ pbc, int32_t B,
                                                         const StructGeom* __restrict__ geom,
                                                         const int64_t* __restrict__ bin_base,
                                                         const int64_t* __restrict__ bin_start,
                                                         const int4* __restrict__ bin_m,
                                                         const double4* __restrict__ bin_x, double r2max,
                                                         int64_t* __restrict__ row_count, int64_t n_atoms,
                                                         uint64_t* __restrict__ row_keys, int kslot,
                                                         int64_t over_len, int64_t* __restrict__ key_loc,
                                                         int64_t* __restrict__ cursor, int64_t* meta,
                                                         const int32_t* flag) {
  constexpr bool KEYS = MODE == kRowsKeys;
  if (!flag[0]) return;
  __shared__ double cx[kCandMax], cy[kCandMax], cz[kCandMax];
  __shared__ int32_t cj[kCandMax];
  __shared__ int32_t cw[3][kCandMax];  // image of a binned candidate minus the centre atom's cell offset
  __shared__ uint64_t keyw[KEYS ? kGrpWaves : 1][KEYS ? kKeyLds : 1];
  __shared__ int64_t b_start[27];
  __shared__ int32_t b_pre[28];
  __shared__ int32_t b_wr[27][3];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t n_groups = B > 0 ? bin_base[B] : 0;
  for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int c = B > 0 ? wave_search_le(bin_base, B, grp) : 0;  // the group's structure
    // the structure's geometry in registers: stores to the list below are
    // char-typed and would otherwise force reloads of it
    double h[9];
    for (int k = 0; k < 9; ++k) h[k] = geom[c].h[k];
    const int gnb[3] = {geom[c].nb[0], geom[c].nb[1], geom[c].nb[2]};
    const bool small = geom[c].small != 0;
    const bool p3[3] = {pbc[3 * c] != 0, pbc[3 * c + 1] != 0, pbc[3 * c + 2] != 0};
    const int64_t base_c = bin_base[c];
    const int64_t a_lo = bin_start[grp], a_hi = bin_start[grp + 1];
    if (a_lo + (int64_t)blockIdx.y * kGrpWaves >= a_hi) continue;  // no atoms of this group for this block
    const int K0 = small ? gnb[0] : 0, K1 = small ? gnb[1] : 0, K2 = small ? gnb[2] : 0;
    const int w1 = 2 * K1 + 1, w2 = 2 * K2 + 1;
    const int64_t nimg = (int64_t)(2 * K0 + 1) * w1 * w2;
    int64_t total;
    int64_t n_st = 0;  // binned: the candidates staged in LDS, the first kCandMax
    if (small) {
      const int n_at = (int)(a_hi - a_lo);  // <= kSmallMax <= kCandMax
      for (int t = tid; t < n_at; t += kGrpThreads) {
        const double4 x4 = bin_x[a_lo + t];
        cx[t] = x4.x;
        cy[t] = x4.y;
        cz[t] = x4.z;
        cj[t] = bin_m[a_lo + t].x;
      }
      total = (int64_t)n_at * nimg;
    } else {
      if (tid < 64) {
        int cnt_b = 0;
        if (lane < 27) {
          int64_t local = grp - base_c;
          int bi[3];
          bi[2] = (int)(local % gnb[2]);
          local /= gnb[2];
          bi[1] = (int)(local % gnb[1]);
          bi[0] = (int)(local / gnb[1]);
          const int dd[3] = {lane / 9 - 1, (lane / 3) % 3 - 1, lane % 3 - 1};
          int bb[3], wr[3] = {0, 0, 0};
          bool skip = false;
          for (int d = 0; d < 3; ++d) {
            int k = bi[d] + dd[d];
            if (k < 0 || k >= gnb[d]) {
              if (!p3[d]) {
                skip = true;
                break;
              }
              wr[d] = k < 0 ? -1 : 1;
              k -= wr[d] * gnb[d];
            }
            bb[d] = k;
          }
          int64_t b0 = 0;
          if (!skip) {
            const int64_t bin = base_c + ((int64_t)bb[0] * gnb[1] + bb[1]) * gnb[2] + bb[2];
            b0 = bin_start[bin];
            cnt_b = (int)(bin_start[bin + 1] - b0);
          }
          b_start[lane] = b0;
          for (int d = 0; d < 3; ++d) b_wr[lane][d] = p3[d] ? wr[d] : 0;
        }
        int pre = cnt_b;  // inclusive prefix of the 27 counts
        for (int off = 1; off < 32; off <<= 1) {
          const int v = __shfl_up(pre, off);
          if (lane >= off) pre += v;
        }
        if (lane < 27) b_pre[lane + 1] = pre;
        if (lane == 0) b_pre[0] = 0;
      }
      __syncthreads();
      total = b_pre[27];
      n_st = total < kCandMax ? total : kCandMax;
      for (int t = tid; t < n_st; t += kGrpThreads) {
        int lo = 0, hi = 26;  // largest b with b_pre[b] <= t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (b_pre[mid] <= t) lo = mid;
          else hi = mid - 1;
        }
        const int64_t k = b_start[lo] + (t - b_pre[lo]);
        const int4 m4 = bin_m[k];
        const double4 x4 = bin_x[k];
        cx[t] = x4.x;
        cy[t] = x4.y;
        cz[t] = x4.z;
        cj[t] = m4.x;
        cw[0][t] = p3[0] ? b_wr[lo][0] - m4.y : 0;
        cw[1][t] = p3[1] ? b_wr[lo][1] - m4.z : 0;
        cw[2][t] = p3[2] ? b_wr[lo][2] - m4.w : 0;
      }
    }
    __syncthreads();
    for (int64_t a = a_lo + (int64_t)blockIdx.y * kGrpWaves + wv; a < a_hi; a += (int64_t)kGrpWaves * gridDim.y) {
      const int4 mi4 = bin_m[a];
      const double4 xi4 = bin_x[a];
      const int32_t i = mi4.x;
      const double xi[3] = {xi4.x, xi4.y, xi4.z};
      const int mi[3] = {mi4.y, mi4.z, mi4.w};
      // one pass over the candidates; sink(slot, key) receives each entry's
      // key with slot = its position in candidate order
      bool shift_bad = false;
      auto scan = [&](auto&& sink) -> int {
        int count = 0;
        for (int64_t t0 = 0; t0 < total; t0 += kWave) {
          const int64_t t = t0 + lane;
          const bool active = t < total;
          int32_t j = 0;
          double xj[3] = {0.0, 0.0, 0.0};
          int n[3] = {0, 0, 0};
          if (active) {
            if (small) {
              const int jj = (int)(t / nimg);
              int im = (int)(t - (int64_t)jj * nimg);
              n[2] = im % w2 - K2;
              im /= w2;
              n[1] = im % w1 - K1;
              n[0] = im / w1 - K0;
              j = cj[jj];
              xj[0] = cx[jj];
              xj[1] = cy[jj];
              xj[2] = cz[jj];
            } else if (t < n_st) {
              j = cj[t];
              xj[0] = cx[t];
              xj[1] = cy[t];
              xj[2] = cz[t];
              for (int d = 0; d < 3; ++d) n[d] = p3[d] ? cw[d][t] + mi[d] : 0;
            } else {
              int lo = 0, hi = 26;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (b_pre[mid] <= t) lo = mid;
                else hi = mid - 1;
              }
              const int64_t k = b_start[lo] + (t - b_pre[lo]);
              const int4 m4 = bin_m[k];
              const double4 x4 = bin_x[k];
              j = m4.x;
              xj[0] = x4.x;
              xj[1] = x4.y;
              xj[2] = x4.z;
              const int mj[3] = {m4.y, m4.z, m4.w};
              for (int d = 0; d < 3; ++d) n[d] = p3[d] ? b_wr[lo][d] - mj[d] + mi[d] : 0;
            }
          }
          bool acc = false;
          if (active && !(j == i && n[0] == 0 && n[1] == 0 && n[2] == 0)) {
            double d[3];
            displacement64(xi, xj, h, n[0], n[1], n[2], d);
            acc = norm2_64(d) < r2max;
            if (acc && (n[0] < -127 || n[0] > 127 || n[1] < -127 || n[1] > 127 || n[2] < -127 || n[2] > 127)) {
              shift_bad = true;
              acc = false;
            }
          }
          const uint64_t m = __ballot(acc);
          if (acc) sink(count + __popcll(m & lt), entry_key(j, n[0], n[1], n[2]));
          count += __popcll(m);
        }
        return count;
      };
      const int count = scan([&](int slot, uint64_t k) {
        if (KEYS && slot < kKeyLds) keyw[wv][slot] = k;
      });
      if (lane == 0) {
        row_count[i] = count;
        if (count > kRowMax) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrTooMany);
      }
      if (__any(shift_bad) && lane == 0)
        atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrShift);
      if (KEYS && count <= kRowMax) {
        // where the row's keys go: its slab, or a range of the overflow area
        // after the N slabs, reserved with one atomic (a range past the
        // area's end means the list cannot hold the entries either; the
        // capacity check then stops the build).  A row longer than the LDS
        // buffer also reserves room for its unsorted keys and is scanned a
        // second time to write them there.
        const bool in_lds = count <= kKeyLds;
        int64_t base = i * (int64_t)kslot, raw = -1;
        if (count > kslot || !in_lds) {
          const int64_t need = in_lds ? count : 2 * (int64_t)count;
          int64_t off = 0;
          if (lane == 0) off = (int64_t)atomicAdd((unsigned long long*)cursor, (unsigned long long)need);
          off = __shfl(off, 0);
          base = off + need <= over_len ? n_atoms * (int64_t)kslot + off : -1;
          if (!in_lds && base >= 0) raw = base + count;
        }
        if (lane == 0) key_loc[i] = base;
        if (base >= 0) {
          const uint64_t* kw = keyw[wv];
          if (!in_lds) {
            uint64_t* rk = row_keys + raw;
            scan([&](int slot, uint64_t k) { rk[slot] = k; });
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            kw = rk;
          } else {
            wave_lds_sync();
          }
          uint64_t* dst = row_keys + base;
          for (int t = lane; t < count; t += kWave) {
            const uint64_t k = kw[t];
            int rank = 0;
            int u = 0;
            for (; u + 8 <= count; u += 8) {  // eight independent reads in flight
              uint64_t v[8];
#pragma unroll
              for (int q = 0; q < 8; ++q) v[q] = kw[u + q];
#pragma unroll
              for (int q = 0; q < 8; ++q) rank += v[q] < k ? 1 : 0;
            }
            for (; u < count; ++u) rank += kw[u] < k ? 1 : 0;
            dst[rank] = k;
          }
          wave_lds_sync();
        }
      }
    }
    __syncthreads();
  }
}

// After the scan of row counts: record nnz, check the capacity, and decide
// whether the fill runs (flag[1]).
__device__ void capacity_decision(const CapacityJob& cj, int64_t nnz) {
  int64_t* meta = cj.meta;
  meta[kMetaNnz] = nnz;
  meta[kMetaRebuilt] = 1;
  if (nnz > cj.capacity || (meta[kMetaErr] & (kErrShift | kErrTooMany | kErrNonFinite | kErrCell))) {
    if (nnz > cj.capacity) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrCapacity);
    meta[kMetaValid] = 0;
    cj.flag[1] = 0;
  } else {
    cj.flag[1] = 1;
  }
}

__global__ void k_nb_capacity(const int64_t* offsets, int64_t N, CapacityJob cj) {
  if (!cj.flag[0]) {
    cj.flag[1] = 0;
    cj.meta[kMetaRebuilt] = 0;
    return;
  }
  capacity_decision(cj, offsets[N]);
}

__device__ __forceinline__ void decode_key(uint64_t k, int32_t& j, char4& sv) {
  j = (int32_t)(k >> 24);
  sv.x = (signed char)((int)((k >> 16) & 255) - 128);
  sv.y = (signed char)((int)((k >> 8) & 255) - 128);
  sv.z = (signed char)((int)(k & 255) - 128);
  sv.w = 0;
}

// Writes the rows from the keys the counting pass left (key_loc), with the
// reverse entry of every entry (i -> j, n): the entry (j -> i, -n) of row j,
// whose position is found among row j's sorted keys by bisection (about
// log2(len) + 1 reads; rounds of seven independent probes, fewer dependent
// rounds but about 16 reads on a row of 100, were slower from 4096 atoms up).
// Each lane runs the searches of kEmitU entries in lockstep, so that their
// chains of dependent reads overlap.  Also records the positions of this
// build (skin reference) and marks the list valid.  LPA lanes per atom
// (64 / LPA atoms per one-wave block), each lane taking every LPA-th entry
// of the row; with
// the bin order, block b takes the atoms at slots ((b mod 8) * per + b / 8)
// * 64 / LPA + (0 .. 64 / LPA - 1), so each XCD walks a contiguous stretch
// of space and the neighbor rows it searches stay in its L2.
constexpr int kEmitU = 4;

template <int LPA>
__global__ void __launch_bounds__(64) k_nb_emit(int64_t N, const uint64_t* __restrict__ row_keys,
                                                const int64_t* __restrict__ key_loc,
                                                const int64_t* __restrict__ offsets, int32_t* __restrict__ nbr,
                                                int8_t* __restrict__ shift, int32_t* __restrict__ rev,
                                                const double* __restrict__ pos, double* __restrict__ ref_pos,
                                                const int32_t* __restrict__ order, int64_t* meta, const int32_t* flag,
                                                const int32_t* gflag) {
  if (!flag[1] || !*gflag) return;
  constexpr int kApw = kWave / LPA;  // atoms per wave
  const int lane = threadIdx.x, sl = lane % LPA;
  int64_t slot = (int64_t)blockIdx.x * kApw + lane / LPA;
  if (order) {
    const int64_t per = (gridDim.x + 7) / 8;
    slot = ((int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8) * kApw + lane / LPA;
  }
  if (slot >= N) return;  // no cross-lane operations below
  const int64_t i = order ? (int64_t)order[slot] : slot;
  if (ref_pos && sl < 3) ref_pos[3 * i + sl] = pos[3 * i + sl];
  if (blockIdx.x == 0 && lane == 0) {
    meta[kMetaValid] = 1;
    meta[kMetaBuilds] += 1;
  }
  const int64_t e0 = offsets[i];
  const int len = (int)(offsets[i + 1] - e0);
  const uint64_t* mine = row_keys + key_loc[i];
  char4* sh4 = reinterpret_cast<char4*>(shift);
  for (int t0 = sl; t0 < len; t0 += kEmitU * LPA) {
    uint64_t want[kEmitU];
    const uint64_t* theirs[kEmitU];
    int64_t f0[kEmitU];
    int lj[kEmitU], lo[kEmitU], n[kEmitU];
#pragma unroll
    for (int u = 0; u < kEmitU; ++u) {
      const int t = t0 + u * LPA;
      lo[u] = 0;
      n[u] = 0;
      lj[u] = 0;
      f0[u] = 0;
      want[u] = 0;
      theirs[u] = row_keys;
      if (t < len) {
        int32_t j;
        char4 sv;
        decode_key(mine[t], j, sv);
        nbr[e0 + t] = j;
        sh4[e0 + t] = sv;
        want[u] = entry_key((int32_t)i, -sv.x, -sv.y, -sv.z);
        f0[u] = offsets[j];
        lj[u] = (int)(offsets[j + 1] - f0[u]);
        n[u] = lj[u];
        theirs[u] = row_keys + key_loc[j];
      }
    }
    // lower bounds: the first position whose key is not below want[u] is in
    // [lo[u], lo[u] + n[u]]
    while (true) {
      bool more = false;
      uint64_t k[kEmitU];
#pragma unroll
      for (int u = 0; u < kEmitU; ++u) k[u] = n[u] > 0 ? theirs[u][lo[u] + (n[u] >> 1)] : 0;
#pragma unroll
      for (int u = 0; u < kEmitU; ++u) {
        if (n[u] > 0) {
          const int h = n[u] >> 1;
          if (k[u] < want[u]) {
            lo[u] += h + 1;
            n[u] -= h + 1;
          } else {
            n[u] = h;
          }
        }
        more |= n[u] > 0;
      }
      if (!more) break;
    }
#pragma unroll
    for (int u = 0; u < kEmitU; ++u) {
      const int t = t0 + u * LPA;
      if (t < len) {
        const bool found = lo[u] < lj[u] && theirs[u][lo[u]] == want[u];
        // a missing reverse entry cannot happen for an exactly symmetric
        // list; point at the entry itself (zero net force) and flag it
        rev[e0 + t] = (int32_t)(found ? f0[u] + lo[u] : e0 + t);
        if (!found) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrTooMany);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cluster passes: batches of small molecules
//
// flag[0]: (re)build; flag[1]: the list fits (emit); flag[2]: the generic
// passes run; flag[3]: structures the cluster passes cannot take.
// ---------------------------------------------------------------------------

constexpr int kClusterMax = 64;  // atoms of a structure the cluster passes take (one per lane)

// One wave per structure.  A structure of at most 64 atoms with no periodic
// direction has no images: lane i tests every j != i of its structure with
// the same FP64 displacement and inclusion test as the generic passes, and
// its row is the bit mask of the j inside the radius (ascending j is the
// canonical row order).  counts[i] = its length; with masks, the mask is
// kept for the emit pass.  Any other structure adds to flag[3] and sets
// flag[2] (the generic passes then build the whole list).  Non-finite positions are reported as
// in the generic binning (the list is then not valid).
__global__ void __launch_bounds__(64) k_cl_count(const double* __restrict__ pos, const int64_t* __restrict__ atom_ptr,
                                                 const uint8_t* __restrict__ pbc, double r2max,
                                                 int64_t* __restrict__ counts, int64_t* __restrict__ masks,
                                                 int64_t* meta, int32_t* flag) {
  if (!flag[0]) return;
  __shared__ double px[kClusterMax], py[kClusterMax], pz[kClusterMax];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int64_t a0 = atom_ptr[c], n = atom_ptr[c + 1] - a0;
  const uint8_t* pb = pbc + 3 * (int64_t)c;
  if (n > kClusterMax || pb[0] || pb[1] || pb[2]) {
    if (lane == 0) {
      atomicAdd(&flag[3], 1);
      atomicOr(&flag[2], 1);  // the generic passes run (every such block sets the same value)
    }
    return;
  }
  const bool in = lane < n;
  double xi[3] = {0.0, 0.0, 0.0};
  bool fin = true;
  if (in) {
    for (int k = 0; k < 3; ++k) xi[k] = pos[3 * (a0 + lane) + k];
    fin = isfinite(xi[0]) && isfinite(xi[1]) && isfinite(xi[2]);
    px[lane] = xi[0];
    py[lane] = xi[1];
    pz[lane] = xi[2];
  }
  if (__any(!fin) && lane == 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrNonFinite);
  wave_lds_sync();
  uint64_t m = 0;
  if (in) {
#pragma clang fp contract(off)
    for (int j = 0; j < (int)n; ++j) {
      if (j == lane) continue;
      const double dx = px[j] - xi[0], dy = py[j] - xi[1], dz = pz[j] - xi[2];
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 < r2max) m |= 1ull << j;
    }
    counts[a0 + lane] = fin ? __popcll(m) : 0;
    if (masks) masks[a0 + lane] = fin ? (int64_t)m : 0;
  }
}

// The rows from the masks (when the list fits and the cluster passes built
// it): one wave per structure, one row at a time, lane j writing the entry
// of j at its rank in the row.  The reverse of entry (i -> j) is the entry
// (j -> i) at the rank of i in row j.  Also the skin reference positions,
// the identity order, and the list marked valid.
__global__ void __launch_bounds__(64) k_cl_emit(const int64_t* __restrict__ atom_ptr,
                                                const int64_t* __restrict__ masks,
                                                const int64_t* __restrict__ offsets, int32_t* __restrict__ nbr,
                                                int8_t* __restrict__ shift, int32_t* __restrict__ rev,
                                                const double* __restrict__ pos, double* __restrict__ ref_pos,
                                                int32_t* __restrict__ order, int64_t* meta, const int32_t* flag) {
  if (!flag[1] || flag[2]) return;
  __shared__ uint64_t ms[kClusterMax];
  __shared__ int64_t off[kClusterMax];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int64_t a0 = atom_ptr[c];
  const int n = (int)(atom_ptr[c + 1] - a0);
  if (c == 0 && lane == 0) {
    meta[kMetaValid] = 1;
    meta[kMetaBuilds] += 1;
  }
  const bool in = lane < n;
  uint64_t mine = 0;
  int64_t mo = 0;
  if (in) {
    const int64_t i = a0 + lane;
    mine = (uint64_t)masks[i];
    mo = offsets[i];
    ms[lane] = mine;
    off[lane] = mo;
    if (ref_pos)
      for (int k = 0; k < 3; ++k) ref_pos[3 * i + k] = pos[3 * i + k];
    if (order) order[i] = (int32_t)i;
  }
  wave_lds_sync();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // lane j: the entry (i -> j) of each row i that holds j, and its reverse
  // (j -> i) at the rank of i among the bits of j's row
  char4* sh4 = reinterpret_cast<char4*>(shift);
  for (int r = 0; r < n; ++r) {
    const uint64_t mr = ms[r];
    if (in && ((mr >> lane) & 1)) {
      const int64_t e = off[r] + __popcll(mr & lt);
      nbr[e] = (int32_t)(a0 + lane);
      sh4[e] = make_char4(0, 0, 0, 0);
      const uint64_t below_r = (r == 0) ? 0ull : (~0ull >> (64 - r));
      rev[e] = (int32_t)(mo + __popcll(mine & below_r));
    }
  }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

int row_key_slot(int64_t n_atoms, int64_t capacity) {
  if (n_atoms <= 0 || capacity <= 0) return 0;
  const int64_t want = (3 * ((capacity + n_atoms - 1) / n_atoms) + 1) / 2;
  int k = 64;
  while (k < want && k < kRowMax) k <<= 1;
  return k;
}

void launch_neighbors(const NbLaunch& L, bool use_skin, double skin, bool count_only, hipStream_t s) {
  const nn_system* sys = L.sys;
  const int64_t N = sys->n_atoms;
  const int32_t B = sys->n_structs;
  const unsigned gN = (unsigned)((N + 255) / 256 > 0 ? (N + 255) / 256 : 1);
  // batches try the cluster passes first; the generic passes then run only
  // on their predicate flag[2] (else on the build flag flag[0])
  const bool try_cl = B > 1 && N > 0;
  const int32_t* gflag = try_cl ? L.flag + 2 : L.flag;
  int32_t* gflag_w = const_cast<int32_t*>(gflag);
  const bool sep_prep = use_skin || B == 0 || try_cl;  // else the geometry launch does it
  if (sep_prep)
    hipLaunchKernelGGL(k_nb_prep, dim3(1), dim3(256), 0, s, sys->atom_ptr, B, N, L.meta, L.flag, L.cursor,
                       use_skin ? 1 : 0);
  if (use_skin && L.nl && L.nl->ref_pos && N > 0)
    hipLaunchKernelGGL(k_skin_check, dim3(gN), dim3(256), 0, s, sys->pos, L.nl->ref_pos, N, 0.25 * skin * skin,
                       L.meta, L.flag, 1);
  if (try_cl) {
    hipLaunchKernelGGL(k_cl_count, dim3((unsigned)B), dim3(64), 0, s, sys->pos, sys->atom_ptr, sys->pbc,
                       L.radius * L.radius, L.counts, count_only ? (int64_t*)nullptr : L.key_loc, L.meta, L.flag);
  }
  int32_t* order = (count_only || !L.nl) ? (int32_t*)nullptr : L.nl->order;
  if (B == 1 && N <= kOneAtoms) {
    hipLaunchKernelGGL(k_nb_one, dim3(1), dim3(kOneThreads), 0, s, sys->pos, sys->atom_ptr, sys->cell, sys->pbc,
                       L.radius, L.geom, L.n_bins, L.bin_base, L.bin_start, L.bin_m, L.bin_x, order, L.counts, N,
                       L.meta, L.flag, L.cursor, sep_prep ? 0 : 1);
  } else {
    const int64_t n_zero = L.max_bins + 1;
    const unsigned gGeom = (unsigned)std::max<int64_t>(B, std::min<int64_t>((n_zero + 1023) / 1024, 4096));
    if (B > 0)
      hipLaunchKernelGGL(k_nb_geom, dim3(gGeom), dim3(64), 0, s, sys->pos, sys->atom_ptr, sys->cell, sys->pbc, B,
                         L.radius, L.geom, L.n_bins, L.bin_count, n_zero, B == 1 ? L.bin_base : (int64_t*)nullptr,
                         N, L.meta, sep_prep ? gflag_w : L.flag, L.cursor, sep_prep ? 0 : 1);
    if (B != 1) exclusive_scan_i64(L.n_bins, L.bin_base, B, L.scan_tmp, s, gflag);
    if (N > 0)
      hipLaunchKernelGGL(k_nb_bin, dim3(gN), dim3(256), 0, s, sys->pos, sys->atom_ptr, sys->pbc, B, N, L.geom,
                         L.bin_base, L.bin_count, L.atom_bin, L.bin_rank, L.counts, L.meta, gflag);
    exclusive_scan_i64(L.bin_count, L.bin_start, L.max_bins, L.scan_tmp, s, gflag, L.bin_base + B);
    if (N > 0)
      hipLaunchKernelGGL(k_nb_scatter, dim3(gN), dim3(256), 0, s, N, sys->pos, L.atom_bin, L.bin_rank, L.bin_start,
                         L.bin_m, L.bin_x, order, gflag);
  }
  const double r2 = L.radius * L.radius;
  // groups (bins) are known on the device only: a grid-stride loop over them
  const unsigned gRows = (unsigned)std::max<int64_t>(1, std::min<int64_t>(L.max_bins, 2048));
  if (N > 0) {
    if (count_only)
      hipLaunchKernelGGL(k_nb_rows<kRowsCount>, dim3(gRows, grp_split(N)), dim3(kGrpThreads), 0, s, sys->atom_ptr,
                         sys->pbc, B, L.geom, L.bin_base, L.bin_start, L.bin_m, L.bin_x, r2, L.counts, N,
                         (uint64_t*)nullptr, 0, (int64_t)0, (int64_t*)nullptr, L.cursor, L.meta, gflag);
    else
      hipLaunchKernelGGL(k_nb_rows<kRowsKeys>, dim3(gRows, grp_split(N)), dim3(kGrpThreads), 0, s, sys->atom_ptr,
                         sys->pbc, B, L.geom, L.bin_base, L.bin_start, L.bin_m, L.bin_x, r2, L.counts, N, L.row_keys,
                         L.kslot, 2 * L.capacity, L.key_loc, L.cursor, L.meta, gflag);
  }
  const CapacityJob cj{count_only ? (int64_t)INT64_MAX : L.capacity, L.meta, L.flag};
  if (N <= kScanSmall) {
    hipLaunchKernelGGL(k_scan_small<true>, dim3(1), dim3(kScanSmallThreads), 0, s, L.counts, N,
                       (const int64_t*)nullptr, L.offsets, L.flag, cj);
  } else {
    exclusive_scan_i64(L.counts, L.offsets, N, L.scan_tmp, s, L.flag);
    hipLaunchKernelGGL(k_nb_capacity, dim3(1), dim3(1), 0, s, L.offsets, N, cj);
  }
  if (count_only || N == 0) return;
  nn_nlist* nl = L.nl;
  // lanes per atom: 16 for short rows (capacity per atom, about 1.25 times
  // the mean row length when a counting pass sized the list, at most 16) and
  // for lists of 16384 atoms or more, where fewer waves with longer loops
  // serve better; 32 otherwise
  const int lpa = (L.capacity <= 16 * N || N >= 16384) ? 16 : 32;
  const int64_t nw = (N + kWave / lpa - 1) / (kWave / lpa);
  const unsigned gEmit = nl->order ? (unsigned)((nw + 7) / 8 * 8) : (unsigned)nw;  // whole rounds of the 8 XCDs
  if (lpa == 16)
    hipLaunchKernelGGL(k_nb_emit<16>, dim3(gEmit), dim3(64), 0, s, N, L.row_keys, L.key_loc, nl->offsets, nl->nbr,
                       nl->shift, nl->rev, sys->pos, nl->ref_pos, nl->order, L.meta, L.flag, gflag);
  else
    hipLaunchKernelGGL(k_nb_emit<32>, dim3(gEmit), dim3(64), 0, s, N, L.row_keys, L.key_loc, nl->offsets, nl->nbr,
                       nl->shift, nl->rev, sys->pos, nl->ref_pos, nl->order, L.meta, L.flag, gflag);
  if (try_cl)
    hipLaunchKernelGGL(k_cl_emit, dim3((unsigned)B), dim3(64), 0, s, sys->atom_ptr, L.key_loc, nl->offsets, nl->nbr,
                       nl->shift, nl->rev, sys->pos, nl->ref_pos, nl->order, L.meta, L.flag);
}

}  // namespace nnp
