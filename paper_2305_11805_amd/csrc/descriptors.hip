// mBP descriptors and their adjoint on gfx950.
//
// One 64-lane wave per atom.  The wave stages the atom's neighbors inside rc
// in LDS, sorted by species (stable).  Per neighbor the pair geometry is
// formed once from FP64 positions -- d = (x_j - x_i) + image shift, r, the
// unit vector d/r, rc - r and the cosine cutoff -- and rounded to FP32 only
// after the subtractions that would otherwise cancel (r is kept as a hi/lo
// float pair).  Everything per triplet is FP32.
//
// Forward (radial + angular descriptor, Sec. II.A / III.A):
//   radial: lane k owns radial bin k and sums over the neighbors of each
//   species segment;
//   angular: for every unordered species pair block (a <= b) the block's
//   triplets are taken 64 at a time; the bins are the sum over triplets of
//   the separable outer product  A_p(theta) * R_q(r_avg) * 2 fc fc, which
//   runs on the 4x4x1 FP32 MFMA (each lane forms one triplet's geometry, then
//   four lanes share a triplet and supply its angle and radius factors).
//
// Adjoint (forces, Sec. II: forces are derivatives of the energy): given
// lambda_i = dE_i/dG_i, produce dE_i/dd_e for every neighbor entry e.
//   radial: lane <-> neighbor;
//   angular: lane <-> neighbor j on a circular schedule: at step s lane j
//   takes the pair (j, (j + s) mod n), so every unordered pair is visited
//   once and, within one step, no two lanes touch the same partner k.  The
//   j-side gradient accumulates in registers, the k-side one is added to a
//   per-neighbor LDS slot; since no two lanes of an instruction share a slot
//   and instructions retire in program order, the sums are bitwise
//   reproducible.
#include <math.h>

#include <type_traits>

#include "common.h"

namespace nnp {

typedef float floatx4 __attribute__((ext_vector_type(4)));

struct AtomNb {
  float4 d[kMaxNb];   // unit vector d/r (x, y, z), r (hi)
  float4 f[kMaxNb];   // fc, dfc/dr, r (lo), (entry index << 4 | species) as bits
  float ir[kMaxNb];   // 1/r
  int seg[NN_MAX_SPECIES + 1];
  int n;
  int bad;
};

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Orders this wave's LDS accesses: writes before it are seen by reads after
// it in every lane, and the compiler moves no LDS access across it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// Keeps this wave's LDS accesses in program order without waiting for them
// to complete: the LDS serves one wave's instructions in the order they are
// issued, so a read issued after a write of the same address by any lane of
// the wave returns the written value.  Only the compiler has to be kept from
// moving or caching accesses across it.
__device__ __forceinline__ void wave_lds_order() { __asm__ volatile("" ::: "memory"); }
__device__ __forceinline__ int nb_species(const float4& f) { return __float_as_int(f.w) & 15; }
__device__ __forceinline__ int nb_entry(const float4& f) { return __float_as_int(f.w) >> 4; }

// The structure of atom i: the largest c < B with atom_ptr[c] <= i.  Each
// round the 64 lanes probe 64 evenly spaced positions of the remaining range
// and one ballot keeps the stretch after the last probe at or below i, so
// 2048 structures take two dependent rounds of loads instead of eleven.
// Every lane of the wave must call it (with the same i).
__device__ __forceinline__ int struct_of_atom(const int64_t* atom_ptr, int32_t B, int64_t i) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = B;  // atom_ptr[lo] <= i; the answer lies in [lo, hi)
  while (hi - lo > 1) {
    const int step = (hi - lo + 63) / 64;
    const int p = lo + lane * step;
    const uint64_t le = __ballot(p < hi && atom_ptr[p] <= i);  // a prefix of the lanes: atom_ptr does not decrease
    lo += (__popcll(le) - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// The atom a one-atom-per-block descriptor launch works on.  With the
// list's bin order (kept by the list build) the grid is whole rounds of the
// eight XCDs and block b takes slot (b mod 8) * per + b / 8 of that order:
// consecutive blocks go to different XCDs, so each XCD walks one contiguous
// stretch of space and the neighbor positions its atoms gather stay in its
// L2.  Without the order, or while the list is not valid (the order is then
// not a permutation), the slot is the atom.  -1 for slots past the atoms.
__device__ __forceinline__ int64_t atom_of_block(const int32_t* __restrict__ order, int64_t N, bool valid) {
  int64_t slot = blockIdx.x;
  if (order) slot = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  if (slot >= N) return -1;
  return (order && valid) ? (int64_t)order[slot] : slot;
}

// Blocks of such a launch: whole rounds of the eight XCDs with the order.
static inline unsigned atom_grid(int64_t N, const int32_t* order) {
  return (unsigned)(order ? (N + 7) / 8 * 8 : N);
}

constexpr int kStageRounds = 2;  // rows up to 128 entries are staged in one pass

// Packed passes: kPackAtoms atoms per wave, kPackLanes lanes per atom in the
// per-atom phases.  An atom is packed when its row has at most kPackNb
// entries; longer rows go to the one-atom kernels.
constexpr int kPackAtoms = 4;
constexpr int kPackLanes = 16;
constexpr int kPackNb = 32;
// LDS stride of a group's neighbor slots: one spare slot per group puts the
// same slot of the four groups on different LDS banks (at 32 the four
// regions start on one bank, and lanes of different atoms at the same
// offset conflict)
constexpr int kPackSlots = kPackNb + 1;

// sin and cos of x in [0, pi/2] by their Taylor series to x^11 and x^12
// (truncation below 6e-8 at pi/2), without range reduction.
__device__ __forceinline__ void sincos_quarter(float x, float& sn, float& cs) {
  const float z = x * x;
  sn = x * fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, -2.5052108e-8f, 2.7557319e-6f), -1.9841270e-4f), 8.3333333e-3f),
                        -1.6666667e-1f), 1.0f);
  cs = fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, 2.0876757e-9f, -2.7557319e-7f), 2.4801587e-5f), -1.3888889e-3f),
                        4.1666667e-2f), -0.5f), 1.0f);
}

// The staged record of one neighbor inside rc from its FP64 displacement d
// (|d|^2 = r2): (d/r, r hi), (fc, dfc/dr, r lo, entry << 4 | species), 1/r.
// rc - r is formed in FP64 (no cancellation near rc); with x = pi (rc - r) /
// (2 rc) in [0, pi/2], fc = sin^2 x and dfc/dr = -(pi / 2rc) sin 2x =
// -(pi / rc) sin x cos x, from one polynomial sine and cosine.
__device__ __forceinline__ void pair_record(const double (&d)[3], double r2, int e_rel, int sp, const DescConst& P,
                                            float4& dd, float4& ff, float& irf) {
  const double r = sqrt(r2);
  const double ir = 1.0 / r;
  const double u = P.rc64 - r;
  const float r_hi = (float)r;
  const float r_lo = (float)(r - (double)r_hi);
  float sa, ca;
  sincos_quarter((float)(P.half_pi_over_rc64 * u), sa, ca);
  const float fc = sa * sa;
  const float dfc = -P.pi_over_rc * (sa * ca);
  dd = make_float4((float)(d[0] * ir), (float)(d[1] * ir), (float)(d[2] * ir), r_hi);
  ff = make_float4(fc, dfc, r_lo, __int_as_float((e_rel << 4) | sp));
  irf = (float)ir;
}

// Stage the neighbors of atom i inside rc into LDS, sorted by species.
// Entries at r >= rc get a zero pair gradient if pg != nullptr; with d64
// the FP64 displacements are staged too ([slot][3]).
__device__ void stage_neighbors(AtomNb& nb, int64_t i, const nn_system& sys, const int64_t* __restrict__ offsets,
                                const int32_t* __restrict__ nbr, const int8_t* __restrict__ shift,
                                const DescConst& P, int64_t* meta, float4* __restrict__ pg,
                                double* d64 = nullptr, const float* __restrict__ field = nullptr,
                                float4* tw = nullptr) {
  // wave 0 does the work; every thread of the block passes the barriers
  const int lane = threadIdx.x & 63;
  const bool w0 = threadIdx.x < 64;
  // the structure's cell: only image shifts need it (with all shifts zero
  // displacement64 gives x_j - x_i exactly whatever the cell)
  double h[9];
  auto load_cell = [&]() {
    const int c = struct_of_atom(sys.atom_ptr, sys.n_structs, i);
    for (int k = 0; k < 9; ++k) h[k] = sys.cell[9 * (int64_t)c + k];
  };
  const double xi[3] = {sys.pos[3 * i], sys.pos[3 * i + 1], sys.pos[3 * i + 2]};
  const int64_t e0 = offsets[i], e1 = offsets[i + 1];
  const double rc2 = P.rc64 * P.rc64;
  const int S = P.S;
  const char4* sh4 = reinterpret_cast<const char4*>(shift);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // with a displacement field: v_i now, and per neighbor ((v_j - v_i) / r,
  // r_dot = d^ . (v_j - v_i)) into tw[slot] as the neighbor is placed
  float vx = 0.f, vy = 0.f, vz = 0.f;
  if (tw) {
    vx = field[3 * i];
    vy = field[3 * i + 1];
    vz = field[3 * i + 2];
  }
  // entry e (neighbor j of species sp, FP64 displacement d, |d|^2 = r2 <
  // rc^2) into staging slot `slot`
  auto put = [&](int64_t e, int32_t j, int slot, const double (&d)[3], double r2, int sp) {
    float4 dd, ff;
    float irf;
    pair_record(d, r2, (int)(e - e0), sp, P, dd, ff, irf);
    nb.d[slot] = dd;
    nb.f[slot] = ff;
    nb.ir[slot] = irf;
    if (tw) {
      const float dx = field[3 * (int64_t)j] - vx, dy = field[3 * (int64_t)j + 1] - vy,
                  dz = field[3 * (int64_t)j + 2] - vz;
      tw[slot] = make_float4(dx * irf, dy * irf, dz * irf, fmaf(dd.x, dx, fmaf(dd.y, dy, dd.z * dz)));
    }
    if (d64) {
      d64[3 * slot] = d[0];
      d64[3 * slot + 1] = d[1];
      d64[3 * slot + 2] = d[2];
    }
  };
  if (e1 - e0 <= kStageRounds * kWave) {
    // at most 128 entries: one pass, entry e0 + 64 r + lane in round r of
    // wave 0, held in registers; the ballots give every lane the per-species
    // counts, so each knows its slots (the same slots as the two passes below)
    if (w0) {
      bool valid[kStageRounds];
      int sp[kStageRounds];
      int32_t jr[kStageRounds];
      char4 s4r[kStageRounds];
      double d[kStageRounds][3], r2[kStageRounds];
      bool bad = false, shifted = false;
#pragma unroll
      for (int r = 0; r < kStageRounds; ++r) {
        const int64_t e = e0 + r * kWave + lane;
        jr[r] = 0;
        s4r[r] = make_char4(0, 0, 0, 0);
        if (e < e1) {
          jr[r] = nbr[e];
          s4r[r] = sh4[e];
          shifted = shifted || (s4r[r].x | s4r[r].y | s4r[r].z) != 0;
        }
      }
      if (__any(shifted)) {
        load_cell();
      } else {
        for (int k = 0; k < 9; ++k) h[k] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < kStageRounds; ++r) {
        const int64_t e = e0 + r * kWave + lane;
        valid[r] = false;
        sp[r] = 0;
        d[r][0] = d[r][1] = d[r][2] = 0.0;
        r2[r] = 0.0;
        if (e < e1) {
          const int32_t j = jr[r];
          const char4 s4 = s4r[r];
          displacement64(xi, sys.pos + 3 * (int64_t)j, h, s4.x, s4.y, s4.z, d[r]);
          r2[r] = norm2_64(d[r]);
          valid[r] = r2[r] < rc2;
          sp[r] = sys.species[j];
          if (sp[r] < 0 || sp[r] >= S) {
            bad = bad || valid[r];
            valid[r] = false;
          }
          if (!valid[r] && pg) pg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      if (__any(bad) && lane == 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrSpecies);
      int slot[kStageRounds] = {};
      int total = 0;
      for (int s2 = 0; s2 < S; ++s2) {
        if (lane == 0) nb.seg[s2] = total;
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) {
          const uint64_t m = __ballot(valid[r] && sp[r] == s2);
          if (valid[r] && sp[r] == s2) slot[r] = total + __popcll(m & lt_mask);
          total += __popcll(m);
        }
      }
      if (lane == 0) {
        nb.seg[S] = total;
        nb.n = total;
        nb.bad = 0;
      }
#pragma unroll
      for (int r = 0; r < kStageRounds; ++r)
        if (valid[r]) put(e0 + r * kWave + lane, jr[r], slot[r], d[r], r2[r], sp[r]);
    }
    __syncthreads();
    return;
  }
  load_cell();
  int cnt[NN_MAX_SPECIES];
  for (int s = 0; s < NN_MAX_SPECIES; ++s) cnt[s] = 0;
  bool bad = false;
  // pass A: count neighbors inside rc per species
  for (int64_t base = e0; w0 && base < e1; base += kWave) {
    int64_t e = base + lane;
    bool valid = false;
    int sp = 0;
    if (e < e1) {
      int32_t j = nbr[e];
      char4 s4 = sh4[e];
      double d[3];
      displacement64(xi, sys.pos + 3 * (int64_t)j, h, s4.x, s4.y, s4.z, d);
      valid = norm2_64(d) < rc2;
      sp = sys.species[j];
      if (valid && (sp < 0 || sp >= S)) {
        bad = true;
        valid = false;
      }
    }
    for (int s = 0; s < S; ++s) cnt[s] += __popcll(__ballot(valid && sp == s));
  }
  if (w0 && __any(bad) && lane == 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrSpecies);
  int total = 0;
  if (threadIdx.x == 0) {
    for (int s = 0; s < S; ++s) {
      nb.seg[s] = total;
      total += cnt[s];
    }
    nb.seg[S] = total;
    nb.n = total;
    nb.bad = total > kMaxNb;
    if (total > kMaxNb) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrTooMany);
  }
  __syncthreads();
  if (nb.bad) return;
  int run[NN_MAX_SPECIES];
  for (int s = 0; s < S; ++s) run[s] = nb.seg[s];
  // pass B: pair geometry, scattered in species order
  for (int64_t base = e0; w0 && base < e1; base += kWave) {
    int64_t e = base + lane;
    bool valid = false;
    int sp = 0;
    int32_t j = 0;
    double d[3] = {0, 0, 0};
    double r2 = 0;
    if (e < e1) {
      j = nbr[e];
      char4 s4 = sh4[e];
      displacement64(xi, sys.pos + 3 * (int64_t)j, h, s4.x, s4.y, s4.z, d);
      r2 = norm2_64(d);
      valid = r2 < rc2;
      sp = sys.species[j];
      if (sp < 0 || sp >= S) valid = false;
      if (!valid && pg) pg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    int slot = 0;
    for (int s = 0; s < S; ++s) {
      uint64_t m = __ballot(valid && sp == s);
      if (valid && sp == s) slot = run[s] + __popcll(m & lt_mask);
      run[s] += __popcll(m);
    }
    if (valid) put(e, j, slot, d, r2, sp);
  }
  __syncthreads();
}

// x^e for a small positive integer e, on an array (exponent bits outside).
template <int N>
__device__ __forceinline__ void ipow_array(const float (&x)[N], int e, float (&out)[N]) {
  float base[N];
#pragma unroll
  for (int p = 0; p < N; ++p) {
    out[p] = 1.0f;
    base[p] = x[p];
  }
  while (e) {
    if (e & 1) {
#pragma unroll
      for (int p = 0; p < N; ++p) out[p] *= base[p];
    }
    e >>= 1;
    if (e) {
#pragma unroll
      for (int p = 0; p < N; ++p) base[p] *= base[p];
    }
  }
}

// x^E for a compile-time E (fully unrolled); E = 0 selects the runtime loop.
template <int E, int N>
__device__ __forceinline__ void ipow_sel(const float (&x)[N], int e_runtime, float (&out)[N]) {
  if constexpr (E == 0) {
    ipow_array<N>(x, e_runtime, out);
  } else {
    float base[N];
    bool first = true;
#pragma unroll
    for (int p = 0; p < N; ++p) base[p] = x[p];
#pragma unroll
    for (int bit = 0; bit < 11; ++bit) {
      if ((E >> bit) == 0) break;
      if ((E >> bit) & 1) {
#pragma unroll
        for (int p = 0; p < N; ++p) out[p] = first ? base[p] : out[p] * base[p];
        first = false;
      }
      if ((E >> (bit + 1)) != 0) {
#pragma unroll
        for (int p = 0; p < N; ++p) base[p] *= base[p];
      }
    }
  }
}

// q = t / n, r = t mod n for 0 <= t < 2^24 and 0 < n < 2^12, through a
// float reciprocal: the float quotient is off by at most one.
__device__ __forceinline__ void divmod_small(int t, int n, float inv_n, int& q, int& r) {
  q = (int)((float)t * inv_n);
  r = t - q * n;
  if (r < 0) {
    --q;
    r += n;
  } else if (r >= n) {
    ++q;
    r -= n;
  }
}

__device__ __forceinline__ int pair_block(int S, int a, int b) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  return a * S - a * (a - 1) / 2 + (b - a);
}

// Angle terms of one triplet from the two unit vectors: cos(theta), the
// smoothed sine sqrt(sin^2 + eps), and the average radius as hi (exact half
// of a rounded sum) + lo (the rounding error of that sum plus the lo parts).
struct TripGeom {
  float c, ssm, rbar, rbar_lo;
};

// EXACT_SQRT: the correctly rounded square root (descriptor values); the
// gradient passes take the hardware's 1-ulp one.
template <bool EXACT_SQRT = true>
__device__ __forceinline__ TripGeom triplet_geom(const float4& u, const float4& fu, const float4& v, const float4& fv,
                                                 float eps) {
  TripGeom t;
  t.c = fmaf(u.x, v.x, fmaf(u.y, v.y, u.z * v.z));
  const float cx = fmaf(u.y, v.z, -u.z * v.y);
  const float cy = fmaf(u.z, v.x, -u.x * v.z);
  const float cz = fmaf(u.x, v.y, -u.y * v.x);
  const float s2 = fmaf(cx, cx, fmaf(cy, cy, fmaf(cz, cz, eps)));
  t.ssm = EXACT_SQRT ? sqrtf(s2) : __builtin_amdgcn_sqrtf(s2);
  const float s = u.w + v.w;  // TwoSum: s + err == u.w + v.w exactly
  const float bb = s - u.w;
  const float err = (u.w - (s - bb)) + (v.w - bb);
  t.rbar = 0.5f * s;
  t.rbar_lo = 0.5f * (err + fu.z + fv.z);
  return t;
}

// ZC selects the angular term: a compile-time mBP exponent (50), 0 for a
// run-time mBP exponent, or kZcBP for the standard BP term.
constexpr int kZcBP = -1;

// x^e for a run-time 0 <= e < 2^nbits (binary exponentiation over a
// wave-uniform number of bits, so lanes with different e do not diverge).
__device__ __forceinline__ float ipow_rt(float x, int e, int nbits) {
  float r = 1.0f;
  for (int b = 0; b < nbits; ++b) {
    r = ((e >> b) & 1) ? r * x : r;
    x *= x;
  }
  return r;
}

// x^e for a run-time e >= 0 that is the same in every lane.
__device__ __forceinline__ float ipow_uniform(float x, int e) {
  float r = 1.0f;
  while (e) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}


// Standard BP triplet terms from the two staged neighbors (unit vector,
// r): cos(theta), s2 = r_ij^2 + r_ik^2 + r_jk^2, the third side w = d_k -
// d_j and its cutoff fc(r_jk) (with the derivative when DERIV).
struct BpGeom {
  float c, s2, wx, wy, wz, rw, fw, dfw;
};
template <bool DERIV>
__device__ __forceinline__ BpGeom bp_geom(const float4& u, const float4& v, const DescConst& P) {
  BpGeom g;
  g.c = fmaf(u.x, v.x, fmaf(u.y, v.y, u.z * v.z));
  g.wx = fmaf(v.w, v.x, -u.w * u.x);
  g.wy = fmaf(v.w, v.y, -u.w * u.y);
  g.wz = fmaf(v.w, v.z, -u.w * u.z);
  const float rw2 = fmaf(g.wx, g.wx, fmaf(g.wy, g.wy, g.wz * g.wz));
  g.rw = sqrtf(rw2);
  g.s2 = fmaf(u.w, u.w, fmaf(v.w, v.w, rw2));
  g.fw = 0.f;
  g.dfw = 0.f;
  if (g.rw < P.rc) {
    float sn, cs;
    sincos_quarter(P.half_pi_over_rc * (P.rc - g.rw), sn, cs);
    g.fw = sn * sn;  // sin^2(pi (rc - r) / (2 rc))
    if (DERIV) g.dfw = -2.0f * P.half_pi_over_rc * sn * cs;
  }
  return g;
}

// The third side w = d_k - d_j from the FP64 displacements of the two
// neighbors, and its cutoff with rc - r_jk = (rc^2 - r_jk^2) / (rc + r_jk),
// so that fc(r_jk) and its derivative keep their relative precision up to
// rc (r_jk itself only enters that denominator).
struct BpSide {
  float wx, wy, wz, rw2, rw, fw, dfw;
};
__device__ __forceinline__ BpSide bp_side64(const double* __restrict__ dj, const double* __restrict__ dk,
                                            const DescConst& P) {
  BpSide b;
  const double wx = dk[0] - dj[0], wy = dk[1] - dj[1], wz = dk[2] - dj[2];
  const double rw2 = fma(wx, wx, fma(wy, wy, wz * wz));
  b.wx = (float)wx;
  b.wy = (float)wy;
  b.wz = (float)wz;
  b.rw2 = (float)rw2;
  b.rw = __builtin_amdgcn_sqrtf(b.rw2);
  b.fw = 0.f;
  b.dfw = 0.f;
  if (rw2 < P.rc64 * P.rc64) {
    float sn, cs;
    sincos_quarter(P.half_pi_over_rc * (float)(fma(P.rc64, P.rc64, -rw2)) * frcp(P.rc + b.rw), sn, cs);
    b.fw = sn * sn;
    b.dfw = -2.0f * P.half_pi_over_rc * sn * cs;
  }
  return b;
}

constexpr int kFuseTriplets = 256;  // triplets per atom for the pair-block-per-MFMA-block forward

// The descriptor row of atom i by the block (WPA waves).
template <int NT, int NRA, int WPA, int ZC>
__device__ __forceinline__ void desc_fwd_atom(int64_t i, bool list_ok, const nn_system& sys,
                                              const int64_t* __restrict__ offsets, const int32_t* __restrict__ nbr,
                                              const int8_t* __restrict__ shift, const DescConst& P,
                                              float* __restrict__ G, int64_t* meta) {
  constexpr int NB = NT * NRA;
  __shared__ AtomNb nb;
  // per-wave partial sums (radial bins: S * n_rad <= 512; angular block: NB)
  __shared__ float xch[WPA > 1 ? WPA * NN_MAX_SPECIES * kMaxRad : 1];
  __shared__ float4 tgeo[WPA][kWave];  // per chunk: cos, smoothed sine, average radius (hi, lo)
  __shared__ float tf2[WPA][kWave];    // and 2 fc fc
  __shared__ double d64[ZC == kZcBP ? 3 * kMaxNb : 1];  // BP: FP64 displacements for the third side
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  float* Gi = G + i * (int64_t)P.D;
  if (!list_ok) {  // no valid list: never read its entries
    for (int d = tid; d < P.D; d += 64 * WPA) Gi[d] = 0.f;
    return;
  }
  stage_neighbors(nb, i, sys, offsets, nbr, shift, P, meta, nullptr, ZC == kZcBP ? d64 : nullptr);
  if (nb.bad) {
    for (int d = tid; d < P.D; d += 64 * WPA) Gi[d] = 0.f;
    return;
  }
  const int S = P.S;
  const float eta_r2 = P.eta_rad * 1.4426950408889634f;
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  // radial bins: lane k owns bin k; wave w sums the neighbors t = w mod WPA
  for (int k0 = 0; k0 < P.n_rad; k0 += kWave) {
    const int k = k0 + lane;
    const float rs = k < P.n_rad ? P.rs_rad[k] : 0.f;
    const float rs_lo = k < P.n_rad ? P.rs_rad_lo[k] : 0.f;
    for (int s = 0; s < S; ++s) {
      float acc = 0.f;
      for (int t = nb.seg[s] + wv; t < nb.seg[s + 1]; t += WPA) {
        const float dr = (nb.d[t].w - rs) + (nb.f[t].z - rs_lo);
        acc = fmaf(fexp2(-eta_r2 * dr * dr), nb.f[t].x, acc);
      }
      if constexpr (WPA == 1) {
        if (k < P.n_rad) Gi[s * P.n_rad + k] = acc;
      } else {
        if (k < P.n_rad) xch[wv * NN_MAX_SPECIES * kMaxRad + s * P.n_rad + k] = acc;
      }
    }
    if constexpr (WPA > 1) {
      __syncthreads();
      for (int x = tid; x < S * P.n_rad; x += 64 * WPA) {
        const int s = x / P.n_rad, kk = x - s * P.n_rad;
        if (kk < k0 || kk >= k0 + kWave) continue;
        float v = 0.f;
        for (int w = 0; w < WPA; ++w) v += xch[w * NN_MAX_SPECIES * kMaxRad + x];
        Gi[x] = v;
      }
      __syncthreads();
    }
  }
  const int ang0 = P.n_rad * S;
  constexpr int NP = NT / 4, NQ = NRA / 4;
  const int li = lane & 3, blk = lane >> 2;
  // this lane's angle terms p = 4u + li and radius terms q = 4v + li
  float xa[NP], xb[NP], rsq[NQ], rsq_lo[NQ];
  int zexp[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    if constexpr (ZC == kZcBP) {
      xa[u] = P.bp_pref[4 * u + li];
      xb[u] = P.bp_lam[4 * u + li];
      zexp[u] = P.bp_zeta[4 * u + li];
    } else {
      xa[u] = P.x_a[4 * u + li];
      xb[u] = P.x_b[4 * u + li];
      zexp[u] = 0;
    }
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    if constexpr (ZC == kZcBP) {
      rsq[u] = P.bp_eta[4 * u + li] * 1.4426950408889634f;
      rsq_lo[u] = 0.f;
    } else {
      rsq[u] = P.rs_ang[4 * u + li];
      rsq_lo[u] = P.rs_ang_lo[4 * u + li];
    }
  }
  // one triplet's geometry: (cos, smoothed sine, average radius hi, lo)
  // and 2 fc fc for mBP; (1 + cos, 1 - cos, sum of the squared sides) and
  // the three cutoffs for BP
  auto trip_geom = [&](int j, int k, float4& geo, float& F2) {
    const float4 fu = nb.f[j], fv = nb.f[k];
    if constexpr (ZC == kZcBP) {
      // 1 + cos and 1 - cos as |u^ +- v^|^2 / 2 (no cancellation near
      // cos = -+1); the third side from the FP64 displacements, with
      // rc - r_jk = (rc^2 - r_jk^2) / (rc + r_jk), so that its cutoff
      // keeps its relative precision up to rc
      const float4 u = nb.d[j], v = nb.d[k];
      const float px = u.x + v.x, py = u.y + v.y, pz = u.z + v.z;
      const float mx = u.x - v.x, my = u.y - v.y, mz = u.z - v.z;
      const BpSide w3 = bp_side64(d64 + 3 * j, d64 + 3 * k, P);
      geo = make_float4(0.5f * fmaf(px, px, fmaf(py, py, pz * pz)), 0.5f * fmaf(mx, mx, fmaf(my, my, mz * mz)),
                        fmaf(u.w, u.w, fmaf(v.w, v.w, w3.rw2)), 0.f);
      F2 = fu.x * fv.x * w3.fw;  // three cutoffs
    } else {
      const TripGeom g = triplet_geom(nb.d[j], fu, nb.d[k], fv, P.eps_ang);
      geo = make_float4(g.c, g.ssm, g.rbar, g.rbar_lo);
      F2 = 2.0f * fu.x * fv.x;
    }
  };
  // this lane's factors of one triplet: angle terms A_(4u+li) and radius
  // terms R_(4v+li) F2
  auto lane_factors = [&](const float4& q4, float f2, float (&A)[NP], float (&R)[NQ]) {
    if constexpr (ZC == kZcBP) {
      // 2^(2 - zeta) (1 + lambda cos)^zeta and exp(-eta s2) fc fc fc
#pragma unroll
      for (int u = 0; u < NP; ++u) A[u] = xa[u] * ipow_rt(xb[u] > 0.f ? q4.x : q4.y, zexp[u], P.bp_zbits);
#pragma unroll
      for (int v = 0; v < NQ; ++v) R[v] = fexp2(-rsq[v] * q4.z) * f2;
    } else {
      float x[NP];
#pragma unroll
      for (int u = 0; u < NP; ++u) x[u] = fmaf(q4.x, xa[u], fmaf(q4.y, xb[u], P.x_c));
      ipow_sel<(ZC > 0 ? ZC : 0), NP>(x, P.zeta, A);
#pragma unroll
      for (int v = 0; v < NQ; ++v) {
        const float dq = (q4.z - rsq[v]) + (q4.w - rsq_lo[v]);
        R[v] = fexp2(-eta_a2 * dq * dq) * f2;
      }
    }
  };
  // triplet t of species-pair block (a, b), m = na (a == b) or nbb (a < b):
  // a == b numbers the unordered pairs {j, (j + s) mod na} as (s - 1) na + j,
  // a < b every (j, k) of the two segments as j nbb + k
  auto decode = [&](int t, int a, int b, int m, float inv_m, int& j, int& k) {
    int q, r;
    divmod_small(t, m, inv_m, q, r);
    if (a == b) {
      int kk = r + q + 1;
      if (kk >= m) kk -= m;
      j = nb.seg[a] + r;
      k = nb.seg[a] + kk;
    } else {
      j = nb.seg[a] + q;
      k = nb.seg[b] + r;
    }
  };
  // Few triplets (a small molecule with several species): one chunk of 64
  // triplets, a reduction and the stores per species-pair block would
  // mostly idle.  Instead 4-lane MFMA block b of the (single) wave takes
  // species-pair block b (S(S+1)/2 <= 16) and walks its triplets, its lane
  // i supplying A_(4u+i) and R_(4v+i) F2 of each, so that the block's
  // accumulators end up holding exactly that pair block's bins: no
  // reduction across lanes.  The four lanes of a block form each of its
  // triplets' geometry themselves, except for the BP term (whose third side
  // is an FP64 computation) with at most 64 triplets: then each lane first
  // forms one triplet's geometry (numbered block after block) into LDS and
  // the blocks read it back.
  const int nblk = S * (S + 1) / 2;
  const int Tall = nb.n * (nb.n - 1) / 2;
  if (WPA == 1 && nblk > 1 && nblk <= 16 && Tall <= kFuseTriplets) {
    int pa = 0, rem = blk < nblk ? blk : 0;
    while (rem >= S - pa) {
      rem -= S - pa;
      ++pa;
    }
    const int pb = pa + rem;
    const int na = nb.seg[pa + 1] - nb.seg[pa], nbb = nb.seg[pb + 1] - nb.seg[pb];
    const int Tb = blk < nblk ? (pa == pb ? na * (na - 1) / 2 : na * nbb) : 0;
    int Tmax = Tb;
    for (int o = 32; o >= 1; o >>= 1) Tmax = max(Tmax, __shfl_xor(Tmax, o));
    const int m = pa == pb ? na : nbb;
    const float inv_m = m > 0 ? 1.0f / (float)m : 0.f;
    const bool staged = ZC == kZcBP && Tall <= kWave;
    int base = 0;  // first triplet of this lane's block in the block-after-block numbering
    if (staged) {
      float4 geo = make_float4(1.f, 0.f, 0.f, 0.f);
      float F2 = 0.f;
      int c = 0, acc_t = 0;
      for (int a = 0; a < S; ++a)
        for (int b = a; b < S; ++b, ++c) {
          const int ma = nb.seg[a + 1] - nb.seg[a], mb = nb.seg[b + 1] - nb.seg[b];
          const int Tc = a == b ? ma * (ma - 1) / 2 : ma * mb;
          if (c < blk) base += Tc;
          if (lane >= acc_t && lane < acc_t + Tc) {
            const int mm = a == b ? ma : mb;
            int j, k;
            decode(lane - acc_t, a, b, mm, 1.0f / (float)mm, j, k);
            trip_geom(j, k, geo, F2);
          }
          acc_t += Tc;
        }
      tgeo[0][lane] = geo;
      tf2[0][lane] = F2;
      wave_lds_sync();
    }
    floatx4 acc[NP][NQ];
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < Tmax; ++t) {
      float4 q4 = make_float4(1.f, 0.f, 0.f, 0.f);  // past the block's triplets: F2 = 0 adds nothing
      float f2 = 0.f;
      if (t < Tb) {
        if (staged) {
          q4 = tgeo[0][base + t];
          f2 = tf2[0][base + t];
        } else {
          int j, k;
          decode(t, pa, pb, m, inv_m, j, k);
          trip_geom(j, k, q4, f2);
        }
      }
      float A[NP], R[NQ];
      lane_factors(q4, f2, A, R);
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[u], R[v], acc[u][v], 0, 0, 0);
    }
    if (blk < nblk) {
      float* out = Gi + ang0 + blk * NB;  // blk is the pair block's index in the layout order
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[(4 * v + li) * NT + 4 * u + r] = acc[u][v][r];
    }
    return;
  }
  for (int a = 0; a < S; ++a) {
    for (int b = a; b < S; ++b) {
      const int na = nb.seg[a + 1] - nb.seg[a], nbb = nb.seg[b + 1] - nb.seg[b];
      const int T = (a == b) ? na * (na - 1) / 2 : na * nbb;
      floatx4 acc[NP][NQ];
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
      const int m = (a == b) ? na : nbb;
      const float inv_m = m > 0 ? 1.0f / (float)m : 0.f;
      for (int t0 = wv * kWave; t0 < T; t0 += kWave * WPA) {
        const int t = t0 + lane;
        float4 geo = make_float4(1.f, 0.f, 0.f, 0.f);
        float F2 = 0.f;  // zero past the block's triplets: such rows add nothing
        if (t < T) {
          int j, k;
          decode(t, a, b, m, inv_m, j, k);
          trip_geom(j, k, geo, F2);
        }
        tgeo[wv][lane] = geo;
        tf2[wv][lane] = F2;
        wave_lds_sync();
        const int ng = (min(T - t0, kWave) + 15) >> 4;  // groups of 16 triplets holding any of the block's
        for (int gi = 0; gi < ng; ++gi) {
          const float4 q4 = tgeo[wv][16 * gi + blk];
          const float f2 = tf2[wv][16 * gi + blk];
          float A[NP], R[NQ];
          lane_factors(q4, f2, A, R);
#pragma unroll
          for (int u = 0; u < NP; ++u)
#pragma unroll
            for (int v = 0; v < NQ; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[u], R[v], acc[u][v], 0, 0, 0);
        }
        wave_lds_sync();  // this chunk's reads are done before the next chunk's writes
      }
      // sum over the 16 blocks (lanes of equal lane mod 4); lanes 0..3 then
      // hold bin (p = 4u + r, q = 4v + lane)
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float y = acc[u][v][r];
            y += __shfl_xor(y, 4);
            y += __shfl_xor(y, 8);
            y += __shfl_xor(y, 16);
            y += __shfl_xor(y, 32);
            acc[u][v][r] = y;
          }
      float* out = Gi + ang0 + pair_block(S, a, b) * NB;
      if (lane < 4) {
#pragma unroll
        for (int u = 0; u < NP; ++u)
#pragma unroll
          for (int v = 0; v < NQ; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int bin = (4 * v + lane) * NT + 4 * u + r;
              if constexpr (WPA == 1) out[bin] = acc[u][v][r];
              else xch[wv * NB + bin] = acc[u][v][r];
            }
      }
      if constexpr (WPA > 1) {
        __syncthreads();
        for (int x = tid; x < NB; x += 64 * WPA) {
          float v = 0.f;
          for (int w = 0; w < WPA; ++w) v += xch[w * NB + x];
          out[x] = v;
        }
        __syncthreads();
      }
    }
  }
}

// With one species the descriptor launch also writes the identity grouping.
__device__ __forceinline__ void identity_group(IdentityGroup one, const nn_system& sys, int64_t i, int64_t* meta) {
  one.perm[i] = (int32_t)i;
  if (sys.species[i] != 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrSpecies);
  if (i == 0) {
    one.sp_start[0] = 0;
    one.sp_start[1] = sys.n_atoms;
  }
}

template <int NT, int NRA, int WPA, int ZC>
__global__ void __launch_bounds__(64 * WPA) k_desc_fwd(nn_system sys, const int64_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ nbr,
                                                       const int8_t* __restrict__ shift, DescConst P,
                                                       float* __restrict__ G, int64_t* meta, IdentityGroup one,
                                                       const int32_t* __restrict__ order) {
  const bool list_ok = meta[kMetaValid] == 1;
  const int64_t i = atom_of_block(order, sys.n_atoms, list_ok);
  if (i < 0) return;
  if (one.perm && threadIdx.x == 0) identity_group(one, sys, i, meta);
  desc_fwd_atom<NT, NRA, WPA, ZC>(i, list_ok, sys, offsets, nbr, shift, P, G, meta);
}

// The atoms a packed launch leaves out (rows over kPackNb entries), one
// wave per block of 64 atom slots: the lanes test their slots' rows and the
// wave then takes the long ones one after another.  Also writes the
// identity grouping of all atoms.  Nothing else to do while the list is not
// valid (the packed launch zeroes every row then).
template <int NT, int NRA, int ZC>
__global__ void __launch_bounds__(64) k_desc_fwd_long(nn_system sys, const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ nbr,
                                                      const int8_t* __restrict__ shift, DescConst P,
                                                      float* __restrict__ G, int64_t* meta, IdentityGroup one,
                                                      const int32_t* __restrict__ order) {
  const bool list_ok = meta[kMetaValid] == 1;
  const int64_t slot = (int64_t)blockIdx.x * kWave + threadIdx.x;
  const bool in = slot < sys.n_atoms;
  const int64_t i = !in ? -1 : (order && list_ok) ? (int64_t)order[slot] : slot;
  if (one.perm && in) identity_group(one, sys, i, meta);
  if (!list_ok) return;
  uint64_t m = __ballot(in && offsets[i + 1] - offsets[i] > kPackNb);
  while (m) {
    const int b = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    desc_fwd_atom<NT, NRA, 1, ZC>(__shfl(i, b), true, sys, offsets, nbr, shift, P, G, meta);
    __syncthreads();  // this atom's LDS reads are done before the next one's staging
  }
}

// Directional derivative of the descriptors along a displacement field v
// [N][3] (the forward-mode product that the weight gradient of a loss on
// forces needs, Sec. II.A with forces as derivatives of the energy):
//   u_i = sum_k (dG_i/dx_k) v_k = sum over neighbors j of (dG_i/dd_ij) (v_j - v_i).
// Same neighbor staging, work split and sums as k_desc_fwd, with each
// radial or triplet term replaced by its derivative along the field:
//   radial: d/de g(r) = g'(r) r_dot with r_dot = d^ . (v_j - v_i);
//   angular: d/de [A_p R_q F2] = A_p_dot R_q F2 + A_p R_q (F2_dot + F2 R_q_dot / R_q),
//   cos_dot = v^ . w_j + u^ . w_k - cos (r_dot_j / r_j + r_dot_k / r_k) with
//   w = (v_j - v_i) / r, ssm_dot = -cos cos_dot / ssm.
template <int NT, int NRA, int WPA, int ZC>
__global__ void __launch_bounds__(64 * WPA) k_desc_tan(nn_system sys, const int64_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ nbr,
                                                       const int8_t* __restrict__ shift, DescConst P,
                                                       const float* __restrict__ field, float* __restrict__ U,
                                                       int64_t* meta, const int32_t* __restrict__ order) {
  constexpr int NB = NT * NRA;
  __shared__ AtomNb nb;
  __shared__ float4 tw[kMaxNb];  // per neighbor: (v_j - v_i) / r, and r_dot
  __shared__ float xch[WPA > 1 ? WPA * NN_MAX_SPECIES * kMaxRad : 1];
  __shared__ float4 tgeo[WPA][kWave], tdot[WPA][kWave];  // per chunk: geometry; F2, zeta cos_dot, zeta ssm_dot, F2_dot
  __shared__ float tg2[WPA][kWave];                      // and -2 eta r_dot F2
  __shared__ double d64[ZC == kZcBP ? 3 * kMaxNb : 1];  // BP: FP64 displacements for the third side
  const bool list_ok = meta[kMetaValid] == 1;
  const int64_t i = atom_of_block(order, sys.n_atoms, list_ok);
  if (i < 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  float* Ui = U + i * (int64_t)P.D;
  if (!list_ok) {
    for (int d = tid; d < P.D; d += 64 * WPA) Ui[d] = 0.f;
    return;
  }
  stage_neighbors(nb, i, sys, offsets, nbr, shift, P, meta, nullptr, ZC == kZcBP ? d64 : nullptr, field, tw);
  if (nb.bad) {
    for (int d = tid; d < P.D; d += 64 * WPA) Ui[d] = 0.f;
    return;
  }
  const int S = P.S;
  const float eta_r2 = P.eta_rad * 1.4426950408889634f;
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  for (int k0 = 0; k0 < P.n_rad; k0 += kWave) {
    const int k = k0 + lane;
    const float rs = k < P.n_rad ? P.rs_rad[k] : 0.f;
    const float rs_lo = k < P.n_rad ? P.rs_rad_lo[k] : 0.f;
    for (int s = 0; s < S; ++s) {
      float acc = 0.f;
      for (int t = nb.seg[s] + wv; t < nb.seg[s + 1]; t += WPA) {
        const float4 f = nb.f[t];
        const float dr = (nb.d[t].w - rs) + (f.z - rs_lo);
        const float g = fexp2(-eta_r2 * dr * dr);
        acc = fmaf(g * fmaf(-2.0f * P.eta_rad * dr, f.x, f.y), tw[t].w, acc);
      }
      if constexpr (WPA == 1) {
        if (k < P.n_rad) Ui[s * P.n_rad + k] = acc;
      } else {
        if (k < P.n_rad) xch[wv * NN_MAX_SPECIES * kMaxRad + s * P.n_rad + k] = acc;
      }
    }
    if constexpr (WPA > 1) {
      __syncthreads();
      for (int x = tid; x < S * P.n_rad; x += 64 * WPA) {
        const int s = x / P.n_rad, kk = x - s * P.n_rad;
        if (kk < k0 || kk >= k0 + kWave) continue;
        float v = 0.f;
        for (int w = 0; w < WPA; ++w) v += xch[w * NN_MAX_SPECIES * kMaxRad + x];
        Ui[x] = v;
      }
      __syncthreads();
    }
  }
  // angular blocks: the tangent bins are the sum over triplets of
  // A_dot_p (R_q F2) + A_p R_q (F2_dot - 2 eta dq r_dot F2), two outer
  // products per triplet on the 4x4x1 FP32 MFMA, with the same lane roles as
  // the forward pass (one triplet's geometry and tangents per lane into LDS,
  // then four lanes per triplet supply its factors)
  const int ang0 = P.n_rad * S;
  const int zeta1 = P.zeta - 1;
  const float zf = (float)P.zeta;
  constexpr int NP = NT / 4, NQ = NRA / 4;
  const int li = lane & 3, blk = lane >> 2;
  float xa[NP], xb[NP], rsq[NQ], rsq_lo[NQ];
  int zexp[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    if constexpr (ZC == kZcBP) {  // prefactor, lambda, zeta of angle term 4u + li
      xa[u] = P.bp_pref[4 * u + li];
      xb[u] = P.bp_lam[4 * u + li];
      zexp[u] = P.bp_zeta[4 * u + li];
    } else {
      xa[u] = P.x_a[4 * u + li];
      xb[u] = P.x_b[4 * u + li];
      zexp[u] = 0;
    }
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    if constexpr (ZC == kZcBP) {  // eta log2(e) and eta of radius term 4u + li
      rsq[u] = P.bp_eta[4 * u + li] * 1.4426950408889634f;
      rsq_lo[u] = P.bp_eta[4 * u + li];
    } else {
      rsq[u] = P.rs_ang[4 * u + li];
      rsq_lo[u] = P.rs_ang_lo[4 * u + li];
    }
  }
  // one triplet's geometry and tangents: (cos, ...) in geo, the factors'
  // tangents in dot and g2 (the layout the factor step below reads)
  auto trip_terms = [&](int j, int k, float4& geo, float4& dot, float& g2) {
    const float4 u = nb.d[j], v = nb.d[k];
    const float4 fu = nb.f[j], fv = nb.f[k];
    const float4 wj = tw[j], wk = tw[k];
    const float cdot0 = fmaf(v.x, wj.x, fmaf(v.y, wj.y, v.z * wj.z)) + fmaf(u.x, wk.x, fmaf(u.y, wk.y, u.z * wk.z));
    if constexpr (ZC == kZcBP) {
      // s2_dot = 2 (r_j r_j_dot + r_k r_k_dot + w . (delta_k - delta_j)),
      // F3_dot = fc'_j r_j_dot fc_k fc_w + fc_j fc'_k r_k_dot fc_w + fc_j fc_k fc'_w (w^ . (delta_k - delta_j))
      const BpSide g = bp_side64(d64 + 3 * j, d64 + 3 * k, P);
      const float c = fmaf(u.x, v.x, fmaf(u.y, v.y, u.z * v.z));
      const float cdot = cdot0 - c * fmaf(wj.w, nb.ir[j], wk.w * nb.ir[k]);
      const float ddx = fmaf(wk.x, v.w, -wj.x * u.w), ddy = fmaf(wk.y, v.w, -wj.y * u.w),
                  ddz = fmaf(wk.z, v.w, -wj.z * u.w);
      const float wdd = fmaf(g.wx, ddx, fmaf(g.wy, ddy, g.wz * ddz));
      const float s2dot = 2.0f * fmaf(u.w, wj.w, fmaf(v.w, wk.w, wdd));
      const float F3 = fu.x * fv.x * g.fw;
      const float F3dot = fmaf(fu.y * wj.w, fv.x * g.fw, fu.x * fv.y * wk.w * g.fw) +
                          (g.rw > 0.f ? fu.x * fv.x * g.dfw * wdd * frcp(g.rw) : 0.f);
      geo = make_float4(c, fmaf(u.w, u.w, fmaf(v.w, v.w, g.rw2)), 0.f, 0.f);
      dot = make_float4(F3, cdot, F3dot, 0.f);
      g2 = s2dot * F3;
    } else {
      const TripGeom g = triplet_geom(u, fu, v, fv, P.eps_ang);
      const float cdot = cdot0 - g.c * fmaf(wj.w, nb.ir[j], wk.w * nb.ir[k]);
      const float sdot = -g.c * cdot * frcp(g.ssm);
      const float F2 = 2.0f * fu.x * fv.x;
      const float F2dot = 2.0f * fmaf(fu.y * wj.w, fv.x, fu.x * fv.y * wk.w);
      const float rbdot = 0.5f * (wj.w + wk.w);
      geo = make_float4(g.c, g.ssm, g.rbar, g.rbar_lo);
      dot = make_float4(F2, zf * cdot, zf * sdot, F2dot);
      g2 = -2.0f * P.eta_ang * rbdot * F2;
    }
  };
  // this lane's factors of one triplet: angle terms 4u + li and radius terms
  // 4v + li with their tangents
  auto lane_factors = [&](const float4& q4, const float4& d4, float h2, float (&A)[NP], float (&Ad)[NP],
                          float (&RF)[NQ], float (&RT)[NQ]) {
    if constexpr (ZC == kZcBP) {
      // A = pref base^zeta, A_dot = pref zeta lambda base^(zeta-1) cos_dot;
      // R F3 and R (F3_dot - eta s2_dot F3)
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const float base = fmaf(xb[u], q4.x, 1.0f);
        const float P1 = ipow_rt(base, zexp[u] - 1, P.bp_zbits);
        A[u] = xa[u] * P1 * base;
        Ad[u] = xa[u] * (float)zexp[u] * xb[u] * P1 * d4.y;
      }
#pragma unroll
      for (int v = 0; v < NQ; ++v) {
        const float R = fexp2(-rsq[v] * q4.y);
        RF[v] = R * d4.x;
        RT[v] = R * fmaf(-rsq_lo[v], h2, d4.z);
      }
    } else {
      float x[NP], P1[NP];
#pragma unroll
      for (int u = 0; u < NP; ++u) x[u] = fmaf(q4.x, xa[u], fmaf(q4.y, xb[u], P.x_c));
      ipow_sel<(ZC > 0 ? ZC - 1 : 0), NP>(x, zeta1, P1);
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        A[u] = P1[u] * x[u];
        Ad[u] = P1[u] * fmaf(xa[u], d4.y, xb[u] * d4.z);
      }
#pragma unroll
      for (int v = 0; v < NQ; ++v) {
        const float dq = (q4.z - rsq[v]) + (q4.w - rsq_lo[v]);
        const float R = fexp2(-eta_a2 * dq * dq);
        RF[v] = R * d4.x;
        RT[v] = R * fmaf(h2, dq, d4.w);
      }
    }
  };
  // few triplets with several species: 4-lane block b walks the triplets of
  // species-pair block b (as in the forward pass)
  const int nblk = S * (S + 1) / 2;
  if (WPA == 1 && nblk > 1 && nblk <= 16 && nb.n * (nb.n - 1) / 2 <= kFuseTriplets) {
    int pa = 0, rem = blk < nblk ? blk : 0;
    while (rem >= S - pa) {
      rem -= S - pa;
      ++pa;
    }
    const int pb = pa + rem;
    const int na = nb.seg[pa + 1] - nb.seg[pa], nbb = nb.seg[pb + 1] - nb.seg[pb];
    const int Tb = blk < nblk ? (pa == pb ? na * (na - 1) / 2 : na * nbb) : 0;
    int Tmax = Tb;
    for (int o = 32; o >= 1; o >>= 1) Tmax = max(Tmax, __shfl_xor(Tmax, o));
    const int m = pa == pb ? na : nbb;
    const float inv_m = m > 0 ? 1.0f / (float)m : 0.f;
    floatx4 acc[NP][NQ];
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < Tmax; ++t) {
      float4 geo = make_float4(1.f, 0.f, 0.f, 0.f), dot = make_float4(0.f, 0.f, 0.f, 0.f);
      float g2 = 0.f;  // all zero past the block's triplets: such terms add nothing
      if (t < Tb) {
        int q, r, j, k;
        divmod_small(t, m, inv_m, q, r);
        if (pa == pb) {
          int kk = r + q + 1;
          if (kk >= na) kk -= na;
          j = nb.seg[pa] + r;
          k = nb.seg[pa] + kk;
        } else {
          j = nb.seg[pa] + q;
          k = nb.seg[pb] + r;
        }
        trip_terms(j, k, geo, dot, g2);
      }
      float A[NP], Ad[NP], RF[NQ], RT[NQ];
      lane_factors(geo, dot, g2, A, Ad, RF, RT);
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) {
          acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ad[u], RF[v], acc[u][v], 0, 0, 0);
          acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[u], RT[v], acc[u][v], 0, 0, 0);
        }
    }
    if (blk < nblk) {
      float* out = Ui + ang0 + blk * NB;
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[(4 * v + li) * NT + 4 * u + r] = acc[u][v][r];
    }
    return;
  }
  for (int a = 0; a < S; ++a) {
    for (int b = a; b < S; ++b) {
      const int na = nb.seg[a + 1] - nb.seg[a], nbb = nb.seg[b + 1] - nb.seg[b];
      const int T = (a == b) ? na * (na - 1) / 2 : na * nbb;
      floatx4 acc[NP][NQ];
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
      const int m = (a == b) ? na : nbb;
      const float inv_m = m > 0 ? 1.0f / (float)m : 0.f;
      for (int t0 = wv * kWave; t0 < T; t0 += kWave * WPA) {
        const int t = t0 + lane;
        float4 geo = make_float4(1.f, 0.f, 0.f, 0.f), dot = make_float4(0.f, 0.f, 0.f, 0.f);
        float g2 = 0.f;  // all zero past the block's triplets: such rows add nothing
        if (t < T) {
          int q, r, j, k;
          divmod_small(t, m, inv_m, q, r);
          if (a == b) {
            int kk = r + q + 1;
            if (kk >= na) kk -= na;
            j = nb.seg[a] + r;
            k = nb.seg[a] + kk;
          } else {
            j = nb.seg[a] + q;
            k = nb.seg[b] + r;
          }
          trip_terms(j, k, geo, dot, g2);
        }
        tgeo[wv][lane] = geo;
        tdot[wv][lane] = dot;
        tg2[wv][lane] = g2;
        wave_lds_sync();
        const int ng = (min(T - t0, kWave) + 15) >> 4;
        for (int gi = 0; gi < ng; ++gi) {
          const float4 q4 = tgeo[wv][16 * gi + blk];
          const float4 d4 = tdot[wv][16 * gi + blk];
          const float h2 = tg2[wv][16 * gi + blk];
          float A[NP], Ad[NP], RF[NQ], RT[NQ];
          lane_factors(q4, d4, h2, A, Ad, RF, RT);
#pragma unroll
          for (int u = 0; u < NP; ++u)
#pragma unroll
            for (int v = 0; v < NQ; ++v) {
              acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ad[u], RF[v], acc[u][v], 0, 0, 0);
              acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[u], RT[v], acc[u][v], 0, 0, 0);
            }
        }
        wave_lds_sync();
      }
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float y = acc[u][v][r];
            y += __shfl_xor(y, 4);
            y += __shfl_xor(y, 8);
            y += __shfl_xor(y, 16);
            y += __shfl_xor(y, 32);
            acc[u][v][r] = y;
          }
      float* out = Ui + ang0 + pair_block(S, a, b) * NB;
      if (lane < 4) {
#pragma unroll
        for (int u = 0; u < NP; ++u)
#pragma unroll
          for (int v = 0; v < NQ; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int bin = (4 * v + lane) * NT + 4 * u + r;
              if constexpr (WPA == 1) out[bin] = acc[u][v][r];
              else xch[wv * NB + bin] = acc[u][v][r];
            }
      }
      if constexpr (WPA > 1) {
        __syncthreads();
        for (int x = tid; x < NB; x += 64 * WPA) {
          float v = 0.f;
          for (int w = 0; w < WPA; ++w) v += xch[w * NB + x];
          out[x] = v;
        }
        __syncthreads();
      }
    }
  }
}

// Per-pair energy gradients dE_i/dd_e (float4 per entry, w unused) from
// lambda_i = dE_i/dG_i.
// Floats of the adjoint's radial lambda in LDS: S n_rad rounded up to a
// multiple of 4, so that the angular blocks after it are float4-aligned.
__host__ __device__ constexpr int adj_lam_radial(int S, int n_rad) { return (S * n_rad + 3) / 4 * 4; }

template <int NT, int NRA, bool ONE_SPECIES, int WPA, int ZC>
__device__ __forceinline__ void desc_adj_atom(int64_t i, const nn_system& sys, const int64_t* __restrict__ offsets,
                                              const int32_t* __restrict__ nbr, const int8_t* __restrict__ shift,
                                              const DescConst& P, const float* __restrict__ lambda,
                                              float4* __restrict__ pg, int64_t* meta) {
  constexpr int NB = NT * NRA;
  constexpr int NBP = NB + 4;  // padded block stride in LDS (bank spread)
  __shared__ AtomNb nb;
  __shared__ float4 gxyz[WPA][kMaxNb];  // one accumulator set per wave: dE/dd of each slot (x, y, z, -)
  // [S * n_rad] radial lambda, padded to a multiple of 4 floats, then the
  // angular blocks (16-byte aligned, read as float4)
  extern __shared__ float4 dyn_lds4[];
  float* lam_r = reinterpret_cast<float*>(dyn_lds4);
  float* lam_a = lam_r + adj_lam_radial(P.S, P.n_rad);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t e0 = offsets[i];
  // this atom's lambda is requested before the neighbor staging (whose
  // loads it then overlaps) and put into LDS after it
  const float* lam = lambda + i * (int64_t)P.D;
  constexpr int kLamPre = 8;
  float lpre[kLamPre];
#pragma unroll
  for (int q = 0; q < kLamPre; ++q) {
    const int d = tid + q * 64 * WPA;
    lpre[q] = d < P.D ? lam[d] : 0.f;
  }
  stage_neighbors(nb, i, sys, offsets, nbr, shift, P, meta, pg);
  if (nb.bad) {
    for (int64_t e = e0 + tid; e < offsets[i + 1]; e += 64 * WPA) pg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const int S = P.S;
  const int n = nb.n;
  const int ang0 = P.n_rad * S;
  auto put_lam = [&](int d, float x) {
    if (d < ang0) {
      lam_r[d] = x;
    } else {
      const int da = d - ang0;
      lam_a[(da / NB) * NBP + da % NB] = x;
    }
  };
#pragma unroll
  for (int q = 0; q < kLamPre; ++q) {
    const int d = tid + q * 64 * WPA;
    if (d < P.D) put_lam(d, lpre[q]);
  }
  for (int d = tid + kLamPre * 64 * WPA; d < P.D; d += 64 * WPA) put_lam(d, lam[d]);
  for (int t = lane; t < n; t += kWave) gxyz[wv][t] = make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  const float eta_r2 = P.eta_rad * 1.4426950408889634f;
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  // radial: lane <-> neighbor (waves take alternate chunks); dE/dd = (dE/dr) d/r
  for (int t0 = wv * kWave; t0 < n; t0 += kWave * WPA) {
    const int t = t0 + lane;
    if (t < n) {
      const float4 u = nb.d[t], fu = nb.f[t];
      const float* lr = lam_r + nb_species(fu) * P.n_rad;
      float gr = 0.f;
      for (int k = 0; k < P.n_rad; ++k) {
        const float dr = (u.w - P.rs_rad[k]) + (fu.z - P.rs_rad_lo[k]);
        const float g = fexp2(-eta_r2 * dr * dr);
        gr = fmaf(lr[k] * g, fmaf(-2.0f * P.eta_rad * dr, fu.x, fu.y), gr);
      }
      float4 a = gxyz[wv][t];
      a.x += gr * u.x;
      a.y += gr * u.y;
      a.z += gr * u.z;
      gxyz[wv][t] = a;
    }
  }
  const int zeta1 = P.zeta - 1;
  const float zf = (float)P.zeta;
  const float sq_eta_a2 = sqrtf(eta_a2);
  float rs_sc[NRA];
#pragma unroll
  for (int q = 0; q < NRA; ++q) rs_sc[q] = P.rs_ang[q] * sq_eta_a2;
  // angular: the unordered pairs {j, (j + s) mod n} for s = 1 .. n/2 (for
  // even n the step n/2 only for j < n/2), numbered t = (s - 1) n + j and
  // taken 64 at a time (wave w: chunks w, w + WPA, ...), so every lane has a
  // triplet whatever n is.  A chunk spans a few steps; the gradients are
  // added to the per-neighbor LDS slots one step at a time, and within one
  // step the lanes' j are distinct and so are their k = j + s: no two lanes
  // of an add share a slot, and the order of all adds is fixed.
  const int T = n * (n - 1) / 2;
  const float inv_n = n > 0 ? 1.0f / (float)n : 0.f;
  for (int t0 = wv * kWave; t0 < T; t0 += kWave * WPA) {
    const bool take = t0 + lane < T;
    int q, j;
    divmod_small(t0 + lane, n, inv_n, q, j);
    const int sj_step = q + 1;
    int k = j + sj_step;
    if (k >= n) k -= n;
    float gjx = 0.f, gjy = 0.f, gjz = 0.f, gkx = 0.f, gky = 0.f, gkz = 0.f;
    if (take && ZC == kZcBP) {
      // standard BP: E_t = F3 sum_q R_q T_q with R_q = exp(-eta_q s2),
      // T_q = sum_p lambda_qp A_p, A_p = pref_p (1 + lam_p cos)^zeta_p
      const float4 u = nb.d[j], fu = nb.f[j];
      const float4 v = nb.d[k], fv = nb.f[k];
      const float* La = lam_a;
      if (!ONE_SPECIES) La = lam_a + pair_block(S, nb_species(fu), nb_species(fv)) * NBP;
      const BpGeom g = bp_geom<true>(u, v, P);
      float P1[NT], A[NT], R[NRA];
#pragma unroll
      for (int p = 0; p < NT; ++p) {
        const float base = fmaf(P.bp_lam[p], g.c, 1.0f);
        P1[p] = ipow_uniform(base, P.bp_zeta[p] - 1);
        A[p] = P.bp_pref[p] * P1[p] * base;
      }
#pragma unroll
      for (int q = 0; q < NRA; ++q) R[q] = fexp2(-P.bp_eta[q] * 1.4426950408889634f * g.s2);
      float Tq[NRA], U[NT];
#pragma unroll
      for (int p = 0; p < NT; ++p) U[p] = 0.f;
#pragma unroll
      for (int q = 0; q < NRA; ++q) {
        float tq = 0.f;
#pragma unroll
        for (int p = 0; p < NT; ++p) {
          const float l = La[q * NT + p];
          tq = fmaf(l, A[p], tq);
          U[p] = fmaf(l, R[q], U[p]);
        }
        Tq[q] = tq;
      }
      float sRT = 0.f, sERT = 0.f;
#pragma unroll
      for (int q = 0; q < NRA; ++q) {
        sRT = fmaf(Tq[q], R[q], sRT);
        sERT = fmaf(Tq[q] * R[q], P.bp_eta[q], sERT);
      }
      float dEdc = 0.f;
#pragma unroll
      for (int p = 0; p < NT; ++p) dEdc = fmaf(U[p] * P1[p], P.bp_pref[p] * (float)P.bp_zeta[p] * P.bp_lam[p], dEdc);
      const float F3 = fu.x * fv.x * g.fw;
      dEdc *= F3;
      const float two_ds2 = -2.0f * F3 * sERT;  // 2 dE/ds2
      // d cos / d d_j = (v^ - cos u^) / r_j;  d s2 / d d_j = 2 d_j - 2 w, d s2 / d d_k = 2 d_k + 2 w;
      // d F3 / d d_j = fc'_j u^ fc_k fc_w - fc_j fc_k fc'_w w^, d F3 / d d_k = fc_j fc'_k v^ fc_w + fc_j fc_k fc'_w w^
      const float cu = dEdc * nb.ir[j], cv = dEdc * nb.ir[k];
      const float fj = sRT * fu.y * fv.x * g.fw, fk = sRT * fu.x * fv.y * g.fw;
      const float fwv = g.rw > 0.f ? sRT * fu.x * fv.x * g.dfw * frcp(g.rw) : 0.f;
      gjx = cu * (v.x - g.c * u.x) + two_ds2 * fmaf(u.w, u.x, -g.wx) + fj * u.x - fwv * g.wx;
      gjy = cu * (v.y - g.c * u.y) + two_ds2 * fmaf(u.w, u.y, -g.wy) + fj * u.y - fwv * g.wy;
      gjz = cu * (v.z - g.c * u.z) + two_ds2 * fmaf(u.w, u.z, -g.wz) + fj * u.z - fwv * g.wz;
      gkx = cv * (u.x - g.c * v.x) + two_ds2 * fmaf(v.w, v.x, g.wx) + fk * v.x + fwv * g.wx;
      gky = cv * (u.y - g.c * v.y) + two_ds2 * fmaf(v.w, v.y, g.wy) + fk * v.y + fwv * g.wy;
      gkz = cv * (u.z - g.c * v.z) + two_ds2 * fmaf(v.w, v.z, g.wz) + fk * v.z + fwv * g.wz;
    } else if (take) {
      const float4 u = nb.d[j], fu = nb.f[j];
      const float4 v = nb.d[k], fv = nb.f[k];
      const float* La = lam_a;
      if (!ONE_SPECIES) La = lam_a + pair_block(S, nb_species(fu), nb_species(fv)) * NBP;
      const float4* La4 = reinterpret_cast<const float4*>(La);  // NBP and the block base are multiples of 4
      const float iru = nb.ir[j], irv = nb.ir[k];
      const TripGeom g = triplet_geom<false>(u, fu, v, fv, P.eps_ang);
      const float c = g.c;
      const float F2 = 2.0f * fu.x * fv.x;
      float x[NT], P1[NT], A[NT];
#pragma unroll
      for (int p = 0; p < NT; ++p) x[p] = fmaf(c, P.x_a[p], fmaf(g.ssm, P.x_b[p], P.x_c));
      ipow_sel<(ZC > 0 ? ZC - 1 : 0), NT>(x, zeta1, P1);
#pragma unroll
      for (int p = 0; p < NT; ++p) A[p] = P1[p] * x[p];
      // R_q = 2^(-dq_q^2) with dq_q = sqrt(eta log2 e) (rbar - Rs'_q); the
      // hi/lo split of rbar and Rs' that the forward pass keeps for the
      // descriptor values is below what the gradient needs
      float R[NRA], dq[NRA];
      const float rb = g.rbar * sq_eta_a2;
#pragma unroll
      for (int q = 0; q < NRA; ++q) {
        dq[q] = rb - rs_sc[q];
        R[q] = fexp2(-dq[q] * dq[q]);
      }
      float Tq[NRA], U[NT];
#pragma unroll
      for (int p = 0; p < NT; ++p) U[p] = 0.f;
#pragma unroll
      for (int q = 0; q < NRA; ++q) {
        float tq = 0.f;
#pragma unroll
        for (int p4 = 0; p4 < NT / 4; ++p4) {
          const float4 l4 = La4[q * (NT / 4) + p4];  // LDS (a broadcast with one species)
          const float l[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int p = 4 * p4 + c;
            tq = fmaf(l[c], A[p], tq);
            U[p] = fmaf(l[c], R[q], U[p]);
          }
        }
        Tq[q] = tq;
      }
      // E_t = F2 sum_q R_q T_q, T_q = sum_p lambda_qp A_p
      float dEdF2 = 0.f, dEdravg = 0.f;
#pragma unroll
      for (int q = 0; q < NRA; ++q) {
        dEdF2 = fmaf(Tq[q], R[q], dEdF2);
        dEdravg = fmaf(Tq[q] * R[q], dq[q], dEdravg);
      }
      dEdravg *= -2.0f * P.eta_ang / sq_eta_a2 * F2;
      float dEdc = 0.f, dEdssm = 0.f;
#pragma unroll
      for (int p = 0; p < NT; ++p) {
        const float gp = U[p] * P1[p];
        dEdc = fmaf(gp, P.x_a[p], dEdc);
        dEdssm = fmaf(gp, P.x_b[p], dEdssm);
      }
      dEdc *= zf * F2;
      dEdssm *= zf * F2;
      // sin^2 = 1 - cos^2, so d ssm / d cos = -cos / ssm
      const float coef = dEdc - dEdssm * c * frcp(g.ssm);
      const float dEdru = 0.5f * dEdravg + dEdF2 * 2.0f * fu.y * fv.x;
      const float dEdrv = 0.5f * dEdravg + dEdF2 * 2.0f * fu.x * fv.y;
      // d cos / d d_u = (v^ - cos u^) / r_u
      const float cu = coef * iru, cv = coef * irv;
      gjx = cu * (v.x - c * u.x) + dEdru * u.x;
      gjy = cu * (v.y - c * u.y) + dEdru * u.y;
      gjz = cu * (v.z - c * u.z) + dEdru * u.z;
      gkx = cv * (u.x - c * v.x) + dEdrv * v.x;
      gky = cv * (u.y - c * v.y) + dEdrv * v.y;
      gkz = cv * (u.z - c * v.z) + dEdrv * v.z;
    }
    // steps present in this chunk: from lane 0's to the last taking lane's
    const int last = min(kWave - 1, T - 1 - t0);
    const int s_lo = __shfl(sj_step, 0), s_hi = __shfl(sj_step, last);
    for (int ss = s_lo; ss <= s_hi; ++ss) {
      if (take && sj_step == ss) {  // plain read-add-write: no two lanes share a slot here
        float4 a = gxyz[wv][k];
        a.x += gkx;
        a.y += gky;
        a.z += gkz;
        gxyz[wv][k] = a;
      }
      wave_lds_order();
      if (take && sj_step == ss) {
        float4 a = gxyz[wv][j];
        a.x += gjx;
        a.y += gjy;
        a.z += gjz;
        gxyz[wv][j] = a;
      }
      wave_lds_order();
    }
  }
  __syncthreads();
  for (int t = tid; t < n; t += 64 * WPA) {
    float x = 0.f, y = 0.f, z = 0.f;
#pragma unroll
    for (int w = 0; w < WPA; ++w) {
      const float4 a = gxyz[w][t];
      x += a.x;
      y += a.y;
      z += a.z;
    }
    pg[e0 + nb_entry(nb.f[t])] = make_float4(x, y, z, 0.f);
  }
}

template <int NT, int NRA, bool ONE_SPECIES, int WPA, int ZC>
__global__ void __launch_bounds__(64 * WPA) k_desc_adj(nn_system sys, const int64_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ nbr,
                                                       const int8_t* __restrict__ shift, DescConst P,
                                                       const float* __restrict__ lambda, float4* __restrict__ pg,
                                                       int64_t* meta, const int32_t* __restrict__ order) {
  if (meta[kMetaValid] != 1) return;  // no valid list: the gather writes zero forces
  const int64_t i = atom_of_block(order, sys.n_atoms, true);
  if (i < 0) return;
  desc_adj_atom<NT, NRA, ONE_SPECIES, WPA, ZC>(i, sys, offsets, nbr, shift, P, lambda, pg, meta);
}

// The atoms a packed adjoint leaves out (rows over kPackNb entries), as in
// k_desc_fwd_long.
template <int NT, int NRA, bool ONE_SPECIES, int ZC>
__global__ void __launch_bounds__(64) k_desc_adj_long(nn_system sys, const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ nbr,
                                                      const int8_t* __restrict__ shift, DescConst P,
                                                      const float* __restrict__ lambda, float4* __restrict__ pg,
                                                      int64_t* meta, const int32_t* __restrict__ order) {
  if (meta[kMetaValid] != 1) return;
  const int64_t slot = (int64_t)blockIdx.x * kWave + threadIdx.x;
  const bool in = slot < sys.n_atoms;
  const int64_t i = !in ? -1 : order ? (int64_t)order[slot] : slot;
  uint64_t m = __ballot(in && offsets[i + 1] - offsets[i] > kPackNb);
  while (m) {
    const int b = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    desc_adj_atom<NT, NRA, ONE_SPECIES, 1, ZC>(__shfl(i, b), sys, offsets, nbr, shift, P, lambda, pg, meta);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Packed passes for short rows (small molecules): kPackAtoms atoms per
// one-wave block, kPackLanes lanes per atom while staging and in the radial
// terms; the triplets of all the wave's atoms are spread over all 64 lanes.
// ---------------------------------------------------------------------------

struct PackNb {
  float4 d[kPackAtoms * kPackSlots];  // as AtomNb; atom g's neighbors at g kPackSlots + [0, n_g)
  float4 f[kPackAtoms * kPackSlots];
  int seg[kPackAtoms][NN_MAX_SPECIES + 1];
  int64_t atom[kPackAtoms];  // the atom of each group, -1 if the group has none to pack
};

// The atom of lane group g of a packed launch: atom kPackAtoms w + g, w the
// wave's block of atoms, taken XCD by XCD as in atom_of_block (block b ->
// w = (b mod 8) per + b / 8), or -1.  The atoms a wave packs together set
// the order of its sums, so they follow the atom index, not the list's bin
// order (whose order within a bin is that of the binning atomics).
__device__ __forceinline__ int64_t packed_atom(int64_t N, int g) {
  const int64_t w = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int64_t i = w * kPackAtoms + g;
  return i < N ? i : -1;
}

static inline unsigned packed_grid(int64_t N) {
  const int64_t w = (N + kPackAtoms - 1) / kPackAtoms;
  return (unsigned)((w + 7) / 8 * 8);
}

// struct_of_atom for every 16-lane group at once (its own atom i; groups
// with has = false get 0): each round a group's lanes probe 16 evenly
// spaced positions of its remaining range.
__device__ __forceinline__ int struct_of_atom16(const int64_t* atom_ptr, int32_t B, int64_t i, bool has) {
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  int lo = 0, hi = has ? B : 1;
  while (__any(hi - lo > 1)) {
    const bool act = hi - lo > 1;
    const int step = (hi - lo + 15) / 16;
    const int p = lo + l * step;
    const uint64_t le = __ballot(act && p < hi && atom_ptr[p] <= i);
    if (act) {
      lo += (__popcll((le >> (16 * g)) & 0xffffull) - 1) * step;
      hi = min(hi, lo + step);
    }
  }
  return lo;
}

// Group g's lanes stage atom i's row (take: it has at most kPackNb entries)
// into slots g kPackSlots + [0, n), sorted by species (stable, so in entry
// order within a species, as stage_neighbors), with nb.seg[g].  With
// ir_in_f (the adjoint) the record's third float holds 1/r instead of the
// low part of r: the gradient passes do not need that part, and the
// separate 1/r array would cost the one-wave block LDS it needs for
// occupancy.  Entries at r >= rc get a zero pair gradient if pg != nullptr.
// Groups that do not take their atom stage nothing (n = 0).
__device__ void stage_packed(PackNb& nb, bool ir_in_f, int64_t i, bool take, const nn_system& sys,
                             const int64_t* __restrict__ offsets, const int32_t* __restrict__ nbr,
                             const int8_t* __restrict__ shift, const DescConst& P, int64_t* meta,
                             float4* __restrict__ pg) {
  constexpr int R = kPackNb / kPackLanes;
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  if (l == 0) nb.atom[g] = take ? i : -1;
  double xi[3] = {0.0, 0.0, 0.0};
  int64_t e0 = 0, e1 = 0;
  if (take) {
    xi[0] = sys.pos[3 * i];
    xi[1] = sys.pos[3 * i + 1];
    xi[2] = sys.pos[3 * i + 2];
    e0 = offsets[i];
    e1 = offsets[i + 1];
  }
  const double rc2 = P.rc64 * P.rc64;
  const int S = P.S;
  const char4* sh4 = reinterpret_cast<const char4*>(shift);
  int32_t jr[R];
  char4 s4r[R];
  bool shifted = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t e = e0 + r * kPackLanes + l;
    jr[r] = 0;
    s4r[r] = make_char4(0, 0, 0, 0);
    if (e < e1) {
      jr[r] = nbr[e];
      s4r[r] = sh4[e];
      shifted = shifted || (s4r[r].x | s4r[r].y | s4r[r].z) != 0;
    }
  }
  // the structure's cell only for rows with image shifts (with all shifts
  // zero displacement64 gives x_j - x_i exactly whatever the cell)
  const bool need = take && ((__ballot(shifted) >> (16 * g)) & 0xffffull) != 0;
  const int c = struct_of_atom16(sys.atom_ptr, sys.n_structs, i, need);
  double h[9];
  for (int k = 0; k < 9; ++k) h[k] = need ? sys.cell[9 * (int64_t)c + k] : 0.0;
  bool valid[R];
  int sp[R];
  double d[R][3], r2[R];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t e = e0 + r * kPackLanes + l;
    valid[r] = false;
    sp[r] = 0;
    d[r][0] = d[r][1] = d[r][2] = 0.0;
    r2[r] = 0.0;
    if (e < e1) {
      const int32_t j = jr[r];
      const char4 s4 = s4r[r];
      displacement64(xi, sys.pos + 3 * (int64_t)j, h, s4.x, s4.y, s4.z, d[r]);
      r2[r] = norm2_64(d[r]);
      valid[r] = r2[r] < rc2;
      sp[r] = sys.species[j];
      if (sp[r] < 0 || sp[r] >= S) {
        bad = bad || valid[r];
        valid[r] = false;
      }
      if (!valid[r] && pg) pg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  if (__any(bad) && lane == 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrSpecies);
  const uint32_t lt = (1u << l) - 1u;
  int slot[R] = {};
  int total = 0;
  for (int s2 = 0; s2 < S; ++s2) {
    if (l == 0) nb.seg[g][s2] = total;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t m = (uint32_t)(__ballot(valid[r] && sp[r] == s2) >> (16 * g)) & 0xffffu;
      if (valid[r] && sp[r] == s2) slot[r] = total + __popc(m & lt);
      total += __popc(m);
    }
  }
  if (l == 0) nb.seg[g][S] = total;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (valid[r]) {
      float4 dd, ff;
      float irf;
      pair_record(d[r], r2[r], r * kPackLanes + l, sp[r], P, dd, ff, irf);
      const int t = g * kPackSlots + slot[r];
      nb.d[t] = dd;
      nb.f[t] = ir_in_f ? make_float4(ff.x, ff.y, irf, ff.w) : ff;
    }
  wave_lds_sync();
}

// x broadcast from lane R of each group of four lanes (DPP quad_perm).
template <int R>
__device__ __forceinline__ int quad_bcast(int x) {
  return __builtin_amdgcn_mov_dpp(x, R * 0x55, 0xf, 0xf, false);
}
template <int R>
__device__ __forceinline__ float quad_bcast(float x) {
  return __int_as_float(quad_bcast<R>(__float_as_int(x)));
}

// Dynamic LDS of k_desc_fwd_packed: the segment table (int4 [nseg + 1],
// float [nseg]; int4 [nseg] with each segment's start and place in G).  The
// heads and tails of split segments stay in registers.
static inline size_t packed_fwd_lds(int S, int NB) {
  const int nseg = kPackAtoms * S * (S + 1) / 2;
  (void)NB;
  return sizeof(int4) * (2 * nseg + 1) + sizeof(float) * ((nseg + 3) / 4 * 4);
}

// Descriptor rows of kPackAtoms atoms per one-wave block, for atoms whose
// rows have at most kPackNb entries (k_desc_fwd_long takes the others).
// The radial bins as in k_desc_fwd with one wave, 16 lanes per atom.  The
// angular bins: the wave's triplets are numbered species-pair block after
// block, atom after atom (one segment per atom and block), and the 16 4-lane
// MFMA blocks take equal contiguous ranges of that numbering, so no block
// idles while another walks a long segment.  Each round every lane forms one
// triplet's geometry, then the four lanes of a block take their four
// triplets in turn (broadcast within the quad), each lane supplying its
// angle and radius factors to the 4x4x1 MFMA as in k_desc_fwd.  When a block
// passes the end of a segment its accumulators hold the segment's last
// piece: a segment that lies inside the block's range goes straight to G; a
// piece that began in an earlier range (the block's head) and the piece still
// open at the end of its range (its tail) stay in the block's registers.  A
// segment split over ranges is then written by the block that ends it, as the
// tails of the ranges before in range order plus its head, so every sum has a
// fixed order.
template <int NT, int NRA, int ZC>
__global__ void __launch_bounds__(64) k_desc_fwd_packed(nn_system sys, const int64_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ nbr,
                                                        const int8_t* __restrict__ shift, DescConst P,
                                                        float* __restrict__ G, int64_t* meta) {
  static_assert(ZC != kZcBP, "the packed forward takes the mBP term");
  constexpr int NB = NT * NRA, NP = NT / 4, NQ = NRA / 4;
  __shared__ PackNb nb;
  __shared__ int hseg[16], tseg[16];
  extern __shared__ float4 pk_lds[];
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  const bool list_ok = meta[kMetaValid] == 1;
  const int64_t i = packed_atom(sys.n_atoms, g);
  const int D = P.D;
  if (!list_ok) {  // no valid list: never read its entries
    if (i >= 0)
      for (int d = l; d < D; d += kPackLanes) G[i * D + d] = 0.f;
    return;
  }
  const bool take = i >= 0 && offsets[i + 1] - offsets[i] <= kPackNb;
  if (!__any(take)) return;
  if (lane < 16) hseg[lane] = tseg[lane] = -1;
  stage_packed(nb, false, i, take, sys, offsets, nbr, shift, P, meta, nullptr);
  const int S = P.S, nblk = S * (S + 1) / 2, nseg = kPackAtoms * nblk, ang0 = P.n_rad * S;
  // radial bins: lane l of group g owns bins l, l + 16, ... of its atom
  {
    float* Gi = G + (take ? i : 0) * (int64_t)D;
    const float eta_r2 = P.eta_rad * 1.4426950408889634f;
    for (int k0 = 0; k0 < P.n_rad; k0 += kPackLanes) {
      const int k = k0 + l;
      const bool kin = k < P.n_rad;
      const float rs = kin ? P.rs_rad[k] : 0.f, rs_lo = kin ? P.rs_rad_lo[k] : 0.f;
      for (int s = 0; s < S; ++s) {
        float acc = 0.f;
        const int t1 = g * kPackSlots + nb.seg[g][s + 1];
        for (int t = g * kPackSlots + nb.seg[g][s]; t < t1; ++t) {
          const float dr = (nb.d[t].w - rs) + (nb.f[t].z - rs_lo);
          acc = fmaf(fexp2(-eta_r2 * dr * dr), nb.f[t].x, acc);
        }
        if (take && kin) Gi[s * P.n_rad + k] = acc;
      }
    }
  }
  // segment table: segment s = a nblk + (layout index of species pair
  // (pa, pb)) holds its first triplet in the wave's numbering, the slots of
  // its j and k runs, m | same << 16 and 1/m; empty segments are written as
  // zeros here
  int4* stab = reinterpret_cast<int4*>(pk_lds);
  int4* sdst = stab + nseg + 1;  // start, offset of the segment's bins in G (lo, hi)
  float* sinv = reinterpret_cast<float*>(sdst + nseg);
  const bool vec4 = (ang0 & 3) == 0;  // then D is a multiple of 4 too: 16-byte bin stores
  int carry = 0;
  for (int s0 = 0; s0 < nseg; s0 += kWave) {
    const int s = s0 + lane;
    int cnt = 0;
    if (s < nseg) {
      const int a = s / nblk, pbi = s - a * nblk;
      int pa = 0, rem = pbi;
      while (rem >= S - pa) {
        rem -= S - pa;
        ++pa;
      }
      const int pb = pa + rem;
      const int ja = nb.seg[a][pa], na = nb.seg[a][pa + 1] - ja;
      const int kb = nb.seg[a][pb], nbb = nb.seg[a][pb + 1] - kb;
      const bool same = pa == pb;
      const int m = same ? na : nbb;
      cnt = same ? na * (na - 1) / 2 : na * nbb;
      stab[s] = make_int4(0, a * kPackSlots + ja, a * kPackSlots + kb, m | (same ? 1 << 16 : 0));
      sinv[s] = m > 0 ? 1.0f / (float)m : 0.f;
      const int64_t ia = nb.atom[a];
      const int64_t go = (ia >= 0 ? ia : 0) * (int64_t)D + ang0 + pbi * NB;
      sdst[s] = make_int4(0, (int)(uint32_t)go, (int)(go >> 32), 0);
      if (cnt == 0 && ia >= 0) {
        float* o = G + ia * (int64_t)D + ang0 + pbi * NB;
        if (vec4) {
          for (int x = 0; x < NB; x += 4) *reinterpret_cast<float4*>(o + x) = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          for (int x = 0; x < NB; ++x) o[x] = 0.f;
        }
      }
    }
    int x = cnt;  // inclusive prefix sum over the wave
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (s < nseg) stab[s].x = sdst[s].x = carry + x - cnt;
    carry += __shfl(x, kWave - 1);
  }
  if (lane == 0) stab[nseg] = make_int4(carry, 0, 0, 0);
  wave_lds_sync();
  const int Tw = carry;
  const int blk = lane >> 2, li = lane & 3;
  float xa[NP], xb[NP], rsq[NQ], rsq_lo[NQ];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    xa[u] = P.x_a[4 * u + li];
    xb[u] = P.x_b[4 * u + li];
  }
#pragma unroll
  for (int v = 0; v < NQ; ++v) {
    rsq[v] = P.rs_ang[4 * v + li];
    rsq_lo[v] = P.rs_ang_lo[4 * v + li];
  }
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  const int L4 = (Tw + 63) / 64;  // rounds: block blk takes triplets [4 L4 blk, 4 L4 (blk + 1))
  const int r_lo = 4 * L4 * blk, r_hi = min(r_lo + 4 * L4, Tw);
  floatx4 acc[NP][NQ];
#pragma unroll
  for (int u = 0; u < NP; ++u)
#pragma unroll
    for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
  int acc_seg = -1;
  int4 acc_dst = make_int4(0, 0, 0, 0);  // sdst of acc_seg, read when the block enters it
  // this block's head (the last piece of a segment begun in an earlier range)
  // and tail (the piece open at the end of its range)
  floatx4 hacc[NP][NQ], tacc[NP][NQ];
#pragma unroll
  for (int u = 0; u < NP; ++u)
#pragma unroll
    for (int v = 0; v < NQ; ++v) hacc[u][v] = tacc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
  // a segment's bins (this lane's: (4 v + li) NT + 4 u + r) into G at its sdst entry
  auto store_g = [&](const int4& sd, const floatx4 (&val)[NP][NQ]) {
    float* dst = G + (int64_t)(((uint64_t)(uint32_t)sd.z << 32) | (uint32_t)sd.y);
    if (vec4) {
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
          *reinterpret_cast<float4*>(dst + (4 * v + li) * NT + 4 * u) =
              make_float4(val[u][v][0], val[u][v][1], val[u][v][2], val[u][v][3]);
    } else {
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[(4 * v + li) * NT + 4 * u + r] = val[u][v][r];
    }
  };
  // this block's accumulators into G (a whole segment), its tail (open at
  // the end of the range) or its head
  auto flush = [&](bool open) {
    if (open) {
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) tacc[u][v] = acc[u][v];
      tseg[blk] = acc_seg;
      return;
    }
    if (acc_dst.x < r_lo) {
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) hacc[u][v] = acc[u][v];
      hseg[blk] = acc_seg;
      return;
    }
    store_g(acc_dst, acc);
  };
  // one triplet of this block, broadcast from quad lane R: flush on a new
  // segment, then the lane's factors into the MFMA
  auto substep = [&](auto rc, const float4& geo, float f2, int sg) {
    constexpr int R = decltype(rc)::value;
    const float4 q4 = make_float4(quad_bcast<R>(geo.x), quad_bcast<R>(geo.y), quad_bcast<R>(geo.z),
                                  quad_bcast<R>(geo.w));
    const float fr = quad_bcast<R>(f2);
    const int sr = quad_bcast<R>(sg);
    if (sr >= 0 && sr != acc_seg) {  // the same in the block's four lanes
      if (acc_seg >= 0) flush(false);
#pragma unroll
      for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int v = 0; v < NQ; ++v) acc[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc_seg = sr;
      acc_dst = sdst[sr];
    }
    float x[NP], A[NP], Rq[NQ];
#pragma unroll
    for (int u = 0; u < NP; ++u) x[u] = fmaf(q4.x, xa[u], fmaf(q4.y, xb[u], P.x_c));
    ipow_sel<(ZC > 0 ? ZC : 0), NP>(x, P.zeta, A);
#pragma unroll
    for (int v = 0; v < NQ; ++v) {
      const float dq = (q4.z - rsq[v]) + (q4.w - rsq_lo[v]);
      Rq[v] = fexp2(-eta_a2 * dq * dq) * fr;
    }
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int v = 0; v < NQ; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[u], Rq[v], acc[u][v], 0, 0, 0);
  };
  // the segment of triplet r_lo: the last one starting at or before it
  int cur = 0;
  if (r_lo < r_hi) {
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (stab[mid].x <= r_lo) lo = mid;
      else hi = mid;
    }
    cur = lo;
  }
  int4 ce = stab[cur];
  int cend = stab[cur + 1].x;
  float cinv = sinv[cur];
  for (int it = 0; it < L4; ++it) {
    const int idx = r_lo + 4 * it + li;
    float4 geo = make_float4(1.f, 0.f, 0.f, 0.f);
    float f2 = 0.f;  // past the range: F2 = 0 adds nothing
    int sg = -1;
    if (idx < r_hi) {
      while (idx >= cend) {
        ++cur;
        ce = stab[cur];
        cend = stab[cur + 1].x;
        cinv = sinv[cur];
      }
      const int m = ce.w & 0xffff;
      int q, r;
      divmod_small(idx - ce.x, m, cinv, q, r);
      int j, k;
      if (ce.w >> 16) {  // one species: the unordered pairs {r, r + q + 1 mod m}
        int kk = r + q + 1;
        if (kk >= m) kk -= m;
        j = ce.y + r;
        k = ce.y + kk;
      } else {
        j = ce.y + q;
        k = ce.z + r;
      }
      const float4 fu = nb.f[j], fv = nb.f[k];
      const TripGeom tg = triplet_geom(nb.d[j], fu, nb.d[k], fv, P.eps_ang);
      geo = make_float4(tg.c, tg.ssm, tg.rbar, tg.rbar_lo);
      f2 = 2.0f * fu.x * fv.x;
      sg = cur;
    }
    substep(std::integral_constant<int, 0>{}, geo, f2, sg);
    substep(std::integral_constant<int, 1>{}, geo, f2, sg);
    substep(std::integral_constant<int, 2>{}, geo, f2, sg);
    substep(std::integral_constant<int, 3>{}, geo, f2, sg);
  }
  if (acc_seg >= 0) flush(stab[acc_seg + 1].x > r_hi);
  wave_lds_sync();
  // segments split over ranges: the tails of the ranges before, in range
  // order, plus the head of the range that ends them, by that range's block.
  // A tail's bins sit in the same lane position of its block (lane 4 bb +
  // li holds the bins of lane li of block blk), so each lane fetches them
  // with a shuffle; the loop runs the same number of times in every lane.
  const int hs = hseg[blk];
  int b0 = blk;
  if (hs >= 0)
    while (b0 > 0 && tseg[b0 - 1] == hs) --b0;
  const int ntl = blk - b0;  // tails this block adds (0 without a head)
  floatx4 v[NP][NQ];
#pragma unroll
  for (int u = 0; u < NP; ++u)
#pragma unroll
    for (int w = 0; w < NQ; ++w) v[u][w] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; __any(it < ntl); ++it) {
    const bool add = it < ntl;
    const int src = 4 * (add ? b0 + it : blk) + li;
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int w = 0; w < NQ; ++w)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float t = __shfl(tacc[u][w][r], src);
          if (add) v[u][w][r] += t;
        }
  }
  if (hs >= 0) {
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
      for (int w = 0; w < NQ; ++w) v[u][w] += hacc[u][w];
    store_g(sdst[hs], v);
  }
}

// Dynamic LDS of k_desc_adj_packed: the lambda rows, each [radial S n_rad,
// padded to a multiple of 4][angular blocks][4 spare floats].  The spare
// floats move each row by four banks: a row of a multiple of 64 floats would
// start every group's row on one bank.  (Padding each pair block to NB + 4
// as well removed most of the remaining bank conflicts but cost a block per
// CU of occupancy, and the pass got slower; reading the radial part from
// global memory instead of LDS gained a block per CU and was slower too.)
__host__ __device__ inline int packed_lam_stride(int S, int n_rad, int NB) {
  return (S * n_rad + 3) / 4 * 4 + S * (S + 1) / 2 * NB + 4;
}

// Per-pair energy gradients for kPackAtoms atoms per one-wave block (rows
// of at most kPackNb entries; k_desc_adj_long takes the others).  Staging
// and the radial terms take 16 lanes per atom (lane <-> neighbor).  The
// triplets of the four atoms are numbered as in k_desc_adj, atom after
// atom, and taken 64 at a time, one per lane, with the same arithmetic.
// The gradients go to the per-neighbor LDS slots one step at a time, the
// step counted from the first step of the lane's atom in the chunk: within
// one such round every lane of an atom is at the same step (distinct j,
// distinct k), and atoms own disjoint slots, so no two lanes of an add
// share a slot and the order of all adds is fixed.
template <int NT, int NRA, bool ONE_SPECIES, int ZC>
__global__ void __launch_bounds__(64) k_desc_adj_packed(nn_system sys, const int64_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ nbr,
                                                        const int8_t* __restrict__ shift, DescConst P,
                                                        const float* __restrict__ lambda, float4* __restrict__ pg,
                                                        int64_t* meta) {
  static_assert(ZC != kZcBP, "the packed adjoint takes the mBP term");
  constexpr int NB = NT * NRA;
  constexpr int kLamPre4 = 4;  // float4 (or four values) of lambda per lane requested before the staging
  __shared__ PackNb nb;
  __shared__ float gx[kPackAtoms * kPackSlots], gy[kPackAtoms * kPackSlots], gz[kPackAtoms * kPackSlots];
  extern __shared__ float4 pk_lds[];
  if (meta[kMetaValid] != 1) return;  // no valid list: the gather writes zero forces
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  const int64_t i = packed_atom(sys.n_atoms, g);
  const bool take = i >= 0 && offsets[i + 1] - offsets[i] <= kPackNb;
  if (!__any(take)) return;
  const int S = P.S, D = P.D, ang0 = P.n_rad * S;
  const int Dp = packed_lam_stride(S, P.n_rad, NB), angp = (ang0 + 3) / 4 * 4;
  float* lam_s = reinterpret_cast<float*>(pk_lds);
  // this group's lambda row, requested before the staging; with S n_rad a
  // multiple of 4 it is copied to LDS as float4
  const bool vec4 = (ang0 & 3) == 0;
  const float* lam = lambda + (take ? i : 0) * (int64_t)D;
  const float4* lam4 = reinterpret_cast<const float4*>(lam);
  float4 lp4[kLamPre4];
#pragma unroll
  for (int q = 0; q < kLamPre4; ++q) {
    if (vec4) {
      const int d4 = l + q * kPackLanes;
      lp4[q] = (take && 4 * d4 < D) ? lam4[d4] : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      float c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int d = l + (4 * q + k) * kPackLanes;
        c[k] = (take && d < D) ? lam[d] : 0.f;
      }
      lp4[q] = make_float4(c[0], c[1], c[2], c[3]);
    }
  }
  stage_packed(nb, true, i, take, sys, offsets, nbr, shift, P, meta, pg);
  float* lrow = lam_s + g * Dp;
  if (take) {
    if (vec4) {  // then the LDS row is the row itself
      float4* lr4 = reinterpret_cast<float4*>(lrow);
#pragma unroll
      for (int q = 0; q < kLamPre4; ++q) {
        const int d4 = l + q * kPackLanes;
        if (4 * d4 < D) lr4[d4] = lp4[q];
      }
      for (int d4 = l + kLamPre4 * kPackLanes; 4 * d4 < D; d4 += kPackLanes) lr4[d4] = lam4[d4];
    } else {
      auto put_lam = [&](int d, float x) { lrow[d < ang0 ? d : d - ang0 + angp] = x; };
#pragma unroll
      for (int q = 0; q < kLamPre4; ++q) {
        const float c[4] = {lp4[q].x, lp4[q].y, lp4[q].z, lp4[q].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int d = l + (4 * q + k) * kPackLanes;
          if (d < D) put_lam(d, c[k]);
        }
      }
      for (int d = l + 4 * kLamPre4 * kPackLanes; d < D; d += kPackLanes) put_lam(d, lam[d]);
    }
  }
  wave_lds_sync();
  const int ng = nb.seg[g][S];
  // radial: lane <-> neighbor of its group's atom; dE/dd = (dE/dr) d/r
  const float eta_r2 = P.eta_rad * 1.4426950408889634f;
  for (int t = l; t < ng; t += kPackLanes) {
    const int ts = g * kPackSlots + t;
    const float4 u = nb.d[ts], fu = nb.f[ts];
    const float* lr = lrow + nb_species(fu) * P.n_rad;
    float gr = 0.f;
    for (int k = 0; k < P.n_rad; ++k) {
      const float dr = (u.w - P.rs_rad[k]) - P.rs_rad_lo[k];  // r hi only: fu.z holds 1/r here
      const float gk = fexp2(-eta_r2 * dr * dr);
      gr = fmaf(lr[k] * gk, fmaf(-2.0f * P.eta_rad * dr, fu.x, fu.y), gr);
    }
    gx[ts] = gr * u.x;
    gy[ts] = gr * u.y;
    gz[ts] = gr * u.z;
  }
  // the atoms' triplet counts and first triplets in the wave's numbering
  int na[kPackAtoms], ts0[kPackAtoms + 1];
  ts0[0] = 0;
#pragma unroll
  for (int a = 0; a < kPackAtoms; ++a) {
    na[a] = nb.seg[a][S];
    ts0[a + 1] = ts0[a] + na[a] * (na[a] - 1) / 2;
  }
  const int Tw = ts0[kPackAtoms];
  const int zeta1 = P.zeta - 1;
  const float zf = (float)P.zeta;
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  const float sq_eta_a2 = sqrtf(eta_a2);
  float rs_sc[NRA];
#pragma unroll
  for (int q = 0; q < NRA; ++q) rs_sc[q] = P.rs_ang[q] * sq_eta_a2;
  wave_lds_sync();  // the radial terms are in the slots before the first angular add
  for (int c0 = 0; c0 < Tw; c0 += kWave) {
    const int idx = c0 + lane;
    const bool tk = idx < Tw;
    const int a = (idx >= ts0[1]) + (idx >= ts0[2]) + (idx >= ts0[3]);
    int n = na[0], t0a = ts0[0];
#pragma unroll
    for (int b = 1; b < kPackAtoms; ++b)
      if (a == b) {
        n = na[b];
        t0a = ts0[b];
      }
    int q = 0, j = 0;
    if (tk) divmod_small(idx - t0a, n, 1.0f / (float)n, q, j);
    const int step = q + 1;
    int k = j + step;
    if (k >= n) k -= n;
    j += a * kPackSlots;
    k += a * kPackSlots;
    float gjx = 0.f, gjy = 0.f, gjz = 0.f, gkx = 0.f, gky = 0.f, gkz = 0.f;
    if (tk) {
      const float4 u = nb.d[j], fu = nb.f[j];
      const float4 v = nb.d[k], fv = nb.f[k];
      const float* La = lam_s + a * Dp + angp;
      if (!ONE_SPECIES) La += pair_block(S, nb_species(fu), nb_species(fv)) * NB;
      const float4* La4 = reinterpret_cast<const float4*>(La);
      const float iru = fu.z, irv = fv.z;  // 1/r (staged in place of the low part of r)
      const TripGeom tg = triplet_geom<false>(u, fu, v, fv, P.eps_ang);
      const float c = tg.c;
      const float F2 = 2.0f * fu.x * fv.x;
      float x[NT], P1[NT], A[NT];
#pragma unroll
      for (int p = 0; p < NT; ++p) x[p] = fmaf(c, P.x_a[p], fmaf(tg.ssm, P.x_b[p], P.x_c));
      ipow_sel<(ZC > 0 ? ZC - 1 : 0), NT>(x, zeta1, P1);
#pragma unroll
      for (int p = 0; p < NT; ++p) A[p] = P1[p] * x[p];
      float R[NRA], dq[NRA];
      const float rb = tg.rbar * sq_eta_a2;
#pragma unroll
      for (int qq = 0; qq < NRA; ++qq) {
        dq[qq] = rb - rs_sc[qq];
        R[qq] = fexp2(-dq[qq] * dq[qq]);
      }
      float Tq[NRA], U[NT];
#pragma unroll
      for (int p = 0; p < NT; ++p) U[p] = 0.f;
#pragma unroll
      for (int qq = 0; qq < NRA; ++qq) {
        float tq = 0.f;
#pragma unroll
        for (int p4 = 0; p4 < NT / 4; ++p4) {
          const float4 l4 = La4[(qq * NT) / 4 + p4];
          const float lv[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            tq = fmaf(lv[e], A[4 * p4 + e], tq);
            U[4 * p4 + e] = fmaf(lv[e], R[qq], U[4 * p4 + e]);
          }
        }
        Tq[qq] = tq;
      }
      float dEdF2 = 0.f, dEdravg = 0.f;
#pragma unroll
      for (int qq = 0; qq < NRA; ++qq) {
        dEdF2 = fmaf(Tq[qq], R[qq], dEdF2);
        dEdravg = fmaf(Tq[qq] * R[qq], dq[qq], dEdravg);
      }
      dEdravg *= -2.0f * P.eta_ang / sq_eta_a2 * F2;
      float dEdc = 0.f, dEdssm = 0.f;
#pragma unroll
      for (int p = 0; p < NT; ++p) {
        const float gp = U[p] * P1[p];
        dEdc = fmaf(gp, P.x_a[p], dEdc);
        dEdssm = fmaf(gp, P.x_b[p], dEdssm);
      }
      dEdc *= zf * F2;
      dEdssm *= zf * F2;
      const float coef = dEdc - dEdssm * c * frcp(tg.ssm);
      const float dEdru = 0.5f * dEdravg + dEdF2 * 2.0f * fu.y * fv.x;
      const float dEdrv = 0.5f * dEdravg + dEdF2 * 2.0f * fu.x * fv.y;
      const float cu = coef * iru, cv = coef * irv;
      gjx = cu * (v.x - c * u.x) + dEdru * u.x;
      gjy = cu * (v.y - c * u.y) + dEdru * u.y;
      gjz = cu * (v.z - c * u.z) + dEdru * u.z;
      gkx = cv * (u.x - c * v.x) + dEdrv * v.x;
      gky = cv * (u.y - c * v.y) + dEdrv * v.y;
      gkz = cv * (u.z - c * v.z) + dEdrv * v.z;
    }
    // rounds of equal step within each atom: lane fl is the atom's first in this chunk
    const int fl = max(t0a - c0, 0);
    const int rel = step - __shfl(step, fl);
    for (int rr = 0; __any(tk && rel >= rr); ++rr) {
      const bool mine = tk && rel == rr;
      if (mine) {
        gx[k] += gkx;
        gy[k] += gky;
        gz[k] += gkz;
      }
      wave_lds_order();
      if (mine) {
        gx[j] += gjx;
        gy[j] += gjy;
        gz[j] += gjz;
      }
      wave_lds_order();
    }
  }
  if (take) {
    const int64_t e0 = offsets[i];
    for (int t = l; t < ng; t += kPackLanes) {
      const int ts = g * kPackSlots + t;
      pg[e0 + nb_entry(nb.f[ts])] = make_float4(gx[ts], gy[ts], gz[ts], 0.f);
    }
  }
}

// F_k = sum over entries e of row k of (pg[e] - pg[rev[e]]).  Sixteen lanes
// per atom take the row's entries round robin; the partial sums are combined
// by a fixed xor-shuffle tree, so the result does not depend on scheduling.
// With the list's bin order, block b takes the atoms of slot block
// (b mod 8) * per + b / 8: consecutive blocks go to different XCDs, so each
// XCD walks one contiguous stretch of the bin order and the neighbor rows
// its atoms read back stay in its L2.
__global__ void __launch_bounds__(256) k_force_gather(int64_t N, const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ rev, const float4* __restrict__ pg,
                                                      const int32_t* __restrict__ order, float* __restrict__ F,
                                                      const int64_t* meta, unsigned n_gather_blocks, EnergyJob ej) {
  if (blockIdx.x >= n_gather_blocks) {
    energy_block_sum(ej.E_atom, ej.atom_ptr, N, (int)(blockIdx.x - n_gather_blocks), ej.E_struct);
    return;
  }
  const bool valid = meta[kMetaValid] == 1;
  int64_t blk = blockIdx.x;
  if (order) {
    const unsigned per = (n_gather_blocks + 7) / 8;
    blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  const int64_t slot = ((blk * blockDim.x) + threadIdx.x) >> 4;
  const int sub = threadIdx.x & 15;
  int64_t k = slot;
  if (order && valid && slot < N) k = order[slot];
  float fx = 0.f, fy = 0.f, fz = 0.f;
  if (slot < N && valid) {
    const int64_t e1 = offsets[k + 1];
    for (int64_t e = offsets[k] + sub; e < e1; e += 16) {
      const float4 a = pg[e], b = pg[rev[e]];
      fx += a.x - b.x;
      fy += a.y - b.y;
      fz += a.z - b.z;
    }
  }
#pragma unroll
  for (int m = 8; m > 0; m >>= 1) {
    fx += __shfl_xor(fx, m, 16);
    fy += __shfl_xor(fy, m, 16);
    fz += __shfl_xor(fz, m, 16);
  }
  if (sub == 0 && slot < N) {
    F[3 * k] = fx;
    F[3 * k + 1] = fy;
    F[3 * k + 2] = fz;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// The packed passes take the mBP term, with their LDS within 48 KB.
bool packed_supported(const DescConst& P) {
  if (P.kind == NN_DESC_BP) return false;
  const int NB = P.n_theta * P.n_rs_ang;
  const size_t adj = sizeof(float) * kPackAtoms * packed_lam_stride(P.S, P.n_rad, NB);
  return packed_fwd_lds(P.S, NB) <= 48 * 1024 && adj <= 48 * 1024;
}

// Waves per atom: two when the atoms alone would leave the SIMDs with few
// waves to switch between, one otherwise; the packed passes for short rows
// (small molecules: at most 24 list entries per atom on average).  MLP: the
// row-block kernel.
LaunchPlan plan_default(int64_t n_atoms, const DescConst& P, int64_t capacity) {
  const int w = n_atoms <= 16384 ? 2 : 1;
  LaunchPlan plan{w, w, 1};  // the row-block MLP where it takes the shape (FP32), else the tile kernel's default
  const bool short_rows = n_atoms > 0 && capacity <= 24 * n_atoms;
  if (short_rows && packed_supported(P)) {
    plan.wpa_fwd = plan.wpa_adj = 0;
  } else if (short_rows && P.S > 1) {
    // several species: one wave per atom, so that the forward and tangent
    // passes take one MFMA block per species pair
    plan.wpa_fwd = 1;
  }
  return plan;
}

template <int NT, int NRA, int WPA, int ZC>
static void launch_fwd_w(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* G, IdentityGroup one,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_desc_fwd<NT, NRA, WPA, ZC>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64 * WPA), 0, s,
                     sys, nl.offsets, nl.nbr, nl.shift, P, G, nl.meta, one, nl.order);
}

// The packed forward (atoms with rows of at most kPackNb entries) and the
// one-atom pass over the longer rows.
template <int NT, int NRA, int ZC>
static void launch_fwd_packed(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* G,
                              IdentityGroup one, hipStream_t s) {
  hipLaunchKernelGGL((k_desc_fwd_packed<NT, NRA, ZC>), dim3(packed_grid(sys.n_atoms)), dim3(64),
                     packed_fwd_lds(P.S, NT * NRA), s, sys, nl.offsets, nl.nbr, nl.shift, P, G, nl.meta);
  hipLaunchKernelGGL((k_desc_fwd_long<NT, NRA, ZC>), dim3((unsigned)((sys.n_atoms + kWave - 1) / kWave)), dim3(64), 0,
                     s, sys, nl.offsets, nl.nbr, nl.shift, P, G, nl.meta, one, nl.order);
}

template <int NT, int NRA>
static void launch_fwd_t(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* G, IdentityGroup one,
                         int wpa, hipStream_t s) {
  if (wpa == 0 && packed_supported(P)) {
    if (P.zeta == 50) launch_fwd_packed<NT, NRA, 50>(sys, nl, P, G, one, s);
    else launch_fwd_packed<NT, NRA, 0>(sys, nl, P, G, one, s);
    return;
  }
  if (P.kind == NN_DESC_BP) {
    if (wpa == 4) launch_fwd_w<NT, NRA, 4, kZcBP>(sys, nl, P, G, one, s);
    else if (wpa == 2) launch_fwd_w<NT, NRA, 2, kZcBP>(sys, nl, P, G, one, s);
    else launch_fwd_w<NT, NRA, 1, kZcBP>(sys, nl, P, G, one, s);
  } else if (P.zeta == 50) {
    if (wpa == 4) launch_fwd_w<NT, NRA, 4, 50>(sys, nl, P, G, one, s);
    else if (wpa == 2) launch_fwd_w<NT, NRA, 2, 50>(sys, nl, P, G, one, s);
    else launch_fwd_w<NT, NRA, 1, 50>(sys, nl, P, G, one, s);
  } else {
    if (wpa == 4) launch_fwd_w<NT, NRA, 4, 0>(sys, nl, P, G, one, s);
    else if (wpa == 2) launch_fwd_w<NT, NRA, 2, 0>(sys, nl, P, G, one, s);
    else launch_fwd_w<NT, NRA, 1, 0>(sys, nl, P, G, one, s);
  }
}

template <int NT, int NRA, int WPA, int ZC>
static void launch_tan_w(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* v, float* U,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_desc_tan<NT, NRA, WPA, ZC>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64 * WPA), 0, s,
                     sys, nl.offsets, nl.nbr, nl.shift, P, v, U, nl.meta, nl.order);
}

template <int NT, int NRA>
static void launch_tan_t(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* v, float* U,
                         int wpa, hipStream_t s) {
  if (P.kind == NN_DESC_BP) {
    if (wpa == 4) launch_tan_w<NT, NRA, 4, kZcBP>(sys, nl, P, v, U, s);
    else if (wpa == 2) launch_tan_w<NT, NRA, 2, kZcBP>(sys, nl, P, v, U, s);
    else launch_tan_w<NT, NRA, 1, kZcBP>(sys, nl, P, v, U, s);
  } else if (P.zeta == 50) {
    if (wpa == 4) launch_tan_w<NT, NRA, 4, 50>(sys, nl, P, v, U, s);
    else if (wpa == 2) launch_tan_w<NT, NRA, 2, 50>(sys, nl, P, v, U, s);
    else launch_tan_w<NT, NRA, 1, 50>(sys, nl, P, v, U, s);
  } else {
    if (wpa == 4) launch_tan_w<NT, NRA, 4, 0>(sys, nl, P, v, U, s);
    else if (wpa == 2) launch_tan_w<NT, NRA, 2, 0>(sys, nl, P, v, U, s);
    else launch_tan_w<NT, NRA, 1, 0>(sys, nl, P, v, U, s);
  }
}

template <int NT, int NRA, bool ONE, int WPA, int ZC>
static void launch_adj_w(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam, float4* pg,
                         hipStream_t s) {
  const size_t lds =
      sizeof(float) * ((size_t)adj_lam_radial(P.S, P.n_rad) + (size_t)(P.S * (P.S + 1) / 2) * (NT * NRA + 4));
  hipLaunchKernelGGL((k_desc_adj<NT, NRA, ONE, WPA, ZC>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64 * WPA), lds,
                     s, sys, nl.offsets, nl.nbr, nl.shift, P, lam, pg, nl.meta, nl.order);
}

template <int NT, int NRA, bool ONE, int ZC>
static void launch_adj_packed(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam,
                              float4* pg, hipStream_t s) {
  const size_t lds = sizeof(float) * kPackAtoms * packed_lam_stride(P.S, P.n_rad, NT * NRA);
  hipLaunchKernelGGL((k_desc_adj_packed<NT, NRA, ONE, ZC>), dim3(packed_grid(sys.n_atoms)), dim3(64), lds, s, sys,
                     nl.offsets, nl.nbr, nl.shift, P, lam, pg, nl.meta);
  const size_t lds1 =
      sizeof(float) * ((size_t)adj_lam_radial(P.S, P.n_rad) + (size_t)(P.S * (P.S + 1) / 2) * (NT * NRA + 4));
  hipLaunchKernelGGL((k_desc_adj_long<NT, NRA, ONE, ZC>), dim3((unsigned)((sys.n_atoms + kWave - 1) / kWave)),
                     dim3(64), lds1, s, sys, nl.offsets, nl.nbr, nl.shift, P, lam, pg, nl.meta, nl.order);
}

template <int NT, int NRA, bool ONE>
static void launch_adj_o(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam, float4* pg,
                         int wpa, hipStream_t s) {
  if (wpa == 0 && packed_supported(P)) {
    if (P.zeta == 50) launch_adj_packed<NT, NRA, ONE, 50>(sys, nl, P, lam, pg, s);
    else launch_adj_packed<NT, NRA, ONE, 0>(sys, nl, P, lam, pg, s);
    return;
  }
  if (P.kind == NN_DESC_BP) {
    if (wpa == 4) launch_adj_w<NT, NRA, ONE, 4, kZcBP>(sys, nl, P, lam, pg, s);
    else if (wpa == 2) launch_adj_w<NT, NRA, ONE, 2, kZcBP>(sys, nl, P, lam, pg, s);
    else launch_adj_w<NT, NRA, ONE, 1, kZcBP>(sys, nl, P, lam, pg, s);
  } else if (P.zeta == 50) {
    if (wpa == 4) launch_adj_w<NT, NRA, ONE, 4, 50>(sys, nl, P, lam, pg, s);
    else if (wpa == 2) launch_adj_w<NT, NRA, ONE, 2, 50>(sys, nl, P, lam, pg, s);
    else launch_adj_w<NT, NRA, ONE, 1, 50>(sys, nl, P, lam, pg, s);
  } else {
    if (wpa == 4) launch_adj_w<NT, NRA, ONE, 4, 0>(sys, nl, P, lam, pg, s);
    else if (wpa == 2) launch_adj_w<NT, NRA, ONE, 2, 0>(sys, nl, P, lam, pg, s);
    else launch_adj_w<NT, NRA, ONE, 1, 0>(sys, nl, P, lam, pg, s);
  }
}

template <int NT, int NRA>
static void launch_adj_t(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam, float4* pg,
                         int wpa, hipStream_t s) {
  if (P.S == 1) launch_adj_o<NT, NRA, true>(sys, nl, P, lam, pg, wpa, s);
  else launch_adj_o<NT, NRA, false>(sys, nl, P, lam, pg, wpa, s);
}

bool desc_supported(int nt, int nra) {
  return (nt == 4 || nt == 8 || nt == 16) && (nra == 4 || nra == 8) && nt * nra <= 128;
}

#define NNP_DISPATCH(NT_, NRA_, CALL)                                          \
  do {                                                                         \
    if (nt == 4 && nra == 4) { constexpr int NT_ = 4, NRA_ = 4; CALL; }        \
    else if (nt == 4 && nra == 8) { constexpr int NT_ = 4, NRA_ = 8; CALL; }   \
    else if (nt == 8 && nra == 4) { constexpr int NT_ = 8, NRA_ = 4; CALL; }   \
    else if (nt == 8 && nra == 8) { constexpr int NT_ = 8, NRA_ = 8; CALL; }   \
    else if (nt == 16 && nra == 4) { constexpr int NT_ = 16, NRA_ = 4; CALL; } \
    else if (nt == 16 && nra == 8) { constexpr int NT_ = 16, NRA_ = 8; CALL; } \
  } while (0)

void launch_desc_fwd(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* G, IdentityGroup one,
                     int wpa, hipStream_t s) {
  if (sys.n_atoms == 0) return;
  const int nt = P.n_theta, nra = P.n_rs_ang;
  NNP_DISPATCH(A, B, (launch_fwd_t<A, B>(sys, nl, P, G, one, wpa, s)));
}

void launch_desc_adj(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam, float4* pg,
                     int wpa, hipStream_t s) {
  if (sys.n_atoms == 0) return;
  const int nt = P.n_theta, nra = P.n_rs_ang;
  NNP_DISPATCH(A, B, (launch_adj_t<A, B>(sys, nl, P, lam, pg, wpa, s)));
}

void launch_desc_tan(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* v, float* U,
                     int wpa, hipStream_t s) {
  if (sys.n_atoms == 0) return;
  const int nt = P.n_theta, nra = P.n_rs_ang;
  NNP_DISPATCH(A, B, (launch_tan_t<A, B>(sys, nl, P, v, U, wpa, s)));
}

// F from the per-entry gradients; blocks past the gather's sum the
// per-structure energies (ej.B of them) in the same launch.
void launch_force_gather(const nn_system& sys, const nn_nlist& nl, const float4* pg, float* F, const EnergyJob& ej,
                         hipStream_t s) {
  unsigned ng = (unsigned)((sys.n_atoms * 16 + 255) / 256);
  if (nl.order) ng = (ng + 7) / 8 * 8;  // whole rounds of the eight XCDs (the extra slots are past N)
  if (ng + (unsigned)ej.B == 0) return;
  hipLaunchKernelGGL(k_force_gather, dim3(ng + (unsigned)ej.B), dim3(256), 0, s, sys.n_atoms, nl.offsets, nl.rev, pg,
                     nl.order, F, nl.meta, ng, ej);
}


// ---------------------------------------------------------------------------
// Stored Jacobian (the precomputed-derivative mode of Sec. II.A)
//
// Entry e = (i -> j) stores dG_i/dd_e in a compact row of
// js = pad4(n_rad + 3 + 3 S NT NRA) floats:
//   [0, n_rad)        d/dr [exp(-eta_rad (r - Rs_k)^2) fc(r)] of the radial
//                     bins of species s_j (the gradient is that times d/r);
//   [n_rad, n_rad+3)  d/r;
//   then for each partner species b = 0..S-1 the block (s_j, b) as three
//   component arrays (x, y, z), each of the NRA x NT bins dG[(s_j,b)][q][p] / dd_e.
// Entries at r >= rc are all zero.  One lane per neighbor j walks every
// partner k != j (both orders of each pair, so no lane writes another
// lane's row); blocks are flushed when k enters the next species segment.
// ---------------------------------------------------------------------------

__host__ __device__ inline int jac_stride(int n_rad, int S, int NB) { return (n_rad + 3 + 3 * S * NB + 3) / 4 * 4; }

template <int NT, int NRA, bool BP>
__global__ void __launch_bounds__(64) k_desc_jac(nn_system sys, const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ nbr, const int8_t* __restrict__ shift,
                                                 DescConst P, float* __restrict__ J, int64_t* meta,
                                                 const int32_t* __restrict__ order) {
  constexpr int NB = NT * NRA;
  __shared__ AtomNb nb;
  const int lane = threadIdx.x;
  const int S = P.S;
  const int js = jac_stride(P.n_rad, S, NB);
  if (meta[kMetaValid] != 1) return;
  const int64_t i = atom_of_block(order, sys.n_atoms, true);
  if (i < 0) return;
  const int64_t e0 = offsets[i], e1 = offsets[i + 1];
  {
    // rows of entries outside rc (skin lists) are all zero; valid rows are
    // written in full below, so no address is written twice
    const int c = struct_of_atom(sys.atom_ptr, sys.n_structs, i);
    double h[9];
    for (int k = 0; k < 9; ++k) h[k] = sys.cell[9 * (int64_t)c + k];
    const double xi[3] = {sys.pos[3 * i], sys.pos[3 * i + 1], sys.pos[3 * i + 2]};
    const char4* sh4 = reinterpret_cast<const char4*>(shift);
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int32_t j = nbr[e];
      const char4 s4 = sh4[e];
      double d[3];
      displacement64(xi, sys.pos + 3 * (int64_t)j, h, s4.x, s4.y, s4.z, d);
      const int sp = sys.species[j];
      if (!(norm2_64(d) < P.rc64 * P.rc64) || sp < 0 || sp >= S)
        for (int x = 0; x < js; ++x) J[e * js + x] = 0.f;
    }
  }
  stage_neighbors(nb, i, sys, offsets, nbr, shift, P, meta, nullptr);
  if (nb.bad) {
    for (int64_t x = e0 * js + lane; x < e1 * js; x += kWave) J[x] = 0.f;
    return;
  }
  const int n = nb.n;
  const float eta_r2 = P.eta_rad * 1.4426950408889634f;
  const float eta_a2 = P.eta_ang * 1.4426950408889634f;
  const int zeta1 = P.zeta - 1;
  const float zf = (float)P.zeta;
  for (int j0 = 0; j0 < n; j0 += kWave) {
    const int j = j0 + lane;
    const bool active = j < n;
    float4 u = make_float4(1.f, 0.f, 0.f, 1.f), fu = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) {
      u = nb.d[j];
      fu = nb.f[j];
    }
    float* row = J + (e0 + (active ? nb_entry(fu) : 0)) * js;
    if (active) {
      for (int k = 0; k < P.n_rad; ++k) {
        const float dr = (u.w - P.rs_rad[k]) + (fu.z - P.rs_rad_lo[k]);
        const float g = fexp2(-eta_r2 * dr * dr);
        row[k] = g * fmaf(-2.0f * P.eta_rad * dr, fu.x, fu.y);
      }
      row[P.n_rad] = u.x;
      row[P.n_rad + 1] = u.y;
      row[P.n_rad + 2] = u.z;
      for (int x = P.n_rad + 3 + 3 * S * NB; x < js; ++x) row[x] = 0.f;
    }
    const float iru = frcp(u.w);
    for (int b = 0; b < S; ++b) {
      float vx[NB], vy[NB], vz[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) vx[t] = vy[t] = vz[t] = 0.f;
      for (int k = nb.seg[b]; k < nb.seg[b + 1]; ++k) {
        if (!active || k == j) continue;
        const float4 v = nb.d[k], fv = nb.f[k];
        if constexpr (BP) {
          // standard BP term T = A_p(cos) R_q(s2) F3: dT/dd_u = A_p' R_q F3 e + A_p G_q with
          // e = d cos / dd_u and G_q = R_q (-eta_q F3 d s2/dd_u + d F3/dd_u),
          // d s2/dd_u = 2 (d_u - w), d F3/dd_u = fc'_u u^ fc_v fc_w - fc_u fc_v fc'_w w^
          const BpGeom g = bp_geom<true>(u, v, P);
          const float c = g.c;
          const float F3 = fu.x * fv.x * g.fw;
          const float irw = g.rw > 0.f ? frcp(g.rw) : 0.f;
          const float fuw = fu.y * fv.x * g.fw, fww = fu.x * fv.x * g.dfw * irw;
          const float dfx = fmaf(fuw, u.x, -fww * g.wx), dfy = fmaf(fuw, u.y, -fww * g.wy),
                      dfz = fmaf(fuw, u.z, -fww * g.wz);
          const float sx = 2.0f * fmaf(u.w, u.x, -g.wx), sy = 2.0f * fmaf(u.w, u.y, -g.wy),
                      sz = 2.0f * fmaf(u.w, u.z, -g.wz);
          float A[NT], dA[NT];
#pragma unroll
          for (int p = 0; p < NT; ++p) {
            const float base = fmaf(P.bp_lam[p], c, 1.0f);
            const float P1 = ipow_uniform(base, P.bp_zeta[p] - 1);
            A[p] = P.bp_pref[p] * P1 * base;
            dA[p] = P.bp_pref[p] * (float)P.bp_zeta[p] * P.bp_lam[p] * P1;
          }
          const float ex = (v.x - c * u.x) * iru, ey = (v.y - c * u.y) * iru, ez = (v.z - c * u.z) * iru;
#pragma unroll
          for (int q = 0; q < NRA; ++q) {
            const float R = fexp2(-P.bp_eta[q] * 1.4426950408889634f * g.s2);
            const float FR = F3 * R;
            const float ef = -P.bp_eta[q] * FR;
            const float gx = R * dfx + ef * sx, gy = R * dfy + ef * sy, gz = R * dfz + ef * sz;
#pragma unroll
            for (int p = 0; p < NT; ++p) {
              const float a = FR * dA[p];
              const int t = q * NT + p;
              vx[t] = fmaf(a, ex, fmaf(A[p], gx, vx[t]));
              vy[t] = fmaf(a, ey, fmaf(A[p], gy, vy[t]));
              vz[t] = fmaf(a, ez, fmaf(A[p], gz, vz[t]));
            }
          }
          continue;
        }
        const TripGeom g = triplet_geom(u, fu, v, fv, P.eps_ang);
        const float c = g.c;
        const float F2 = 2.0f * fu.x * fv.x;
        const float dF2 = 2.0f * fu.y * fv.x;  // dF2 / dr_u
        float x[NT], P1[NT], A[NT], dA[NT];
#pragma unroll
        for (int p = 0; p < NT; ++p) x[p] = fmaf(c, P.x_a[p], fmaf(g.ssm, P.x_b[p], P.x_c));
        ipow_array<NT>(x, zeta1, P1);
        const float issm = frcp(g.ssm);
#pragma unroll
        for (int p = 0; p < NT; ++p) {
          A[p] = P1[p] * x[p];
          // dA/dcos along the path cos -> (cos, ssm(cos)), ssm' = -cos/ssm
          dA[p] = zf * P1[p] * (P.x_a[p] - P.x_b[p] * c * issm);
        }
        // d cos/dd_u = (v^ - cos u^) / r_u ; d r_u/dd_u = u^
        const float ex = (v.x - c * u.x) * iru, ey = (v.y - c * u.y) * iru, ez = (v.z - c * u.z) * iru;
#pragma unroll
        for (int q = 0; q < NRA; ++q) {
          const float dq = (g.rbar - P.rs_ang[q]) + (g.rbar_lo - P.rs_ang_lo[q]);
          const float R = fexp2(-eta_a2 * dq * dq);
          const float FR = F2 * R;
          const float dFR = fmaf(F2 * R, -P.eta_ang * dq, dF2 * R);  // d(F2 R)/dr_u, with d rbar/dr_u = 1/2
#pragma unroll
          for (int p = 0; p < NT; ++p) {
            const float a = FR * dA[p];
            const float bcoef = A[p] * dFR;
            const int t = q * NT + p;
            vx[t] = fmaf(a, ex, fmaf(bcoef, u.x, vx[t]));
            vy[t] = fmaf(a, ey, fmaf(bcoef, u.y, vy[t]));
            vz[t] = fmaf(a, ez, fmaf(bcoef, u.z, vz[t]));
          }
        }
      }
      if (active) {
        float* blk = row + P.n_rad + 3 + b * NB * 3;  // x, y, z component arrays of NB bins each
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          blk[t] = vx[t];
          blk[NB + t] = vy[t];
          blk[2 * NB + t] = vz[t];
        }
      }
    }
  }
}

// pg[e] = sum_d lambda_i[d] dG_i[d]/dd_e from the stored rows: one wave per
// atom, lambda of the atom in LDS, 16 lanes per entry (four entries at a
// time).  The lanes of an entry stride over its row 16 floats at a time, so
// every load is 64 contiguous bytes per entry; the component-major angular
// blocks give bin t = 16 m + lane of each component without any division.
// The 16 partial sums are combined by a fixed shuffle tree.
template <int NT, int NRA>
__global__ void __launch_bounds__(64) k_jac_contract(nn_system sys, const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ nbr, DescConst P,
                                                     const float* __restrict__ lambda, const float* __restrict__ J,
                                                     float4* __restrict__ pg, int64_t* meta,
                                                     const int32_t* __restrict__ order) {
  constexpr int NB = NT * NRA;
  extern __shared__ float lam[];  // [D]
  const int lane = threadIdx.x, sub = lane & 15, grp = lane >> 4;
  const int S = P.S;
  const int js = jac_stride(P.n_rad, S, NB);
  if (meta[kMetaValid] != 1) return;
  const int64_t i = atom_of_block(order, sys.n_atoms, true);
  if (i < 0) return;
  if (meta[kMetaJac] != meta[kMetaBuilds] + 1) {
    // the list was rebuilt since the Jacobian was stored: its rows refer to
    // other entries, so the pair gradients are zero and the call is flagged
    for (int64_t e = offsets[i] + lane; e < offsets[i + 1]; e += kWave) pg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane == 0) atomicOr((unsigned long long*)&meta[kMetaErr], (unsigned long long)kErrStale);
    return;
  }
  for (int d = lane; d < P.D; d += kWave) lam[d] = lambda[i * (int64_t)P.D + d];
  __syncthreads();
  const int64_t e0 = offsets[i], e1 = offsets[i + 1];
  const int ang0 = P.n_rad * S;
  for (int64_t base = e0; base < e1; base += 4) {  // the same trip count in every lane
    const int64_t e = base + grp;
    float gr = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
    int sj = -1;
    if (e < e1) {
      sj = sys.species[nbr[e]];
      if (sj >= 0 && sj < S) {
        const float* row = J + e * js;
        for (int k = sub; k < P.n_rad; k += 16) gr = fmaf(lam[sj * P.n_rad + k], row[k], gr);
        for (int b = 0; b < S; ++b) {
          const float* L = lam + ang0 + pair_block(S, sj, b) * NB;
          const float* blk = row + P.n_rad + 3 + b * NB * 3;
#pragma unroll
          for (int m = 0; m < NB / 16; ++m) {
            const int t = 16 * m + sub;
            const float l = L[t];
            ax = fmaf(l, blk[t], ax);
            ay = fmaf(l, blk[NB + t], ay);
            az = fmaf(l, blk[2 * NB + t], az);
          }
        }
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      gr += __shfl_xor(gr, o, 16);
      ax += __shfl_xor(ax, o, 16);
      ay += __shfl_xor(ay, o, 16);
      az += __shfl_xor(az, o, 16);
    }
    if (e < e1 && sub == 0) {
      float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
      if (sj >= 0 && sj < S) {
        const float* u = J + e * js + P.n_rad;  // the unit vector d/r
        g = make_float4(fmaf(gr, u[0], ax), fmaf(gr, u[1], ay), fmaf(gr, u[2], az), 0.f);
      }
      pg[e] = g;
    }
  }
}

size_t jacobian_floats(int n_rad, int S, int nt, int nra, int64_t capacity) {
  return (size_t)jac_stride(n_rad, S, nt * nra) * (size_t)capacity;
}

template <int NT, int NRA>
static void launch_jac_t(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* J, hipStream_t s) {
  if (P.kind == NN_DESC_BP)
    hipLaunchKernelGGL((k_desc_jac<NT, NRA, true>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64), 0, s, sys,
                       nl.offsets, nl.nbr, nl.shift, P, J, nl.meta, nl.order);
  else
    hipLaunchKernelGGL((k_desc_jac<NT, NRA, false>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64), 0, s, sys,
                       nl.offsets, nl.nbr, nl.shift, P, J, nl.meta, nl.order);
}

template <int NT, int NRA>
static void launch_contract_t(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam,
                              const float* J, float4* pg, hipStream_t s) {
  hipLaunchKernelGGL((k_jac_contract<NT, NRA>), dim3(atom_grid(sys.n_atoms, nl.order)), dim3(64), sizeof(float) * P.D,
                     s, sys, nl.offsets, nl.nbr, P, lam, J, pg, nl.meta, nl.order);
}

void launch_desc_jac(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* J, hipStream_t s) {
  if (sys.n_atoms == 0) return;
  const int nt = P.n_theta, nra = P.n_rs_ang;
  NNP_DISPATCH(A, B, (launch_jac_t<A, B>(sys, nl, P, J, s)));
}

void launch_jac_contract(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam,
                         const float* J, float4* pg, hipStream_t s) {
  if (sys.n_atoms == 0) return;
  const int nt = P.n_theta, nra = P.n_rs_ang;
  NNP_DISPATCH(A, B, (launch_contract_t<A, B>(sys, nl, P, lam, J, pg, s)));
}

}  // namespace nnp
