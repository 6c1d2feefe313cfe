// Internal definitions shared by the HIP translation units of libnnpot.
// Not part of the public C ABI (that is include/nnpot.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nnpot.h"

namespace nnp {

constexpr int kWave = 64;
constexpr int kMaxRad = 64;      // radial bins per species
constexpr int kMaxTheta = 16;    // angle bins
constexpr int kMaxRsAng = 8;     // average-radius bins
constexpr int kMaxNb = 192;      // neighbors inside rc held per atom on chip
constexpr int kSmallMax = 256;   // structures up to this size use the all-pairs list builder
constexpr int kRowMax = 1024;    // list entries per row the row sorter accepts

// Device error bits, OR-ed into nl->meta[kMetaErr].
enum : int64_t {
  kErrCapacity = 1,   // list capacity exceeded (required size in meta[kMetaNnz])
  kErrCell = 2,       // periodic cell too narrow and structure too large for all-pairs
  kErrSpecies = 4,    // species index out of range
  kErrNonFinite = 8,  // non-finite position
  kErrTooMany = 16,   // more than kMaxNb neighbors inside rc, or a row over kRowMax
  kErrShift = 32,     // lattice image index does not fit in int8
  kErrPtr = 64,       // atom_ptr not 0 .. N nondecreasing
  kErrStale = 128,    // stored descriptors reused after the list was rebuilt
  kErrQeq = 256,      // charge equilibration: structure periodic, over kQeqMax atoms, or not positive definite
};

// Layout of the device metadata block of a neighbor list (nl->meta, int64[8]).
// kMetaJac: 1 + the build count of the list when the workspace's Jacobian
// was last stored (0: never), checked by the reuse path.
enum { kMetaNnz = 0, kMetaValid = 1, kMetaBuilds = 2, kMetaRebuilt = 3, kMetaErr = 4, kMetaJac = 5 };

// Per-structure geometry computed on the device before binning.
struct alignas(16) StructGeom {
  double h[9];      // cell rows a, b, c
  double inv[9];    // inverse: s = x * inv
  int32_t nb[3];    // bins per direction (large path) or image bound K (small path)
  int32_t small;    // 1: all-pairs path
  int64_t bin_base; // first bin of this structure
  int64_t n_bins;
};

// FP32 constants of the descriptor, passed by value to the kernels.
struct DescConst {
  int32_t S, n_rad, n_theta, n_rs_ang, D, zeta;  // zeta: integer exponent
  float rc, eta_rad, eta_ang, eps_ang;
  float pi_over_rc, half_pi_over_rc, fc_scale;   // pi/rc, pi/(2 rc)
  float x_a[kMaxTheta], x_b[kMaxTheta], x_c;     // x = c*x_a + ssm*x_b + x_c
  float rs_rad[kMaxRad], rs_rad_lo[kMaxRad];   // centre = hi + lo (double-float)
  float rs_ang[kMaxRsAng], rs_ang_lo[kMaxRsAng];
  double rc64, half_pi_over_rc64, pi_over_rc64;
  // standard BP angular term (kind 1): per angle term p the prefactor
  // 2 * 2^(1 - zeta_p) (both orders of each neighbor pair), lambda_p and the
  // integer exponent; per radius term q its width eta_q
  int32_t kind;
  float bp_pref[kMaxTheta], bp_lam[kMaxTheta], bp_eta[kMaxRsAng];
  int32_t bp_zeta[kMaxTheta];
  int32_t bp_zbits;  // bit length of the largest exponent
};

// One species' MLP as seen by the kernels.
struct MlpDev {
  int32_t n_layers;
  int32_t width[NN_MAX_LAYERS + 1];
  int32_t act[NN_MAX_LAYERS];
  const float* W[NN_MAX_LAYERS];       // [w_out][w_in] FP32
  const float* b[NN_MAX_LAYERS];
  const __bf16* Wb[NN_MAX_LAYERS];     // BF16 hi part [w_out][w_in] (BF16 modes)
  const __bf16* Wl[NN_MAX_LAYERS];     // BF16 lo part, W - hi (split mode)
  const __bf16* WbT[NN_MAX_LAYERS];    // transposed hi [w_in][w_out]
  const __bf16* WlT[NN_MAX_LAYERS];    // transposed lo
};
struct ModelDev {
  int32_t S;
  MlpDev m[NN_MAX_SPECIES];
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Displacement from atom i to image n of atom j, FP64, in the fixed order
// d = (x_j - x_i) + ((n_a a + n_b b) + n_c c), no contraction.
__device__ __forceinline__ void displacement64(const double* __restrict__ xi, const double* __restrict__ xj,
                                               const double* h, int na, int nb, int nc, double d[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; ++k) {
    double t = (double)na * h[0 + k];
    t = t + (double)nb * h[3 + k];
    t = t + (double)nc * h[6 + k];
    d[k] = (xj[k] - xi[k]) + t;
  }
}

__device__ __forceinline__ double norm2_64(const double d[3]) {
#pragma clang fp contract(off)
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

// ------------------------------------------------------------------------
// host-side launch helpers (defined in the .hip files)
// ------------------------------------------------------------------------

size_t scan_scratch_elems(int64_t n);
// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total), skipped
// when *predicate == 0; with n_dev, the small-n path scans only the first
// *n_dev entries (the large-n path always scans n).
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s,
                        const int32_t* predicate, const int64_t* n_dev = nullptr);

// neighbors.hip
struct NbLaunch {
  const nn_system* sys;
  double radius;
  int64_t capacity;
  nn_nlist* nl;      // null in count-only mode
  int64_t* counts;   // row counts [N+1]
  int64_t* offsets;  // scan output [N+1]: nl->offsets or scratch
  StructGeom* geom;
  int64_t* n_bins;   // [B+1]
  int64_t* bin_base; // [B+1]
  int64_t* bin_count;
  int64_t* bin_start;
  int32_t* bin_rank;  // [N] rank of each atom inside its bin
  int4* bin_m;       // [N] per binned slot: atom j and its whole-cell offsets
  double4* bin_x;    // [N] per binned slot: the position of j (copied bit for bit)
  uint64_t* row_keys; // N slabs of kslot keys, then an overflow area of 2 * capacity keys
  int64_t* key_loc;   // [N] start of each row's sorted keys in row_keys
  int64_t* cursor;    // overflow area use
  int kslot;
  int32_t* atom_bin;
  int64_t* scan_tmp;
  int32_t* flag;
  int64_t* meta;
  int64_t max_bins;
};
// Keys per atom in the counting pass's slab for a list of `capacity` entries
// over n_atoms atoms (0 when there is no list to fill).
int row_key_slot(int64_t n_atoms, int64_t capacity);
void launch_neighbors(const NbLaunch& L, bool use_skin, double skin, bool count_only, hipStream_t s);

// descriptors.hip
bool desc_supported(int nt, int nra);
// With one species the grouping is the identity: the descriptor launch
// writes perm[i] = i and sp_start = {0, N} itself (and flags atoms whose
// species is not 0) when perm is set.
struct IdentityGroup {
  int32_t* perm;
  int64_t* sp_start;
};
// Launch choices that change the speed of a pass but not what it computes
// (only the order of some sums): waves per atom of the descriptor forward
// and adjoint passes (1, 2 or 4; 0 = the packed passes, four short-row atoms
// per wave, where packed_supported) and waves per MLP tile (4 or 8; 0 = the
// default; 1 = the FP32 row-block MLP where mlp_rows_supported).  Defaults
// come from plan_default(); nn_autotune stores measured ones per shape
// class.
struct LaunchPlan {
  int wpa_fwd, wpa_adj, mlp_waves;
};
bool packed_supported(const DescConst& P);
LaunchPlan plan_default(int64_t n_atoms, const DescConst& P, int64_t capacity);
void launch_desc_fwd(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* G, IdentityGroup one,
                     int wpa, hipStream_t s);
void launch_desc_adj(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam, float4* pg,
                     int wpa, hipStream_t s);
// U [N][D] = directional derivative of the descriptors along the
// displacement field v [N][3] (FP32)
void launch_desc_tan(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* v, float* U,
                     int wpa, hipStream_t s);
// FP64 sum of E_atom over structure c by one block of 256 threads (a fixed
// tree, so the result is the same on every run).
__device__ __forceinline__ void energy_block_sum(const float* __restrict__ E_atom, const int64_t* __restrict__ atom_ptr,
                                                 int64_t N, int c, double* __restrict__ E_struct) {
  __shared__ double sh[256];
  const int64_t a0 = min(max(atom_ptr[c], (int64_t)0), N), a1 = min(max(atom_ptr[c + 1], a0), N);
  double acc = 0.0;
  for (int64_t a = a0 + threadIdx.x; a < a1; a += 256) acc += (double)E_atom[a];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) E_struct[c] = sh[0];
}
struct EnergyJob {  // per-structure energy sums run by extra blocks of the gather
  const float* E_atom;
  const int64_t* atom_ptr;
  int32_t B;
  double* E_struct;
};
void launch_force_gather(const nn_system& sys, const nn_nlist& nl, const float4* pg, float* F, const EnergyJob& ej,
                         hipStream_t s);
size_t jacobian_floats(int n_rad, int S, int nt, int nra, int64_t capacity);
void launch_desc_jac(const nn_system& sys, const nn_nlist& nl, const DescConst& P, float* J, hipStream_t s);
void launch_jac_contract(const nn_system& sys, const nn_nlist& nl, const DescConst& P, const float* lam,
                         const float* J, float4* pg, hipStream_t s);

// mlp.hip
struct MlpArgs {
  ModelDev model;
  const float* G;           // [N][D]
  const int32_t* perm;      // [N] atoms grouped by species
  const int64_t* sp_start;  // [S+1]
  float* E_atom;            // [N]
  float* lambda;            // [N][D] (null: energies only)
  int D;
  // optional per-atom stash for the weight gradient (null: not written):
  // a1 / delta1 = dE/dz1 [N][H1], a2 / delta2 = dE/dz2 [N][H2]
  float *st_a1, *st_d1, *st_a2, *st_d2;
};
// The MLP and its tangent along the descriptor tangent U (FP32 MFMA), with
// the per-atom terms of the weight gradient of sum_i (w_i E_i - E_dot_i).
struct MlpFmArgs {
  ModelDev model;
  const float* G;           // [N][D]
  const float* U;           // [N][D] descriptor tangent
  const int32_t* perm;
  const int64_t* sp_start;
  const float* w;           // [N] dL/dE of each atom's structure
  float* E_atom;            // [N]
  int D;
  // per-atom stash [N][H1]: a1, a1_dot (t1), delta1 (d1), x1 = w delta1 - eps1;
  // [N][H2]: delta2 (d2), x2 = w delta2 - eps2, c3 = w a2 - a2_dot
  float *a1, *t1, *d1, *x1, *d2, *x2, *c3;
};
struct ConvJob {
  int n;
  const float* src[NN_MAX_SPECIES * 2];
  __bf16* hi[NN_MAX_SPECIES * 2];
  __bf16* lo[NN_MAX_SPECIES * 2];
  __bf16* hiT[NN_MAX_SPECIES * 2];
  __bf16* loT[NN_MAX_SPECIES * 2];
  int rows[NN_MAX_SPECIES * 2], cols[NN_MAX_SPECIES * 2];
};
void launch_species_group(const int32_t* species, int64_t N, int S, int64_t* cnt, int64_t* off, int64_t* scan_tmp,
                          int32_t* perm, int64_t* sp_start, hipStream_t s);
bool mlp_supported(int h1, int h2);
// mode 0 FP32, 1 BF16, 2 split BF16; waves per tile 4 or 8 (0: default)
void launch_mlp(const MlpArgs& a, int h1, int h2, int mode, int64_t N, int waves, hipStream_t s);
// mlp_rows.hip: the FP32 row-block MLP (64 atoms per block, weights staged in
// LDS); shapes (64, 32) and (128, 128) with D a multiple of 4
bool mlp_rows_supported(int h1, int h2, int D);
void launch_mlp_rows(const MlpArgs& a, int h1, int h2, int64_t N, hipStream_t s);
// its BF16 modes (mode 1 plain, 2 split; the BF16 weight copies prepared),
// D a multiple of 8
bool mlp_rows_bf_supported(int h1, int h2, int D);
void launch_mlp_rows_bf(const MlpArgs& a, int h1, int h2, int mode, int64_t N, hipStream_t s);
void launch_convert_bf16(const ConvJob& job, hipStream_t s);
void launch_mlp_fm(const MlpFmArgs& a, int h1, int h2, int64_t N, int waves, hipStream_t s);
// mlp_layers.hip: per-species networks of any depth (up to NN_MAX_LAYERS
// weight layers) and widths, layer by layer.  Stashes of hidden layer h
// (1 .. NN_MAX_LAYERS - 1) are [rows in species order][ld[h]]: activations a,
// act' (s), and for the passes that need them the adjoint d (delta, or z_bar
// with a loss on forces), the tangent activations at, act'' z_dot (q) and the
// tangent adjoint dt.
struct LayBuf {
  float* a[NN_MAX_LAYERS];
  float* s[NN_MAX_LAYERS];
  float* d[NN_MAX_LAYERS];
  float* at[NN_MAX_LAYERS];
  float* q[NN_MAX_LAYERS];
  float* dt[NN_MAX_LAYERS];
  int ld[NN_MAX_LAYERS];
};
struct LayArgs {
  ModelDev model;
  const int32_t* perm;
  const int64_t* sp_start;
  const float* G;       // [N][D] descriptors (atom order)
  const float* U;       // [N][D] descriptor tangent (loss on forces)
  int D;
  const float* w_atom;  // [N] dL/dE of each atom's structure (gradient passes)
  float* E_atom;        // [N]
  float* lambda;        // [N][D] dE/dG
  LayBuf buf;
  // networks with n_out outputs per atom (charge equilibration: local energy,
  // electronegativity, hardness): out [N][n_out] receives them, and seed
  // [N][n_out] holds the per-atom weights of the outputs that the backward
  // pass and the weight gradient differentiate (null: one output, seed 1)
  int n_out;
  float* out;
  const float* seed;
};
struct LayGradOut {
  float* dW[NN_MAX_SPECIES * NN_MAX_LAYERS];
  float* db[NN_MAX_SPECIES * NN_MAX_LAYERS];
};
// ld[h] of the stashes (widest hidden layer h over the species, rounded up to 16)
void lay_stash_widths(const ModelDev& m, int ld[NN_MAX_LAYERS]);
size_t lay_partial_floats(int64_t N, const ModelDev& m);
// E_atom, and with lambda the stashed deltas and dE/dG
void launch_mlp_layers(const LayArgs& a, int64_t N, bool lambda, hipStream_t s);
// networks with several outputs: the forward pass writing a.out [N][n_out];
// then, once a.seed is known, the stashed deltas of sum_o seed_o out_o and
// (with lambda) its derivative with respect to G
void launch_mlp_layers_outputs(const LayArgs& a, int64_t N, hipStream_t s);
void launch_mlp_layers_seeded_backward(const LayArgs& a, int64_t N, bool lambda, hipStream_t s);
// forward with the tangent along U and the reverse pass of w E - E_dot
void launch_mlp_layers_tangent(const LayArgs& a, int64_t N, hipStream_t s);
// dL/dW, dL/db from the stashes (energy path or, with tangent, both terms)
void launch_lay_wgrad(const LayArgs& a, int64_t N, bool tangent, float* partial, const LayGradOut& out, hipStream_t s);

// qeq.hip: charge equilibration per structure (Sec. II.B)
constexpr int kQeqMax = 64;  // atoms per structure the on-chip solve takes
struct QeqArgs {
  const double* pos;        // [N][3]
  const int32_t* species;   // [N]
  const int64_t* atom_ptr;  // [B+1]
  const uint8_t* pbc;       // [B][3]
  int32_t B;
  int64_t N;
  const float* out;         // [N][3] network outputs E0, chi, J
  const double* total;      // [B] total charge of each structure
  double sigma[NN_MAX_SPECIES];
  double ke;                // e^2 / (4 pi eps0)
  double* E_struct;         // [B]
  double* q;                // [N] charges
  float* seed;              // [N][3] (1, q, q^2 / 2)
  int64_t* meta;            // error bits
};
void launch_qeq_solve(const QeqArgs& a, hipStream_t s);
// F [N][3] += the Coulomb pair forces at the charges a.q
void launch_qeq_coulomb(const QeqArgs& a, float* F, hipStream_t s);

// wgrad.hip
struct WgradArgs {
  const int32_t* perm;      // atoms grouped by species
  const int64_t* sp_start;  // [S+1]
  const float* w;           // [N] per-atom weight dL/dE of its structure
  float* partial;           // chunk partial sums
  int S;
};
size_t wgrad_partial_floats(int64_t N, int S, const ModelDev& m);
// Per-atom sources of the weight-gradient sums.  Energy term only: G, a1,
// d1 = delta1, a2, d2 = delta2 (weighted by w inside).  With the force term
// (x1 set): a2 holds c3, and x1, x2, U, t1 = a1_dot are used as well.
struct WgradSrc {
  const float *G, *a1, *d1, *a2, *d2;
  const float *U, *t1, *x1, *x2;
};
void launch_wgrad(const WgradArgs& a, const ModelDev& m, const WgradSrc& src, int D, int64_t N, float* const* dW,
                  float* const* db, hipStream_t s);
void launch_atom_weights(const double* dL_dE, const int64_t* atom_ptr, int32_t B, int64_t N, float* w, hipStream_t s);
void launch_pos_grad(const double* dL_dE, const int64_t* atom_ptr, int32_t B, int64_t N, const float* F,
                     float* dL_dpos, hipStream_t s);
void launch_energy_reduce(const float* E_atom, const int64_t* atom_ptr, int32_t B, int64_t N, double* E_struct,
                          hipStream_t s);
// loss.hip
size_t loss_partial_elems(int64_t N, int32_t B);
void launch_loss(const nn_loss_params& lp, const int64_t* atom_ptr, int32_t B, int64_t N, const double* E,
                 const double* T, const float* F, const float* Fr, double* L, double* dL_dE, float* dL_dF,
                 double* partial, hipStream_t s);
// md.hip: one integrator update of the BAOAB Langevin splitting per atom.
//   kMdHalfKickDrift: B A O A (the first step);
//   kMdKickDrift:     a kick of dt (the previous step's last B and this
//                     step's first B), then A O A;
//   kMdKick:          the last B only.
enum { kMdHalfKickDrift = 0, kMdKickDrift = 1, kMdKick = 2 };
void launch_md_update(int64_t N, int mode, double* pos, double* vel, const double* inv_mass, const float* F,
                      const float* noise, double dt, double c1, double c2_sqrt_kT, hipStream_t s);

}  // namespace nnp
