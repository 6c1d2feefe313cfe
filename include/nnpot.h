/*
 * nnpot.h -- C ABI of libnnpot, the MI355X (gfx950) energy/force path of a
 * Behler-Parrinello-type neural network potential with modified-BP (mBP)
 * descriptors and per-species multilayer perceptrons (PANNA 2.0).
 *
 * Conventions shared by every call:
 *  - Pointers marked [device] point to GPU memory of the current HIP device;
 *    pointers marked [host] point to host memory read during the call only.
 *  - The caller owns every buffer, including the workspace; the library never
 *    allocates and never frees.  Inputs are never modified.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work on it and return; the only synchronous call is nn_count_neighbors.
 *  - Host-detectable errors (bad sizes, null pointers, unsupported parameter
 *    combinations, short workspace) are returned before anything is enqueued,
 *    with a message available from nn_last_error().  Errors found on the
 *    device (list overflow, species out of range, non-finite positions, too
 *    many neighbors) are recorded in the list's metadata block and reported
 *    by nn_check(), which synchronizes the stream.
 *  - Results are bitwise reproducible run to run: no floating-point atomics.
 *  - Structures are contiguous atom ranges; each has its own cell and
 *    periodicity.  Energies of different structures never interact (the
 *    energy is a sum of atomic terms with a finite cutoff, Sec. I and II).
 */
#ifndef NNPOT_H
#define NNPOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NN_MAX_SPECIES 8
#define NN_MAX_LAYERS 4

typedef enum nn_status {
  NN_OK = 0,
  NN_E_INVALID = 1,     /* invalid argument (message in nn_last_error)                 */
  NN_E_CAPACITY = 2,    /* neighbor list capacity too small; nn_check reports the size  */
  NN_E_CELL = 3,        /* periodic cell narrower than 3 bins and > 256 atoms          */
  NN_E_WORKSPACE = 4,   /* workspace smaller than nn_workspace_size                     */
  NN_E_UNSUPPORTED = 5, /* parameter combination without a compiled kernel              */
  NN_E_HIP = 6,         /* HIP runtime error (message in nn_last_error)                 */
  NN_E_DEVICE = 7       /* device-side check failed (species, non-finite input, limits) */
} nn_status;

/* Activation codes of Eq. (1): Gaussian exp(-z^2), ReLU, tanh, linear (Sec. II.A). */
enum { NN_ACT_LINEAR = 0, NN_ACT_GAUSSIAN = 1, NN_ACT_RELU = 2, NN_ACT_TANH = 3 };

/* Flags of nn_energy_forces. */
enum {
  NN_BF16_MLP = 1,       /* MLP products on BF16 MFMA, operands rounded to BF16, FP32 sums.
                            Rounding G, W and the activations to 8 significant bits costs
                            force accuracy: measured max |dF| against the FP64 reference is
                            2.7e-2 eV/A on a 32768-atom 4-species bulk cell and 1.3e-2 on a
                            262144-atom one, 13-27x over a 1e-3 eV/A force tolerance (energies
                            stay within 1e-4 eV/atom).  Use NN_BF16X3_MLP where forces must
                            meet 1e-3 eV/A.  Fastest MLP mode (about half the FP32 MLP
                            time on batches of small molecules).                              */
  NN_STORE_JACOBIAN = 2, /* store dG/dx during the descriptor pass if it fits mem_budget        */
  NN_BF16X3_MLP = 4,     /* MLP products on BF16 MFMA with every operand split into BF16 hi + lo
                            and three products (hi*hi + hi*lo + lo*hi), FP32 sums: about 16
                            significant bits per operand (forces within 1e-3 eV/A), and with
                            the row-block MLP faster than FP32 (the MLP in about 0.65x the
                            FP32 time).  Exclusive with NN_BF16_MLP.
                            Neither flag: FP32 MFMA.                                           */
  NN_REUSE_DESCRIPTORS = 8 /* skip the descriptor pass: use G and the Jacobian that an earlier
                              NN_STORE_JACOBIAN call with the same positions and list left in
                              this workspace (weights may have changed).  A list rebuilt since
                              that call is detected on the device: the forces are then zero
                              and nn_check reports NN_E_DEVICE.  Positions moved without a
                              rebuild are not detected.                                        */
};


/*
 * A batch of atomic configurations (Sec. II.A: positions, species, cell).
 *   pos      [device] [N][3] FP64 Cartesian positions (Angstrom); need not be
 *            wrapped into the cell.
 *   species  [device] [N] int32 species index in [0, S).
 *   atom_ptr [device] [B+1] int64; structure c owns atoms
 *            [atom_ptr[c], atom_ptr[c+1]); atom_ptr[0] = 0, atom_ptr[B] = N.
 *   cell     [device] [B][3][3] FP64, rows are the lattice vectors a, b, c.
 *            Must be non-singular also for non-periodic structures, where it
 *            only sets the binning box (atoms may lie outside it).
 *   pbc      [device] [B][3] uint8, 1 = periodic along that lattice vector.
 */
typedef struct nn_system {
  int64_t n_atoms;
  int32_t n_structs;
  const double* pos;
  const int32_t* species;
  const int64_t* atom_ptr;
  const double* cell;
  const uint8_t* pbc;
} nn_system;

/*
 * Neighbor list in CSR form.  Row i lists every (j, n) of the same structure
 * with (j, n) != (i, 0) and |d|^2 < radius^2, where
 * d = (x_j - x_i) + (n_a a + n_b b + n_c c) is evaluated in FP64 in exactly
 * that order; rows are sorted by (j, n_a, n_b, n_c).  Image shifts refer to
 * the input (unwrapped) positions.  All arrays are caller-allocated [device]:
 *   offsets [N+1] int64, nbr [capacity] int32, shift [capacity][4] int8
 *   (n_a, n_b, n_c, 0), rev [capacity] int32 (index of the reverse entry
 *   (j -> i, -n)), ref_pos [N][3] FP64 (positions at the last build),
 *   meta [8] int64 (nnz, valid, builds, rebuilt-last-call, error bits,
 *   1 + builds at the last NN_STORE_JACOBIAN call, -, -); zero meta once
 *   before the first build;
 *   order [N] int32, optional (NULL: not kept): the atoms in cell-bin order
 *   at the last build.  When present, the force gather walks the atoms in
 *   this order, each XCD taking a contiguous run of it, so that the rows
 *   read together are those of nearby atoms and share that XCD's L2.
 * radius is written by nn_build_neighbors (host field).
 */
typedef struct nn_nlist {
  int64_t capacity;
  int64_t* offsets;
  int32_t* nbr;
  int8_t* shift;
  int32_t* rev;
  double* ref_pos;
  int64_t* meta;
  int32_t* order;
  double radius;
} nn_nlist;

/*
 * mBP descriptor hyperparameters [host].  The paper names the mBP descriptor
 * and its bin counts (Sec. II.A, III.A, III.B) but defers its formulas to the
 * first PANNA paper; the form computed is
 *   radial  G[s][k]      = sum_{j: s_j=s} exp(-eta_rad (r_ij - rs_rad[k])^2) fc(r_ij)
 *   angular G[(a,b)][q][p] = sum_{unordered {j,k}: {s_j,s_k}={a,b}}
 *       2 x_p^zeta exp(-eta_ang ((r_ij + r_ik)/2 - rs_ang[q])^2) fc(r_ij) fc(r_ik),
 *   x_p = (1 + cos(t) cos(theta_s[p]) + sqrt(sin^2(t) + eps) sin(theta_s[p]))
 *         / (1 + sqrt(1 + eps)),   fc(r) = (1 + cos(pi r / rc)) / 2 for r < rc.
 * Layout of G: S radial blocks of n_rad, then the angular blocks of the
 * unordered species pairs (0,0), (0,1), ..., (S-1,S-1), each [q][p] with p
 * fastest: D = n_rad*S + n_theta*n_rs_ang*S*(S+1)/2.
 * Limits: S <= 8, n_rad <= 64, (n_theta, n_rs_ang) in {4,8,16} x {4,8} with
 * n_theta*n_rs_ang <= 128, zeta a positive integer <= 1024.
 *
 * kind = NN_DESC_BP selects the standard Behler-Parrinello angular term
 * instead (Sec. II.A names both descriptors):
 *   angular G[(a,b)][q][p] = sum_{ordered (j,k), j != k: {s_j,s_k}={a,b}}
 *       2^(1-bp_zeta[p]) (1 + bp_lambda[p] cos(t))^bp_zeta[p]
 *       exp(-bp_eta[q] (r_ij^2 + r_ik^2 + r_jk^2)) fc(r_ij) fc(r_ik) fc(r_jk),
 * with n_theta angle terms (bp_zeta integer in [1, 64], bp_lambda +1 or -1)
 * and n_rs_ang radius terms (bp_eta >= 0, 1/A^2); theta_s, eta_ang, rs_ang,
 * zeta and eps are then not read.  The radial part, layout and limits are
 * those above.  Every call below accepts either kind.
 */
enum { NN_DESC_MBP = 0, NN_DESC_BP = 1 };
typedef struct nn_mbp_params {
  int32_t n_species;
  double rc;
  int32_t n_rad;
  double eta_rad;
  const double* rs_rad;
  int32_t n_theta;
  const double* theta_s;
  int32_t n_rs_ang;
  double eta_ang;
  const double* rs_ang;
  double zeta;
  double eps;
  int32_t kind;             /* NN_DESC_MBP (0) or NN_DESC_BP (1)          */
  const double* bp_zeta;    /* [n_theta]  BP angle-term exponents          */
  const double* bp_lambda;  /* [n_theta]  BP angle-term signs              */
  const double* bp_eta;     /* [n_rs_ang] BP radius-term widths            */
} nn_mbp_params;

/*
 * Per-species MLP, Eq. (1): a^0 = G_i, z^l = W^l a^(l-1) + b^l,
 * a^l = act[l-1](z^l); the atomic energy is a^L (width[L] = 1, linear
 * output).  Weights are shared by all atoms of a species (Sec. II); each
 * species has its own depth and widths (Sec. II.A).
 *   W[l] [device] FP32 [width[l+1]][width[l]] row-major, b[l] [device] FP32.
 * Limits: 2 <= n_layers <= NN_MAX_LAYERS (one to three hidden layers),
 * hidden widths 1 .. 4096.  Models whose species all have two hidden layers
 * of the same widths (64,32), (128,128) or (256,128) run in a fused kernel
 * (FP32, or BF16 / split-BF16 with the MLP flags); every other model runs
 * layer by layer in FP32 (the BF16 flags then give NN_E_UNSUPPORTED).
 */
typedef struct nn_mlp {
  int32_t n_layers;
  int32_t width[NN_MAX_LAYERS + 1];
  int32_t act[NN_MAX_LAYERS];
  const float* W[NN_MAX_LAYERS];
  const float* b[NN_MAX_LAYERS];
} nn_mlp;

typedef struct nn_model {
  int32_t n_species;
  nn_mlp mlp[NN_MAX_SPECIES];
} nn_model;

/* Descriptor length D for these hyperparameters (see nn_mbp_params). Returns
 * -1 for invalid parameters. */
int64_t nn_descriptor_dim(const nn_mbp_params* p);

/*
 * Row length (floats) of the stored Jacobian: one row per list entry e =
 * (i -> j), js = 4 * ceil((n_rad + 3 + 3 * S * n_theta * n_rs_ang) / 4):
 *   [0, n_rad)   d/dr of the radial bins of species s_j (gradient = value * d/r);
 *   [n_rad, +3)  the unit vector d/r;
 *   then, for partner species b = 0 .. S-1, the angular block (s_j, b) as
 *   three component arrays x, y, z of dG_i/dd_e, each over the bins [q][p].
 *   Rows of entries at r >= rc are zero.
 */
int64_t nn_jacobian_stride(const nn_mbp_params* p);

/*
 * Derivative of every atom's descriptors along a displacement field v
 * [device] FP32 [N][3]:  U_i = sum_k (dG_i/dx_k) . v_k  [device] FP32 [N][D]
 * (the forward-mode product behind the weight gradient of a loss on forces,
 * Sec. II.A with forces as derivatives of the energy, Sec. II).  Computed in
 * FP32 from the same neighbor staging as nn_descriptors; entries at r >= rc
 * contribute nothing.  No workspace.  NN_E_INVALID for NULL buffers.
 */
nn_status nn_descriptor_tangent(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const float* v,
                                float* U, void* stream);

/*
 * Workspace bytes needed by every call below for a system of n_atoms atoms
 * and n_structs structures, a list of `capacity` entries, these descriptor
 * and model parameters (model may be NULL for list/descriptor-only use) and
 * these flags.  With NN_STORE_JACOBIAN the Jacobian is included only if it
 * fits mem_budget.
 */
nn_status nn_workspace_size(int64_t n_atoms, int32_t n_structs, int64_t capacity, const nn_mbp_params* p,
                            const nn_model* model, int32_t flags, size_t mem_budget, size_t* bytes);

/*
 * Number of list entries within `radius` (synchronous: enqueues the counting
 * pass on `stream`, waits, and returns the count in *nnz).  Used to size the
 * list before nn_build_neighbors.
 */
nn_status nn_count_neighbors(const nn_system* sys, double radius, int64_t* nnz, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * Build (or keep) the neighbor list at radius rc + skin (locality and cutoff,
 * Sec. I, III.A).  With skin > 0 and a previous build of this list, the list
 * is rebuilt only if some atom moved farther than skin/2 since that build;
 * the test and the rebuild run on the device, without a host round trip, so
 * the call can be captured in a HIP graph.  Structures of up to 256 atoms use
 * an all-pairs builder over every lattice image in range (any cell size);
 * larger ones use cell binning and need at least 3 bins along each periodic
 * direction (perpendicular width >= 3 (rc + skin)), else NN_E_CELL (device).
 * Capacity overflow sets NN_E_CAPACITY in meta (the list is then invalid and
 * meta[0] holds the required entries).
 */
nn_status nn_build_neighbors(const nn_system* sys, double rc, double skin, nn_nlist* nl, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Descriptors of every atom: G [device] FP32 [N][D] (layout of
 * nn_mbp_params).  Neighbor entries at r >= rc (skin lists) contribute
 * nothing.  If jac != NULL, also the stored Jacobian jac [device] FP32
 * [capacity][nn_jacobian_stride] (rows as documented there): the
 * derivatives the paper's precomputed-descriptor mode stores (Sec. II.A).
 */
nn_status nn_descriptors(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, float* G, float* jac,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Energies and forces (Sec. II: E = sum_i E_{s_i}(G_i); forces are the
 * negative derivatives of the energy):
 *   E_struct [device] FP64 [B]  per-structure energy, summed in FP64;
 *   E_atom   [device] FP32 [N]  atomic energies (may be NULL);
 *   F        [device] FP32 [N][3] forces F_k = -dE/dx_k (may be NULL).
 * Forces come from a hand-written adjoint: lambda_i = dE_i/dG_i by the MLP
 * backward pass, then per-pair vectors dE_i/dd_e by re-running the
 * descriptor's pair and triplet loops against lambda (or, with
 * NN_STORE_JACOBIAN and a Jacobian of capacity * nn_jacobian_stride * 4
 * bytes <= mem_budget, by contracting the Jacobian stored during the
 * descriptor pass, which later calls can reuse with NN_REUSE_DESCRIPTORS;
 * over the budget the call silently recomputes), then a deterministic gather
 * F_k = sum_e dE_k/dd_e - sum_e dE_{j(e)}/dd_rev(e).  G and lambda stay in
 * the workspace for nn_energy_forces_grad.
 */
nn_status nn_energy_forces(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                           const nn_model* model, int32_t flags, size_t mem_budget, double* E_struct,
                           float* E_atom, float* F, void* ws, size_t ws_bytes, void* stream);

/*
 * nn_energy_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and results (bitwise, for the same
 * flags and launch plan) without a caller workspace.  Its scratch (the
 * descriptors, dE/dG, per-pair gradients and species grouping of one call)
 * lives in a 64 MiB device array inside the library, one per GPU, held from
 * the library's load until the process ends.  Needs, in bytes, about
 * N * (8 D + 20) + 16 * nl->capacity + BF16 weight copies; inputs beyond
 * 64 MiB are rejected with NN_E_WORKSPACE before anything is enqueued (the
 * 4096-atom bulk cell of D = 96 takes about 8 MiB).  Every call on a GPU
 * shares that GPU's array and leaves its contents there; calls that overlap
 * on one GPU (several streams or threads at once) race and must be
 * serialized by the caller.  Nothing in the array needs to start at zero.
 * flags: MLP precision flags only (NN_STORE_JACOBIAN / NN_REUSE_DESCRIPTORS
 * give NN_E_INVALID).  Calls no allocating routine.
 */
nn_status nn_energy_forces_noalloc(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                   const nn_model* model, int32_t flags, double* E_struct, float* E_atom, float* F,
                                   void* stream);

/*
 * Launch tuning (the tiles of the batching step): times the launch variants
 * of this workload's passes -- waves per atom of the descriptor forward and
 * adjoint passes (1, 2, 4, or 0: the packed passes, four atoms of at most
 * 32 list entries per wave, mBP term) and waves per MLP tile (4, 8, or 1:
 * the row-block MLP, 64 atoms per block with the weights staged in LDS, for
 * widths (64, 32) and (128, 128) and D a multiple of 4 in FP32, of 8 in the
 * BF16 modes) -- on
 * `stream`, and keeps the fastest for workloads of the same shape class
 * (atom count within a factor of two, list entries per atom, descriptor
 * sizes, MLP widths and MLP mode) in a process-wide table that
 * nn_energy_forces and nn_energy_forces_grad then use; without an entry
 * they use fixed rules.  Needs a valid list (nn_build_neighbors) and the
 * nn_energy_forces workspace; overwrites the workspace's descriptors and
 * lambda.  Blocks until the timings are done, so it must not be called while
 * the stream is being captured into a graph.  A plan changes only the order
 * of some sums: results stay bitwise reproducible for a fixed table.
 * plan_out [host] (nullable) receives {waves/atom forward, waves/atom
 * adjoint, waves/MLP tile}.
 * Environment:
 *   NNPOT_PLAN="f,a,m" (f, a in {0, 1, 2, 4}; m in {1, 4, 8}) overrides every
 *     plan, tuned or default, while it is set: a way to run each launch
 *     variant in tests;
 *   NN_AUTOTUNE_CACHE=<file> keeps the table in a file across processes:
 *     read on the process's first lookup, rewritten (merged) after each
 *     nn_autotune.  One JSON object per line of an array,
 *       {"key": [n_log2, row4, S, n_theta, n_rs_ang, n_rad, h1, h2, mode],
 *        "plan": [f, a, m]}
 *     with n_log2 the bit length of the atom count, row4 =
 *     (ceil(capacity / atoms) + 2) / 4, h1, h2 the first two hidden widths of
 *     species 0 and mode 0 / 1 / 2 for FP32 / BF16 / split BF16.  Plans are
 *     tuned on one GPU model: keep one file per machine type.  Best effort:
 *     a file that cannot be read or written only costs speed.
 */
nn_status nn_autotune(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                      int32_t flags, void* ws, size_t ws_bytes, void* stream, int32_t* plan_out);

/* Forgets every plan in the process's table, including those read from
 * NN_AUTOTUNE_CACHE (the file is left as it is and not read again by this
 * process). */
void nn_autotune_reset(void);

/*
 * The launch plan nn_energy_forces would use for these arguments (NNPOT_PLAN,
 * else the table -- tuned or read from NN_AUTOTUNE_CACHE --, else the fixed
 * rules) into plan_out [host] [3].  Host only: reads no device memory and
 * enqueues nothing.  Errors: NN_E_INVALID / NN_E_UNSUPPORTED for arguments
 * nn_energy_forces would reject.
 */
nn_status nn_launch_plan(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                         int32_t flags, int32_t* plan_out);

/*
 * Backward of E_struct and F with respect to positions and weights, given
 * the upstream gradients of a loss L (Sec. II.A: the loss is minimised over
 * the MLP parameters; forces are derivatives of the energy, Sec. II, so a
 * loss on forces reaches the weights through second derivatives).  Must
 * follow nn_energy_forces with the same arguments and workspace (it reuses
 * G and the list).
 *   dL_dE   [device] FP64 [B] dL/dE_c (may be NULL if dL_dF is given: zero).
 *   dL_dF   [device] FP32 [N][3] dL/dF_k (may be NULL: no force term).  With
 *            it, sum_k dL_dF_k . F_k = -sum_i lambda_i . u_i, where u_i is
 *            the derivative of G_i along the displacement field dL_dF; the
 *            library computes u on the device (overwriting the workspace's
 *            lambda), runs the MLP together with its tangent along u, and
 *            adds the reverse pass of that tangent to the weight gradient.
 *            This part runs in FP32 whatever the MLP flags.
 *   dL_dpos [device] FP32 [N][3] (may be NULL): dL/dx_k = -dL_dE[c(k)] F_k;
 *            needs dL_dE and the F of that call.  Not provided together
 *            with dL_dF (NN_E_UNSUPPORTED): that would need the Hessian.
 *   dW, db [host] arrays of NN_MAX_SPECIES*NN_MAX_LAYERS device pointers
 *            (either array may be NULL): dW[s*NN_MAX_LAYERS + l] receives
 *            dL/dW^(l+1) of species s as FP32 in the layout of W[l], db the
 *            same for b.  Without dL_dF the MLP is re-run on the stored
 *            descriptors in the same precision mode (flags) to recover
 *            dE_i/dz^l; the sums over atoms use FP32 MFMA over fixed atom
 *            chunks reduced in chunk order (bitwise reproducible).
 * Errors: NN_E_INVALID for missing arguments, NN_E_WORKSPACE for a short
 * workspace, NN_E_UNSUPPORTED as above; nothing is enqueued then.
 */
nn_status nn_energy_forces_grad(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                const nn_model* model, int32_t flags, const double* dL_dE, const float* dL_dF,
                                const float* F, float* dL_dpos, float* const* dW, float* const* db, void* ws,
                                size_t ws_bytes, void* stream);

/*
 * Long-range charge equilibration (Sec. II.B).  The paper describes one
 * network per species with three outputs per atom -- the coefficients of a
 * second-order expansion of the atom's energy in its charge: local energy
 * E0, electronegativity chi and hardness J -- feeding a layer that returns
 * the charges and the total energy from a linear system, and defers the
 * theory to another work.  The reading computed here uses Gaussian charges
 * of a per-species width sigma:
 *   E(q) = sum_i [E0_i + chi_i q_i + J_i q_i^2 / 2]
 *          + coulomb [ sum_i q_i^2 / (2 sigma_i sqrt(pi))
 *                      + sum_{i<j} q_i q_j erf(r_ij / (sqrt(2) gamma_ij)) / r_ij ],
 *   gamma_ij^2 = sigma_i^2 + sigma_j^2,
 * minimised over the charges of each structure subject to sum_i q_i = Q_c:
 * every atom ends at the same chemical potential, and the energy is
 * sum E0 + chi.q / 2 + mu Q_c / 2 (mu the chemical potential).  Forces are the
 * derivatives at fixed charges (the minimum makes the derivative of the solve
 * vanish): the network part through the descriptor adjoint with output seeds
 * (1, q_i, q_i^2 / 2), plus the Coulomb pair forces.
 */
typedef struct nn_qeq_params {
  const double* sigma; /* [host] [S] Gaussian charge width of each species (> 0), Angstrom */
  double coulomb;      /* e^2 / (4 pi eps0) in the energy and length units used: 14.399645 eV A */
} nn_qeq_params;

/*
 * Energies, charges and forces with charge equilibration.  Every species'
 * network must have output width 3 (E0, chi, J in that order; FP32, layer by
 * layer).  Structures must be non-periodic with at most 64 atoms each (the
 * per-structure FP64 Cholesky solve runs on chip); a structure outside that,
 * or whose matrix is not positive definite, is reported by nn_check
 * (NN_E_DEVICE) and gets zero charges and energy.
 *   total_charge [device] FP64 [B]  total charge Q_c of each structure (e);
 *   E_struct     [device] FP64 [B]  total energies;
 *   charges      [device] FP64 [N]  equilibrated charges (may be NULL);
 *   F            [device] FP32 [N][3] forces (may be NULL).
 * The workspace is that of nn_workspace_size with this model.
 */
nn_status nn_energy_forces_qeq(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                               const nn_model* model, const nn_qeq_params* qp, const double* total_charge,
                               double* E_struct, double* charges, float* F, void* ws, size_t ws_bytes,
                               void* stream);

/*
 * Weight gradient of a loss on the energies of nn_energy_forces_qeq (which it
 * must follow with the same arguments and workspace): with dL_dE [device]
 * FP64 [B], dL/dtheta = sum_c dL_dE_c sum_{i in c} d(E0_i + chi_i q_i +
 * J_i q_i^2 / 2)/dtheta at the equilibrated charges (the derivative of the
 * charges drops out at the minimum).  dW, db as for nn_energy_forces_grad.
 */
nn_status nn_energy_forces_qeq_grad(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                    const nn_model* model, const double* dL_dE, float* const* dW,
                                    float* const* db, void* ws, size_t ws_bytes, void* stream);

/* Loss of Sec. II.A: energy and force terms with a relative weight. */
enum { NN_LOSS_QUAD = 0, NN_LOSS_EXP = 1 };
typedef struct {
  int32_t energy_kind;  /* NN_LOSS_QUAD: x^2;  NN_LOSS_EXP: exp(x^2) - 1    */
  int32_t force_kind;   /* the same choice for the force components         */
  int32_t per_atom;     /* 1: the energy difference of a structure divided by
                           its atom count (per-atom energies), 0: per structure */
  double energy_weight; /* w_E                                               */
  double force_weight;  /* w_F (the relative factor of the force term)        */
} nn_loss_params;

/*
 * L = w_E / B sum_c l_E(dE_c) + w_F / (3N) sum_{k,a} l_F(F_ka - F_ref_ka), with
 * dE_c = E_c - E_ref_c (per structure) or (E_c - E_ref_c) / N_c (per atom),
 * and its derivatives, the inputs of nn_energy_forces_grad.
 *   E, E_ref [device] FP64 [B];  F, F_ref [device] FP32 [N][3] (both NULL: no
 *   force term, dL_dF not written);  L [device] FP64 [1];  dL_dE [device] FP64
 *   [B];  dL_dF [device] FP32 [N][3].
 * Sums are FP64 over fixed blocks added in block order (bitwise
 * reproducible).  Uses the workspace of nn_energy_forces.
 */
nn_status nn_loss(const nn_system* sys, const nn_loss_params* lp, const double* E, const double* E_ref,
                  const float* F, const float* F_ref, double* L, double* dL_dE, float* dL_dF, void* ws,
                  size_t ws_bytes, void* stream);

/* Langevin dynamics parameters (units: Angstrom, fs, eV, amu). */
typedef struct {
  double dt;       /* time step, fs (> 0)                                   */
  double friction; /* gamma, 1/fs (>= 0); 0 gives velocity Verlet (constant energy) */
  double kT;       /* thermal energy, eV (>= 0)                             */
} nn_langevin;

/*
 * n_steps steps of Langevin dynamics on the potential: the repeated
 * evaluation of Table II (Sec. III.B), integrated with the BAOAB splitting
 * (Leimkuhler and Matthews 2013):  B v += dt/2 F/m;  A x += dt/2 v;
 * O v = c1 v + c2 sqrt(kT/m) xi with c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2);
 * A x += dt/2 v;  list update (nn_build_neighbors with rc, skin: rebuilt on
 * the device only when an atom moved farther than skin/2) and
 * nn_energy_forces at the new x;  B v += dt/2 F/m.
 *   pos      [device] FP64 [N][3], the buffer sys->pos points at (advanced in
 *            place; NN_E_INVALID if pos != sys->pos).
 *   vel      [device] FP64 [N][3] in/out, Angstrom/fs.
 *   inv_mass [device] FP64 [N], 1/amu.
 *   noise    [device] FP32 [n_steps][N][3] standard normal draws xi (the
 *            caller's generator); may be NULL when friction == 0.
 *   E_pot    [device] FP64 [n_steps][B]: the energies after each step.
 *   F        [device] FP32 [N][3] in/out: on entry the forces at pos (as
 *            left by nn_energy_forces or the previous call), on exit those
 *            at the final positions.
 *   flags    MLP precision flags of nn_energy_forces (no stored Jacobian).
 * nl, ws as for nn_build_neighbors / nn_energy_forces (a skin > 0 needs
 * nl->ref_pos).  Everything is enqueued on `stream` with no host round
 * trip, so a whole call can be captured in a HIP graph.  Device-side errors
 * (list capacity, ...) are reported by nn_check; after a capacity overflow
 * the forces of the following steps are zero.
 */
nn_status nn_md_langevin(const nn_system* sys, double* pos, double* vel, const double* inv_mass, nn_nlist* nl,
                         double rc, double skin, const nn_mbp_params* p, const nn_model* model, int32_t flags,
                         const nn_langevin* lp, const float* noise, int32_t n_steps, double* E_pot, float* F,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Synchronize `stream` and report device-side errors recorded in the list's
 * metadata since the last check (then clear them).  *info (may be NULL)
 * receives the required list size for NN_E_CAPACITY.
 */
nn_status nn_check(const nn_nlist* nl, void* stream, int64_t* info);

/* Message for the last non-NN_OK status returned on this thread. */
const char* nn_last_error(void);

/*
 * Stage timing (a tracing aid, off by default).  While enabled, every stage
 * the calls above enqueue is bracketed by two HIP events recorded on the
 * caller's stream (do not enable it while capturing a graph).
 * nn_timing_read synchronizes those events and returns, per stage, the
 * summed elapsed milliseconds and the number of launches since the last
 * nn_timing(1); both arrays [host] have NN_STAGE_COUNT entries.
 */
enum {
  NN_STAGE_NEIGHBORS = 0,   /* skin test + list (re)build                   */
  NN_STAGE_SPECIES = 1,     /* grouping of atoms by species                  */
  NN_STAGE_WEIGHTS = 2,     /* BF16 weight copies                            */
  NN_STAGE_DESC_FWD = 3,    /* radial + angular descriptors                  */
  NN_STAGE_MLP = 4,         /* per-species MLP forward + backward            */
  NN_STAGE_ENERGY = 5,      /* per-structure FP64 energy (energy-only calls)  */
  NN_STAGE_DESC_ADJ = 6,    /* descriptor adjoint: per-pair gradients        */
  NN_STAGE_FORCE_GATHER = 7,/* per-atom forces from per-pair gradients, and
                             * the FP64 energy sums when forces are asked for */
  NN_STAGE_DESC_JAC = 8,    /* stored Jacobian of the descriptors            */
  NN_STAGE_JAC_CONTRACT = 9,/* per-pair gradients from the stored Jacobian   */
  NN_STAGE_COUNT = 10
};
nn_status nn_timing(int32_t enable);
nn_status nn_timing_read(double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* NNPOT_H */
