/*
 * nnref.c -- plain FP64 CPU oracle for the mBP + per-species MLP energy/force path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference against which the HIP
 * path is checked.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never calls it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything here is the plain definition evaluated directly, in double
 * precision, built with -ffp-contract=off and without fast-math:
 *   - neighbor sets by brute force over atoms and lattice images, plus a
 *     cell-binned variant that only pre-filters candidates (pinned to the
 *     brute force by the tests);
 *   - radial and angular mBP descriptors as direct sums over neighbors and
 *     unordered neighbor pairs, with analytic derivatives;
 *   - the dense per-species MLP of Eq. (1) and its backward pass;
 *   - forces F = -dE/dx by the chain rule, and the weight gradient of a
 *     loss on energies and forces (the force part by forward mode through
 *     the MLP along the descriptor tangent, then reverse mode).
 *
 * Sources (PANNA 2.0 paper):
 *   - total energy as a sum of atomic terms, weights shared per species:
 *     Sec. II (opening) and Sec. I (locality, invariance);
 *   - precomputed vs on-the-fly descriptors, derivatives needed for forces:
 *     Sec. II.A;
 *   - mBP descriptor with radial bins, and angular bins over the average
 *     radius and the angle, split by species: Sec. III.A, Sec. III.B;
 *   - MLP layer equation: Sec. II.A, Eq. (1); Gaussian / ReLU / tanh /
 *     linear activations: Sec. II.A;
 *   - loss on energies per configuration, and on forces with a relative
 *     weight: Sec. II.A, Sec. III.A.
 * The paper does not print the mBP formulas (it defers to the first PANNA
 * paper).  The functional form used here is the reading stated in the
 * design notes: ANI-style radial Gaussians times a cosine cutoff, and an
 * angular term 2 * x^zeta * exp(-eta (r_avg - Rs)^2) * fc * fc with
 * x = (1 + cos(theta) cos(theta_s) + sqrt(sin^2(theta) + eps) sin(theta_s))
 *     / (1 + sqrt(1 + eps)),
 * summed over unordered neighbor pairs.  At eps = 0 this is the published
 * ANI modified angular function 2^(1-zeta) (1 + cos(theta - theta_s))^zeta.
 * The standard BP angular term (Sec. II.A names both; Behler and Parrinello's
 * definition) is also provided: for every ordered pair of neighbors (j, k),
 * 2^(1-zeta_p) (1 + lambda_p cos(theta))^zeta_p
 *   exp(-eta_q (r_ij^2 + r_ik^2 + r_jk^2)) fc(r_ij) fc(r_ik) fc(r_jk).
 * Numerical identity with PANNA's own code is parity unpinned (no PANNA
 * code or data is available); every other function below is pinned by the
 * CPU tests (closed forms, invariances, finite differences, brute force,
 * textbook MLP).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_MAX_SPECIES 16
#define REF_MAX_LAYERS 8

/* ------------------------------------------------------------------------ */
/* Data passed in from Python (ctypes mirrors these layouts).                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n_atoms;
    int32_t n_structs;
    const double *pos;       /* [N][3] Cartesian, Angstrom                   */
    const int32_t *species;  /* [N] in [0, S)                                */
    const int64_t *atom_ptr; /* [B+1] structure c owns atoms [ptr[c],ptr[c+1]) */
    const double *cell;      /* [B][3][3], rows are lattice vectors a, b, c  */
    const uint8_t *pbc;      /* [B][3] periodic flag per lattice direction   */
} ref_system;

typedef struct {
    int64_t n_rows;          /* rows of the list                               */
    const int64_t *rows;     /* atom index of each row (NULL: row r = atom r)  */
    const int64_t *offsets;  /* [n_rows+1]                                     */
    const int32_t *nbr;      /* [nnz] neighbor atom index                      */
    const int32_t *shift;    /* [nnz][3] lattice image (n_a, n_b, n_c)         */
} ref_nlist;

typedef struct {
    int32_t n_species;
    double rc;
    int32_t n_rad;
    double eta_rad;
    const double *rs_rad;    /* [n_rad]    */
    int32_t n_theta;
    const double *theta_s;   /* [n_theta]  */
    int32_t n_rs_ang;
    double eta_ang;
    const double *rs_ang;    /* [n_rs_ang] */
    double zeta;
    double eps;
    int32_t kind;            /* 0: mBP angular term; 1: standard BP angular term */
    const double *bp_zeta;   /* [n_theta]  BP: exponent of angle term p        */
    const double *bp_lambda; /* [n_theta]  BP: +1 or -1                        */
    const double *bp_eta;    /* [n_rs_ang] BP: width of radius term q, 1/A^2   */
} ref_params;

/* Per-species dense MLP.  arch[s*(REF_MAX_LAYERS+1) + l] = width of layer l
 * (layer 0 = descriptor), n_layers[s] = number of weight layers L.  act[s*
 * REF_MAX_LAYERS + l] = activation code of weight layer l+1.  The parameters of
 * species s start at params + poff[s] and are W1, b1, W2, b2, ... with W_l
 * stored row-major [width[l]][width[l-1]].                                   */
typedef struct {
    int32_t n_species;
    const int32_t *n_layers;
    const int32_t *arch;
    const int32_t *act;
    const double *params;
    const int64_t *poff;
} ref_model;

enum { ACT_LINEAR = 0, ACT_GAUSSIAN = 1, ACT_RELU = 2, ACT_TANH = 3 };

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------ */

/* Inverse of the 3x3 cell matrix H (rows a, b, c), so that the fractional
 * coordinates of a Cartesian row vector x are s = x H^-1.                   */
static void inverse3(const double h[9], double inv[9]) {
    double c00 = h[4] * h[8] - h[5] * h[7];
    double c01 = h[5] * h[6] - h[3] * h[8];
    double c02 = h[3] * h[7] - h[4] * h[6];
    double det = h[0] * c00 + h[1] * c01 + h[2] * c02;
    inv[0] = c00 / det;
    inv[1] = (h[2] * h[7] - h[1] * h[8]) / det;
    inv[2] = (h[1] * h[5] - h[2] * h[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (h[0] * h[8] - h[2] * h[6]) / det;
    inv[5] = (h[2] * h[3] - h[0] * h[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (h[1] * h[6] - h[0] * h[7]) / det;
    inv[8] = (h[0] * h[4] - h[1] * h[3]) / det;
}

static void frac_coords(const double inv[9], const double x[3], double s[3]) {
    for (int d = 0; d < 3; ++d) s[d] = x[0] * inv[0 + d] + x[1] * inv[3 + d] + x[2] * inv[6 + d];
}

/* Perpendicular width of the cell along each lattice direction:
 * w_a = V / |b x c| and cyclically.                                         */
static void perp_widths(const double h[9], double w[3]) {
    const double *a = h, *b = h + 3, *c = h + 6;
    double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double vol = fabs(a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]);
    w[0] = vol / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    w[1] = vol / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
    w[2] = vol / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
}

/* Displacement from atom i to the image n of atom j:
 *   d = (x_j - x_i) + (n_a a + n_b b + n_c c),
 * evaluated in exactly this order (image vector accumulated a, b, then c;
 * then added to the difference of positions).  This fixed order is the
 * definition of the neighbor inclusion test, r^2 = (dx dx + dy dy) + dz dz,
 * strictly below cutoff^2.                                                  */
static void displacement(const double *xi, const double *xj, const double h[9], const int n[3],
                         double d[3]) {
    for (int k = 0; k < 3; ++k) {
        double t = (double)n[0] * h[0 + k];
        t = t + (double)n[1] * h[3 + k];
        t = t + (double)n[2] * h[6 + k];
        d[k] = (xj[k] - xi[k]) + t;
    }
}

static double norm2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

static int struct_of_atom(const ref_system *sys, int64_t i) {
    int lo = 0, hi = sys->n_structs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (sys->atom_ptr[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Neighbor sets (locality and cutoff: Sec. I, Sec. III.A)                    */
/* ------------------------------------------------------------------------ */

/* Range of lattice images that can hold a neighbor.  For a periodic
 * direction with perpendicular width w and fractional coordinates spread
 * over an interval of length `spread`, a displacement shorter than the
 * cutoff needs |n| < cutoff / w + spread, so |n| <= floor(cutoff/w + spread)
 * + 1 is a safe bound; `extra` widens it further (the tests use this to show
 * that the bound is not binding).                                           */
static void image_bounds(const ref_system *sys, int c, double cutoff, int extra, int K[3]) {
    const double *h = sys->cell + 9 * (int64_t)c;
    double inv[9], w[3], lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    inverse3(h, inv);
    perp_widths(h, w);
    for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a) {
        double s[3];
        frac_coords(inv, sys->pos + 3 * a, s);
        for (int d = 0; d < 3; ++d) {
            if (s[d] < lo[d]) lo[d] = s[d];
            if (s[d] > hi[d]) hi[d] = s[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        if (sys->pbc[3 * c + d]) K[d] = (int)floor(cutoff / w[d] + (hi[d] - lo[d])) + 1 + extra;
        else K[d] = 0;
    }
}

/* Brute force: for the atom of each requested row, every atom j of the same
 * structure and every lattice image n in range, keep (j, n) != (i, 0) when
 * |d|^2 < cutoff^2.  Entries of a row come out sorted by (j, n_a, n_b, n_c).
 * Returns the total number of entries; when nbr == NULL only counts (and
 * fills offsets).  Entries are written only if the total fits in cap.       */
int64_t nnref_neighbors_brute(const ref_system *sys, double cutoff, int extra_images,
                              const int64_t *rows, int64_t n_rows, int64_t cap,
                              int64_t *offsets, int32_t *nbr, int32_t *shift) {
    const double cut2 = cutoff * cutoff;
    int (*K)[3] = malloc(sizeof(int[3]) * (size_t)(sys->n_structs > 0 ? sys->n_structs : 1));
    for (int c = 0; c < sys->n_structs; ++c) image_bounds(sys, c, cutoff, extra_images, K[c]);
    int64_t *count = calloc((size_t)n_rows + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t i = rows ? rows[r] : r;
            int c = struct_of_atom(sys, i);
            const double *h = sys->cell + 9 * (int64_t)c;
            int64_t out = pass ? offsets[r] : 0;
            for (int64_t j = sys->atom_ptr[c]; j < sys->atom_ptr[c + 1]; ++j) {
                int n[3];
                for (n[0] = -K[c][0]; n[0] <= K[c][0]; ++n[0])
                    for (n[1] = -K[c][1]; n[1] <= K[c][1]; ++n[1])
                        for (n[2] = -K[c][2]; n[2] <= K[c][2]; ++n[2]) {
                            if (j == i && n[0] == 0 && n[1] == 0 && n[2] == 0) continue;
                            double d[3];
                            displacement(sys->pos + 3 * i, sys->pos + 3 * j, h, n, d);
                            if (!(norm2(d) < cut2)) continue;
                            if (pass == 0) {
                                count[r]++;
                            } else {
                                nbr[out] = (int32_t)j;
                                shift[3 * out + 0] = n[0];
                                shift[3 * out + 1] = n[1];
                                shift[3 * out + 2] = n[2];
                                out++;
                            }
                        }
            }
        }
        if (pass == 0) {
            offsets[0] = 0;
            for (int64_t r = 0; r < n_rows; ++r) offsets[r + 1] = offsets[r] + count[r];
            if (nbr == NULL || offsets[n_rows] > cap) break;
        }
    }
    int64_t total = offsets[n_rows];
    free(count);
    free(K);
    return total;
}

/* Entry order inside a row: by neighbor index, then image (lexicographic). */
static int entry_less(int32_t ja, const int32_t *sa, int32_t jb, const int32_t *sb) {
    if (ja != jb) return ja < jb;
    for (int d = 0; d < 3; ++d)
        if (sa[d] != sb[d]) return sa[d] < sb[d];
    return 0;
}

/* Cell-binned variant of the same set, for systems too large for the brute
 * force.  It only chooses which (j, n) candidates to test: atoms are binned
 * by wrapped fractional coordinates into bins at least `cutoff` wide (by a
 * relative margin of 1e-6), so every pair closer than the cutoff lies in
 * the same or an adjacent bin.  Each candidate then goes through the same
 * inclusion test as the brute force, and every row is sorted the same way.
 * Structures whose periodic directions hold fewer than 3 bins fall back to
 * the brute force.                                                          */
int64_t nnref_neighbors_cells(const ref_system *sys, double cutoff, const int64_t *rows,
                              int64_t n_rows, int64_t cap, int64_t *offsets, int32_t *nbr,
                              int32_t *shift) {
    const double cut2 = cutoff * cutoff;
    const int64_t N = sys->n_atoms;
    int B = sys->n_structs;
    /* per-structure binning */
    int (*nb)[3] = malloc(sizeof(int[3]) * (size_t)(B > 0 ? B : 1));
    int *brute = malloc(sizeof(int) * (size_t)(B > 0 ? B : 1));
    int64_t *bin_base = malloc(sizeof(int64_t) * (size_t)(B + 1));
    int (*Kb)[3] = malloc(sizeof(int[3]) * (size_t)(B > 0 ? B : 1));
    bin_base[0] = 0;
    for (int c = 0; c < B; ++c) {
        const double *h = sys->cell + 9 * (int64_t)c;
        double w[3];
        perp_widths(h, w);
        brute[c] = 0;
        for (int d = 0; d < 3; ++d) {
            int k = (int)floor(w[d] / (cutoff * (1.0 + 1e-6)));
            if (k < 1) k = 1;
            nb[c][d] = k;
            if (sys->pbc[3 * c + d] && k < 3) brute[c] = 1;
        }
        if (brute[c]) {
            nb[c][0] = nb[c][1] = nb[c][2] = 1;
            image_bounds(sys, c, cutoff, 0, Kb[c]);
        }
        bin_base[c + 1] = bin_base[c] + (int64_t)nb[c][0] * nb[c][1] * nb[c][2];
    }
    int64_t nbins = bin_base[B];
    int32_t *bin_of = malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1) * 4); /* bin, m_a, m_b, m_c */
    int64_t *bin_start = calloc((size_t)nbins + 1, sizeof(int64_t));
    int64_t *bin_atoms = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int (*bcoord)[3] = malloc(sizeof(int[3]) * (size_t)(N > 0 ? N : 1));
    for (int c = 0; c < B; ++c) {
        const double *h = sys->cell + 9 * (int64_t)c;
        double inv[9];
        inverse3(h, inv);
        for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a) {
            double s[3];
            frac_coords(inv, sys->pos + 3 * a, s);
            int b3[3], m[3];
            for (int d = 0; d < 3; ++d) {
                double t = s[d];
                m[d] = 0;
                if (sys->pbc[3 * c + d]) {
                    m[d] = (int)floor(t);
                    t = t - m[d];
                }
                int k = (int)floor(t * nb[c][d]);
                if (k < 0) k = 0;
                if (k > nb[c][d] - 1) k = nb[c][d] - 1;
                b3[d] = k;
            }
            bcoord[a][0] = b3[0];
            bcoord[a][1] = b3[1];
            bcoord[a][2] = b3[2];
            int64_t bin = bin_base[c] + ((int64_t)b3[0] * nb[c][1] + b3[1]) * nb[c][2] + b3[2];
            bin_of[4 * a + 0] = (int32_t)bin;
            bin_of[4 * a + 1] = m[0];
            bin_of[4 * a + 2] = m[1];
            bin_of[4 * a + 3] = m[2];
            bin_start[bin + 1]++;
        }
    }
    for (int64_t b = 0; b < nbins; ++b) bin_start[b + 1] += bin_start[b];
    {
        int64_t *fill = malloc(sizeof(int64_t) * (size_t)(nbins > 0 ? nbins : 1));
        for (int64_t b = 0; b < nbins; ++b) fill[b] = bin_start[b];
        for (int64_t a = 0; a < N; ++a) bin_atoms[fill[bin_of[4 * a]]++] = a;
        free(fill);
    }
    int64_t *count = calloc((size_t)n_rows + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rows; ++r) {
            int64_t i = rows ? rows[r] : r;
            int c = struct_of_atom(sys, i);
            const double *h = sys->cell + 9 * (int64_t)c;
            int64_t out = pass ? offsets[r] : 0;
            int64_t row_begin = out;
            if (brute[c]) {
                for (int64_t j = sys->atom_ptr[c]; j < sys->atom_ptr[c + 1]; ++j) {
                    int n[3];
                    for (n[0] = -Kb[c][0]; n[0] <= Kb[c][0]; ++n[0])
                        for (n[1] = -Kb[c][1]; n[1] <= Kb[c][1]; ++n[1])
                            for (n[2] = -Kb[c][2]; n[2] <= Kb[c][2]; ++n[2]) {
                                if (j == i && n[0] == 0 && n[1] == 0 && n[2] == 0) continue;
                                double d[3];
                                displacement(sys->pos + 3 * i, sys->pos + 3 * j, h, n, d);
                                if (!(norm2(d) < cut2)) continue;
                                if (pass == 0) count[r]++;
                                else {
                                    nbr[out] = (int32_t)j;
                                    shift[3 * out + 0] = n[0];
                                    shift[3 * out + 1] = n[1];
                                    shift[3 * out + 2] = n[2];
                                    out++;
                                }
                            }
                }
                continue; /* brute-force rows are already sorted */
            }
            int di[3];
            for (di[0] = -1; di[0] <= 1; ++di[0])
                for (di[1] = -1; di[1] <= 1; ++di[1])
                    for (di[2] = -1; di[2] <= 1; ++di[2]) {
                        int bb[3], wrap[3], skip = 0;
                        for (int d = 0; d < 3; ++d) {
                            int k = bcoord[i][d] + di[d];
                            wrap[d] = 0;
                            if (k < 0 || k >= nb[c][d]) {
                                if (!sys->pbc[3 * c + d]) { skip = 1; break; }
                                wrap[d] = k < 0 ? -1 : 1;
                                k -= wrap[d] * nb[c][d];
                            }
                            bb[d] = k;
                        }
                        if (skip) continue;
                        int64_t bin = bin_base[c] + ((int64_t)bb[0] * nb[c][1] + bb[1]) * nb[c][2] + bb[2];
                        for (int64_t t = bin_start[bin]; t < bin_start[bin + 1]; ++t) {
                            int64_t j = bin_atoms[t];
                            int n[3];
                            for (int d = 0; d < 3; ++d)
                                n[d] = sys->pbc[3 * c + d] ? wrap[d] + bin_of[4 * i + 1 + d] - bin_of[4 * j + 1 + d] : 0;
                            if (j == i && n[0] == 0 && n[1] == 0 && n[2] == 0) continue;
                            double d[3];
                            displacement(sys->pos + 3 * i, sys->pos + 3 * j, h, n, d);
                            if (!(norm2(d) < cut2)) continue;
                            if (pass == 0) count[r]++;
                            else {
                                nbr[out] = (int32_t)j;
                                shift[3 * out + 0] = n[0];
                                shift[3 * out + 1] = n[1];
                                shift[3 * out + 2] = n[2];
                                out++;
                            }
                        }
                    }
            if (pass == 1) {
                /* insertion sort of the row by (j, n) */
                for (int64_t a = row_begin + 1; a < out; ++a) {
                    int32_t jj = nbr[a], ss[3] = {shift[3 * a], shift[3 * a + 1], shift[3 * a + 2]};
                    int64_t b = a;
                    while (b > row_begin && entry_less(jj, ss, nbr[b - 1], shift + 3 * (b - 1))) {
                        nbr[b] = nbr[b - 1];
                        memcpy(shift + 3 * b, shift + 3 * (b - 1), 3 * sizeof(int32_t));
                        --b;
                    }
                    nbr[b] = jj;
                    memcpy(shift + 3 * b, ss, 3 * sizeof(int32_t));
                }
            }
        }
        if (pass == 0) {
            offsets[0] = 0;
            for (int64_t r = 0; r < n_rows; ++r) offsets[r + 1] = offsets[r] + count[r];
            if (nbr == NULL || offsets[n_rows] > cap) break;
        }
    }
    int64_t total = offsets[n_rows];
    free(count);
    free(bcoord);
    free(bin_atoms);
    free(bin_start);
    free(bin_of);
    free(Kb);
    free(bin_base);
    free(brute);
    free(nb);
    return total;
}

/* ------------------------------------------------------------------------ */
/* mBP descriptor (Sec. II.A; bin layout Sec. III.A / III.B)                  */
/* ------------------------------------------------------------------------ */

/* Descriptor length: n_rad radial bins per neighbor species, then
 * n_theta * n_rs_ang angular bins per unordered species pair.  This gives
 * 240/456/736 for 2/3/4 species with 24 radial and 8x8 angular bins
 * (Sec. III.A) and 152 for one species with 24 + 8x16 (Sec. III.B).        */
int64_t nnref_descriptor_dim(int32_t S, int32_t n_rad, int32_t n_theta, int32_t n_rs_ang) {
    return (int64_t)n_rad * S + (int64_t)n_theta * n_rs_ang * S * (S + 1) / 2;
}

/* Offset of the angular block of the unordered species pair (a, b), a <= b:
 * blocks are ordered (0,0), (0,1), ..., (0,S-1), (1,1), ..., (S-1,S-1).   */
static int64_t pair_block(int S, int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    return (int64_t)a * S - (int64_t)a * (a - 1) / 2 + (b - a);
}

/* Cosine cutoff fc(r) = (1 + cos(pi r / rc)) / 2 for r < rc, else 0, written
 * as sin^2(pi (rc - r) / (2 rc)); and its derivative d fc / d r.          */
static double cutoff_fn(double r, double rc) {
    if (r >= rc) return 0.0;
    double s = sin(M_PI * (rc - r) / (2.0 * rc));
    return s * s;
}
static double cutoff_deriv(double r, double rc) {
    if (r >= rc) return 0.0;
    return -0.5 * M_PI / rc * sin(M_PI * r / rc);
}

/* Standard BP angular part of one atom (kind 1), added to G (and dG, same
 * layout as atom_descriptor): bin (q, p) of the species pair block of (e, f)
 * sums, over every ordered pair of distinct neighbors e, f inside rc,
 *   T = 2^(1 - zeta_p) (1 + lambda_p cos(theta))^zeta_p
 *       exp(-eta_q (r_e^2 + r_f^2 + r_ef^2)) fc(r_e) fc(r_f) fc(r_ef),
 * with r_ef = |d_f - d_e|.                                                   */
static void bp_angular(const ref_params *P, int64_t n_e, const double (*d)[3], const int32_t *sp,
                       const double *r, double *G, double *dG) {
    const int S = P->n_species;
    const int64_t ang0 = (int64_t)P->n_rad * S;
    const int64_t nbins = (int64_t)P->n_theta * P->n_rs_ang;
    const double rc = P->rc;
    for (int64_t e = 0; e < n_e; ++e) {
        if (!(r[e] < rc)) continue;
        for (int64_t f = 0; f < n_e; ++f) {
            if (f == e || !(r[f] < rc)) continue;
            const double *u = d[e], *v = d[f];
            const double ru = r[e], rv = r[f];
            const double w[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};  /* d_f - d_e */
            const double rw = sqrt(norm2(w));
            double uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
            double cos_t = uv / (ru * rv);
            double s2 = ru * ru + rv * rv + rw * rw;
            double fu = cutoff_fn(ru, rc), fv = cutoff_fn(rv, rc), fw = cutoff_fn(rw, rc);
            double dfu = cutoff_deriv(ru, rc), dfv = cutoff_deriv(rv, rc), dfw = cutoff_deriv(rw, rc);
            double F = fu * fv * fw;
            int64_t blk = ang0 + pair_block(S, sp[e], sp[f]) * nbins;
            /* gradients of cos(theta), s2 and F with respect to d_e and d_f */
            double dcos_du[3], dcos_dv[3], ds2_du[3], ds2_dv[3], dF_du[3], dF_dv[3];
            for (int c = 0; c < 3; ++c) {
                dcos_du[c] = v[c] / (ru * rv) - cos_t * u[c] / (ru * ru);
                dcos_dv[c] = u[c] / (ru * rv) - cos_t * v[c] / (rv * rv);
                ds2_du[c] = 2.0 * u[c] - 2.0 * w[c];
                ds2_dv[c] = 2.0 * v[c] + 2.0 * w[c];
                double dw_term = (rw > 0.0) ? fu * fv * dfw * w[c] / rw : 0.0;
                dF_du[c] = dfu * u[c] / ru * fv * fw - dw_term;
                dF_dv[c] = fu * dfv * v[c] / rv * fw + dw_term;
            }
            for (int q = 0; q < P->n_rs_ang; ++q) {
                double R = exp(-P->bp_eta[q] * s2);
                double dR_ds2 = -P->bp_eta[q] * R;
                for (int p = 0; p < P->n_theta; ++p) {
                    double z = P->bp_zeta[p], lam = P->bp_lambda[p];
                    double base = 1.0 + lam * cos_t;
                    double A = pow(2.0, 1.0 - z) * pow(base, z);
                    int64_t idx = blk + (int64_t)q * P->n_theta + p;
                    G[idx] += A * R * F;
                    if (dG) {
                        double dA_dcos = pow(2.0, 1.0 - z) * z * lam * pow(base, z - 1.0);
                        for (int c = 0; c < 3; ++c) {
                            dG[(idx * n_e + e) * 3 + c] +=
                                dA_dcos * dcos_du[c] * R * F + A * dR_ds2 * ds2_du[c] * F + A * R * dF_du[c];
                            dG[(idx * n_e + f) * 3 + c] +=
                                dA_dcos * dcos_dv[c] * R * F + A * dR_ds2 * ds2_dv[c] * F + A * R * dF_dv[c];
                        }
                    }
                }
            }
        }
    }
}

/* Descriptor of one atom from its neighbor displacements d[e] (only entries
 * with r < rc contribute) and neighbor species sp[e].  Writes G[D]; when
 * dG != NULL also writes dG[(d * n_e + e) * 3 + k] = dG_d / d(d_e)_k.
 *
 * Radial bin (s, k):   sum over neighbors e of species s of
 *                      exp(-eta_rad (r_e - Rs_k)^2) fc(r_e).
 * Angular bin (p(a,b), q, p): sum over unordered pairs {e, f} with sorted
 *                      species (a, b) of
 *                      2 x_p^zeta exp(-eta_ang ((r_e + r_f)/2 - Rs'_q)^2)
 *                      fc(r_e) fc(r_f),
 *                      x_p = (1 + cos(theta) cos(ts_p) + sqrt(sin^2(theta)
 *                      + eps) sin(ts_p)) / (1 + sqrt(1 + eps)),
 *                      cos(theta) = d_e.d_f / (r_e r_f),
 *                      sin^2(theta) = |d_e x d_f|^2 / (r_e^2 r_f^2).
 * Within an angular block the bins are ordered [q][p] with p fastest.      */
static void atom_descriptor(const ref_params *P, int64_t n_e, const double (*d)[3],
                            const int32_t *sp, double *G, double *dG) {
    const int S = P->n_species;
    const int64_t D = nnref_descriptor_dim(S, P->n_rad, P->n_theta, P->n_rs_ang);
    const int64_t ang0 = (int64_t)P->n_rad * S;
    const int64_t nbins = (int64_t)P->n_theta * P->n_rs_ang;
    const double rc = P->rc;
    memset(G, 0, sizeof(double) * (size_t)D);
    if (dG) memset(dG, 0, sizeof(double) * (size_t)(D * n_e * 3));
    double *r = malloc(sizeof(double) * (size_t)(n_e > 0 ? n_e : 1));
    for (int64_t e = 0; e < n_e; ++e) r[e] = sqrt(norm2(d[e]));

    /* radial part */
    for (int64_t e = 0; e < n_e; ++e) {
        if (!(r[e] < rc)) continue;
        double fc = cutoff_fn(r[e], rc), dfc = cutoff_deriv(r[e], rc);
        for (int k = 0; k < P->n_rad; ++k) {
            double dr = r[e] - P->rs_rad[k];
            double g = exp(-P->eta_rad * dr * dr);
            int64_t idx = (int64_t)sp[e] * P->n_rad + k;
            G[idx] += g * fc;
            if (dG) {
                double dval_dr = g * (-2.0 * P->eta_rad * dr) * fc + g * dfc;
                for (int c = 0; c < 3; ++c) dG[(idx * n_e + e) * 3 + c] += dval_dr * d[e][c] / r[e];
            }
        }
    }

    if (P->kind == 1) {
        bp_angular(P, n_e, d, sp, r, G, dG);
        free(r);
        return;
    }

    /* angular part */
    const double norm = 1.0 + sqrt(1.0 + P->eps);
    for (int64_t e = 0; e < n_e; ++e) {
        if (!(r[e] < rc)) continue;
        for (int64_t f = e + 1; f < n_e; ++f) {
            if (!(r[f] < rc)) continue;
            const double *u = d[e], *v = d[f];
            double ru = r[e], rv = r[f];
            double uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
            double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            double cr2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
            double ru2 = ru * ru, rv2 = rv * rv;
            double cos_t = uv / (ru * rv);
            double sin2 = cr2 / (ru2 * rv2);
            double ssm = sqrt(sin2 + P->eps);
            double ravg = 0.5 * (ru + rv);
            double fu = cutoff_fn(ru, rc), fv = cutoff_fn(rv, rc);
            double dfu = cutoff_deriv(ru, rc), dfv = cutoff_deriv(rv, rc);
            double F = fu * fv;
            int64_t blk = ang0 + pair_block(S, sp[e], sp[f]) * nbins;
            /* gradients of cos(theta), sin^2(theta), r_u, r_v w.r.t. u and v */
            double dcos_du[3], dcos_dv[3], dsin2_du[3], dsin2_dv[3];
            for (int c = 0; c < 3; ++c) {
                dcos_du[c] = v[c] / (ru * rv) - cos_t * u[c] / ru2;
                dcos_dv[c] = u[c] / (ru * rv) - cos_t * v[c] / rv2;
                /* |u x v|^2 = |u|^2 |v|^2 - (u.v)^2, so d|u x v|^2/du = 2 (|v|^2 u - (u.v) v) */
                dsin2_du[c] = 2.0 * (rv2 * u[c] - uv * v[c]) / (ru2 * rv2) - 2.0 * sin2 * u[c] / ru2;
                dsin2_dv[c] = 2.0 * (ru2 * v[c] - uv * u[c]) / (ru2 * rv2) - 2.0 * sin2 * v[c] / rv2;
            }
            for (int q = 0; q < P->n_rs_ang; ++q) {
                double dq = ravg - P->rs_ang[q];
                double R = exp(-P->eta_ang * dq * dq);
                double dR_dravg = -2.0 * P->eta_ang * dq * R;
                for (int p = 0; p < P->n_theta; ++p) {
                    double ct = cos(P->theta_s[p]), st = sin(P->theta_s[p]);
                    double x = (1.0 + cos_t * ct + ssm * st) / norm;
                    double A = 2.0 * pow(x, P->zeta);
                    int64_t idx = blk + (int64_t)q * P->n_theta + p;
                    G[idx] += A * R * F;
                    if (dG) {
                        double dA_dx = 2.0 * P->zeta * pow(x, P->zeta - 1.0);
                        double dT_dcos = dA_dx * ct / norm * R * F;
                        double dT_dsin2 = dA_dx * st / norm * (0.5 / ssm) * R * F;
                        double dT_dru = A * dR_dravg * 0.5 * F + A * R * dfu * fv;
                        double dT_drv = A * dR_dravg * 0.5 * F + A * R * fu * dfv;
                        for (int c = 0; c < 3; ++c) {
                            dG[(idx * n_e + e) * 3 + c] +=
                                dT_dcos * dcos_du[c] + dT_dsin2 * dsin2_du[c] + dT_dru * u[c] / ru;
                            dG[(idx * n_e + f) * 3 + c] +=
                                dT_dcos * dcos_dv[c] + dT_dsin2 * dsin2_dv[c] + dT_drv * v[c] / rv;
                        }
                    }
                }
            }
        }
    }
    free(r);
}

/* Displacements and neighbor species of row r of a list. */
static int64_t row_geometry(const ref_system *sys, const ref_nlist *nl, int64_t r, double (**d)[3],
                            int32_t **sp) {
    int64_t i = nl->rows ? nl->rows[r] : r;
    int c = struct_of_atom(sys, i);
    const double *h = sys->cell + 9 * (int64_t)c;
    int64_t b = nl->offsets[r], n_e = nl->offsets[r + 1] - b;
    *d = malloc(sizeof(double[3]) * (size_t)(n_e > 0 ? n_e : 1));
    *sp = malloc(sizeof(int32_t) * (size_t)(n_e > 0 ? n_e : 1));
    for (int64_t e = 0; e < n_e; ++e) {
        int n[3] = {nl->shift[3 * (b + e)], nl->shift[3 * (b + e) + 1], nl->shift[3 * (b + e) + 2]};
        int64_t j = nl->nbr[b + e];
        displacement(sys->pos + 3 * i, sys->pos + 3 * j, h, n, (*d)[e]);
        (*sp)[e] = sys->species[j];
    }
    return n_e;
}

/* Descriptors of every row: G[n_rows][D]; when dG != NULL, also the
 * Jacobian dG[(offsets[r] + e) * D * 3 + d * 3 + k] = dG_{r,d} / d(d_e)_k.  */
void nnref_descriptors(const ref_params *P, const ref_system *sys, const ref_nlist *nl, double *G,
                       double *dG) {
    const int64_t D = nnref_descriptor_dim(P->n_species, P->n_rad, P->n_theta, P->n_rs_ang);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nl->n_rows; ++r) {
        double (*d)[3];
        int32_t *sp;
        int64_t n_e = row_geometry(sys, nl, r, &d, &sp);
        double *jac = dG ? malloc(sizeof(double) * (size_t)(D * n_e * 3 + 1)) : NULL;
        atom_descriptor(P, n_e, (const double(*)[3])d, sp, G + r * D, jac);
        if (dG) {
            /* reorder [d][e][k] -> [e][d][k] */
            double *out = dG + nl->offsets[r] * D * 3;
            for (int64_t e = 0; e < n_e; ++e)
                for (int64_t dd = 0; dd < D; ++dd)
                    for (int k = 0; k < 3; ++k) out[(e * D + dd) * 3 + k] = jac[(dd * n_e + e) * 3 + k];
            free(jac);
        }
        free(d);
        free(sp);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-species MLP, Eq. (1) (Sec. II.A)                                      */
/* ------------------------------------------------------------------------ */

static double act_fn(int code, double z) {
    switch (code) {
    case ACT_GAUSSIAN: return exp(-z * z);
    case ACT_RELU: return z > 0.0 ? z : 0.0;
    case ACT_TANH: return tanh(z);
    default: return z;
    }
}
static double act_deriv(int code, double z) {
    switch (code) {
    case ACT_GAUSSIAN: return -2.0 * z * exp(-z * z);
    case ACT_RELU: return z > 0.0 ? 1.0 : 0.0;
    case ACT_TANH: { double t = tanh(z); return 1.0 - t * t; }
    default: return 1.0;
    }
}

static double act_deriv2(int code, double z) {
    switch (code) {
    case ACT_GAUSSIAN: return (4.0 * z * z - 2.0) * exp(-z * z);
    case ACT_TANH: { double t = tanh(z); return -2.0 * t * (1.0 - t * t); }
    default: return 0.0; /* linear; ReLU away from 0 */
    }
}

/* Atomic energy E = a^L (a scalar) of species s for input g:
 *   a^0 = g,  z^l = W^l a^(l-1) + b^l,  a^l = sigma_l(z^l).
 * If lambda != NULL, writes dE/dg.  If dparams != NULL, adds
 * scale * dE/dtheta into dparams (same layout as the parameters).          */
static double mlp_atom(const ref_model *M, int s, const double *g, double *lambda, double *dparams,
                       double scale) {
    const int L = M->n_layers[s];
    const int32_t *w = M->arch + (int64_t)s * (REF_MAX_LAYERS + 1);
    const int32_t *act = M->act + (int64_t)s * REF_MAX_LAYERS;
    const double *par = M->params + M->poff[s];
    double *a[REF_MAX_LAYERS + 1], *z[REF_MAX_LAYERS + 1];
    a[0] = (double *)g;
    z[0] = NULL;
    const double *Wl[REF_MAX_LAYERS + 1], *bl[REF_MAX_LAYERS + 1];
    int64_t pos = 0;
    int64_t woff[REF_MAX_LAYERS + 1], boff[REF_MAX_LAYERS + 1];
    for (int l = 1; l <= L; ++l) {
        woff[l] = pos;
        Wl[l] = par + pos;
        pos += (int64_t)w[l] * w[l - 1];
        boff[l] = pos;
        bl[l] = par + pos;
        pos += w[l];
    }
    for (int l = 1; l <= L; ++l) {
        z[l] = malloc(sizeof(double) * (size_t)w[l]);
        a[l] = malloc(sizeof(double) * (size_t)w[l]);
        for (int o = 0; o < w[l]; ++o) {
            double acc = bl[l][o];
            for (int k = 0; k < w[l - 1]; ++k) acc += Wl[l][(int64_t)o * w[l - 1] + k] * a[l - 1][k];
            z[l][o] = acc;
            a[l][o] = act_fn(act[l - 1], acc);
        }
    }
    double E = a[L][0];
    if (lambda || dparams) {
        /* delta^l = dE/dz^l, propagated from the output */
        double *delta = malloc(sizeof(double) * (size_t)w[L]);
        for (int o = 0; o < w[L]; ++o) delta[o] = (o == 0 ? 1.0 : 0.0) * act_deriv(act[L - 1], z[L][o]);
        for (int l = L; l >= 1; --l) {
            if (dparams) {
                for (int o = 0; o < w[l]; ++o) {
                    for (int k = 0; k < w[l - 1]; ++k)
                        dparams[M->poff[s] + woff[l] + (int64_t)o * w[l - 1] + k] += scale * delta[o] * a[l - 1][k];
                    dparams[M->poff[s] + boff[l] + o] += scale * delta[o];
                }
            }
            double *prev = malloc(sizeof(double) * (size_t)w[l - 1]);
            for (int k = 0; k < w[l - 1]; ++k) {
                double acc = 0.0;
                for (int o = 0; o < w[l]; ++o) acc += Wl[l][(int64_t)o * w[l - 1] + k] * delta[o];
                prev[k] = l > 1 ? acc * act_deriv(act[l - 2], z[l - 1][k]) : acc;
            }
            free(delta);
            delta = prev;
        }
        if (lambda) memcpy(lambda, delta, sizeof(double) * (size_t)w[0]);
        free(delta);
    }
    for (int l = 1; l <= L; ++l) {
        free(z[l]);
        free(a[l]);
    }
    return E;
}

/* MLP over a set of descriptor rows: E[r] and optionally lambda[r][D]. */
void nnref_mlp(const ref_model *M, int64_t n, const int32_t *species, const double *G, int64_t D,
               double *E, double *lambda) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r)
        E[r] = mlp_atom(M, species[r], G + r * D, lambda ? lambda + r * D : NULL, NULL, 0.0);
}

/* For species s, input g and a direction u in descriptor space: the
 * derivative of the atomic energy along u, Et = dE/dg . u, evaluated in
 * forward mode (tangents zt^l = W^l at^(l-1), at^l = sigma'(z^l) zt^l,
 * at^0 = u, Et = at^L), and scale * dEt/dtheta added into dparams by
 * reverse mode through that forward computation:
 *   zbar^l  = abar^l sigma'(z^l) + atbar^l sigma''(z^l) zt^l   (via a^l)
 *   ztbar^l = atbar^l sigma'(z^l)                              (via at^l)
 *   dW^l += zbar^l a^(l-1)T + ztbar^l at^(l-1)T,  db^l += zbar^l,
 *   abar^(l-1) = W^lT zbar^l,  atbar^(l-1) = W^lT ztbar^l,
 * starting from abar^L = 0, atbar^L = 1.  Returns Et.                      */
static double mlp_atom_tangent_grad(const ref_model *M, int s, const double *g, const double *u,
                                    double *dparams, double scale) {
    const int L = M->n_layers[s];
    const int32_t *w = M->arch + (int64_t)s * (REF_MAX_LAYERS + 1);
    const int32_t *act = M->act + (int64_t)s * REF_MAX_LAYERS;
    const double *par = M->params + M->poff[s];
    double *a[REF_MAX_LAYERS + 1], *at[REF_MAX_LAYERS + 1], *z[REF_MAX_LAYERS + 1], *zt[REF_MAX_LAYERS + 1];
    const double *Wl[REF_MAX_LAYERS + 1], *bl[REF_MAX_LAYERS + 1];
    int64_t woff[REF_MAX_LAYERS + 1], boff[REF_MAX_LAYERS + 1];
    int64_t pos = 0;
    for (int l = 1; l <= L; ++l) {
        woff[l] = pos;
        Wl[l] = par + pos;
        pos += (int64_t)w[l] * w[l - 1];
        boff[l] = pos;
        bl[l] = par + pos;
        pos += w[l];
    }
    a[0] = (double *)g;
    at[0] = (double *)u;
    for (int l = 1; l <= L; ++l) {
        z[l] = malloc(sizeof(double) * (size_t)w[l]);
        zt[l] = malloc(sizeof(double) * (size_t)w[l]);
        a[l] = malloc(sizeof(double) * (size_t)w[l]);
        at[l] = malloc(sizeof(double) * (size_t)w[l]);
        for (int o = 0; o < w[l]; ++o) {
            double acc = bl[l][o], acct = 0.0;
            for (int k = 0; k < w[l - 1]; ++k) {
                acc += Wl[l][(int64_t)o * w[l - 1] + k] * a[l - 1][k];
                acct += Wl[l][(int64_t)o * w[l - 1] + k] * at[l - 1][k];
            }
            z[l][o] = acc;
            zt[l][o] = acct;
            a[l][o] = act_fn(act[l - 1], acc);
            at[l][o] = act_deriv(act[l - 1], acc) * acct;
        }
    }
    const double Et = at[L][0];
    double *abar = calloc((size_t)w[L], sizeof(double));
    double *atbar = calloc((size_t)w[L], sizeof(double));
    atbar[0] = 1.0;
    for (int l = L; l >= 1; --l) {
        double *zbar = malloc(sizeof(double) * (size_t)w[l]);
        double *ztbar = malloc(sizeof(double) * (size_t)w[l]);
        for (int o = 0; o < w[l]; ++o) {
            zbar[o] = abar[o] * act_deriv(act[l - 1], z[l][o]) + atbar[o] * act_deriv2(act[l - 1], z[l][o]) * zt[l][o];
            ztbar[o] = atbar[o] * act_deriv(act[l - 1], z[l][o]);
        }
        for (int o = 0; o < w[l]; ++o) {
            for (int k = 0; k < w[l - 1]; ++k)
                dparams[M->poff[s] + woff[l] + (int64_t)o * w[l - 1] + k] +=
                    scale * (zbar[o] * a[l - 1][k] + ztbar[o] * at[l - 1][k]);
            dparams[M->poff[s] + boff[l] + o] += scale * zbar[o];
        }
        double *pa = calloc((size_t)w[l - 1], sizeof(double));
        double *pat = calloc((size_t)w[l - 1], sizeof(double));
        for (int k = 0; k < w[l - 1]; ++k)
            for (int o = 0; o < w[l]; ++o) {
                pa[k] += Wl[l][(int64_t)o * w[l - 1] + k] * zbar[o];
                pat[k] += Wl[l][(int64_t)o * w[l - 1] + k] * ztbar[o];
            }
        free(zbar);
        free(ztbar);
        free(abar);
        free(atbar);
        abar = pa;
        atbar = pat;
    }
    free(abar);
    free(atbar);
    for (int l = 1; l <= L; ++l) {
        free(z[l]);
        free(zt[l]);
        free(a[l]);
        free(at[l]);
    }
    return Et;
}

/* The descriptor tangent of every row atom i along a displacement field v
 * (one 3-vector per atom): u_i = sum_k dG_i/dx_k . v_k
 *                              = sum_{e in row i} dG_i/dd_e . (v_j(e) - v_i). */
void nnref_descriptor_tangent(const ref_params *P, const ref_system *sys, const ref_nlist *nl, const double *v,
                              double *u) {
    const int64_t D = nnref_descriptor_dim(P->n_species, P->n_rad, P->n_theta, P->n_rs_ang);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nl->n_rows; ++r) {
        int64_t i = nl->rows ? nl->rows[r] : r;
        double (*d)[3];
        int32_t *sp;
        int64_t n_e = row_geometry(sys, nl, r, &d, &sp);
        double *G = malloc(sizeof(double) * (size_t)D);
        double *jac = malloc(sizeof(double) * (size_t)(D * n_e * 3 + 1));
        atom_descriptor(P, n_e, (const double(*)[3])d, sp, G, jac);
        for (int64_t dd = 0; dd < D; ++dd) {
            double acc = 0.0;
            for (int64_t e = 0; e < n_e; ++e) {
                int64_t j = nl->nbr[nl->offsets[r] + e];
                for (int k = 0; k < 3; ++k) acc += jac[(dd * n_e + e) * 3 + k] * (v[3 * j + k] - v[3 * i + k]);
            }
            u[r * D + dd] = acc;
        }
        free(jac);
        free(G);
        free(d);
        free(sp);
    }
}

/* Gradient of a loss on energies and forces with respect to every MLP
 * parameter, given the upstream gradients gE[c] = dL/dE_c (NULL: none) and
 * gF[k][3] = dL/dF_k (NULL: none):
 *   dL/dtheta = sum_c gE_c sum_{i in c} dE_i/dtheta
 *             + sum_k gF_k . dF_k/dtheta,
 * and, with F_k = -sum_i dE_i/dx_k = -sum_i lambda_i . dG_i/dx_k,
 *   sum_k gF_k . dF_k/dtheta = -sum_i d/dtheta [lambda_i . u_i],
 * u_i the descriptor tangent along gF (theta-independent).  Needs a list
 * holding every atom's row.  Writes dparams (overwritten).                 */
void nnref_force_loss_grad(const ref_params *P, const ref_model *M, const ref_system *sys,
                           const ref_nlist *nl, const double *gE, const double *gF, double *dparams,
                           int64_t n_params) {
    const int64_t D = nnref_descriptor_dim(P->n_species, P->n_rad, P->n_theta, P->n_rs_ang);
    int64_t N = sys->n_atoms;
    double *G = malloc(sizeof(double) * (size_t)(N * D + 1));
    double *u = gF ? malloc(sizeof(double) * (size_t)(N * D + 1)) : NULL;
    nnref_descriptors(P, sys, nl, G, NULL);
    if (gF) nnref_descriptor_tangent(P, sys, nl, gF, u);
    memset(dparams, 0, sizeof(double) * (size_t)n_params);
    for (int c = 0; c < sys->n_structs; ++c)
        for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a) {
            if (gE) (void)mlp_atom(M, sys->species[a], G + a * D, NULL, dparams, gE[c]);
            if (gF) (void)mlp_atom_tangent_grad(M, sys->species[a], G + a * D, u + a * D, dparams, -1.0);
        }
    free(u);
    free(G);
}

/* ------------------------------------------------------------------------ */
/* Energies and forces (Sec. II: E = sum of atomic terms; forces are the      */
/* derivatives of the energy)                                                */
/* ------------------------------------------------------------------------ */

/* For every row atom i: E_i, and the per-entry gradients
 * pg[(offsets[r] + e) * 3 + k] = dE_i / d(d_e)_k  (d_e = displacement to the
 * e-th neighbor entry).                                                     */
void nnref_atom_energies(const ref_params *P, const ref_model *M, const ref_system *sys,
                         const ref_nlist *nl, double *E_row, double *pg) {
    const int64_t D = nnref_descriptor_dim(P->n_species, P->n_rad, P->n_theta, P->n_rs_ang);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nl->n_rows; ++r) {
        int64_t i = nl->rows ? nl->rows[r] : r;
        double (*d)[3];
        int32_t *sp;
        int64_t n_e = row_geometry(sys, nl, r, &d, &sp);
        double *G = malloc(sizeof(double) * (size_t)D);
        double *lam = malloc(sizeof(double) * (size_t)D);
        double *jac = pg ? malloc(sizeof(double) * (size_t)(D * n_e * 3 + 1)) : NULL;
        atom_descriptor(P, n_e, (const double(*)[3])d, sp, G, jac);
        E_row[r] = mlp_atom(M, sys->species[i], G, pg ? lam : NULL, NULL, 0.0);
        if (pg) {
            for (int64_t e = 0; e < n_e; ++e)
                for (int k = 0; k < 3; ++k) {
                    double acc = 0.0;
                    for (int64_t dd = 0; dd < D; ++dd) acc += lam[dd] * jac[(dd * n_e + e) * 3 + k];
                    pg[(nl->offsets[r] + e) * 3 + k] = acc;
                }
            free(jac);
        }
        free(lam);
        free(G);
        free(d);
        free(sp);
    }
}

/* Forces on a set of target atoms: F_k = -dE/dx_k with E = sum_i E_i.
 * Since d_e = x_j - x_i + (image), dE_i/dx_j += dE_i/dd_e and
 * dE_i/dx_i -= dE_i/dd_e.  The list must hold the rows of every atom whose
 * energy depends on a target (the target itself and its neighbors); rows of
 * other atoms add nothing to the targets.  Also returns E_row.             */
void nnref_forces(const ref_params *P, const ref_model *M, const ref_system *sys,
                  const ref_nlist *nl, const int64_t *targets, int64_t n_targets, double *E_row,
                  double *F) {
    int64_t nnz = nl->offsets[nl->n_rows];
    double *pg = malloc(sizeof(double) * (size_t)(3 * nnz + 1));
    nnref_atom_energies(P, M, sys, nl, E_row, pg);
    /* position of each atom in the target list (or -1) */
    int64_t *slot = malloc(sizeof(int64_t) * (size_t)(sys->n_atoms > 0 ? sys->n_atoms : 1));
    for (int64_t a = 0; a < sys->n_atoms; ++a) slot[a] = -1;
    for (int64_t t = 0; t < n_targets; ++t) slot[targets[t]] = t;
    memset(F, 0, sizeof(double) * (size_t)(3 * n_targets));
    for (int64_t r = 0; r < nl->n_rows; ++r) {
        int64_t i = nl->rows ? nl->rows[r] : r;
        for (int64_t e = nl->offsets[r]; e < nl->offsets[r + 1]; ++e) {
            int64_t j = nl->nbr[e];
            for (int k = 0; k < 3; ++k) {
                if (slot[j] >= 0) F[3 * slot[j] + k] -= pg[3 * e + k];
                if (slot[i] >= 0) F[3 * slot[i] + k] += pg[3 * e + k];
            }
        }
    }
    free(slot);
    free(pg);
}

/* Full evaluation for a list holding the rows of all atoms (rows == NULL):
 * per-structure energies E_struct[B] = sum of E_i over the structure,
 * E_atom[N] and forces F[N][3].                                             */
void nnref_energy_forces(const ref_params *P, const ref_model *M, const ref_system *sys,
                         const ref_nlist *nl, double *E_struct, double *E_atom, double *F) {
    int64_t N = sys->n_atoms;
    int64_t *all = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    for (int64_t a = 0; a < N; ++a) all[a] = a;
    nnref_forces(P, M, sys, nl, all, N, E_atom, F);
    for (int c = 0; c < sys->n_structs; ++c) {
        double acc = 0.0;
        for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a) acc += E_atom[a];
        E_struct[c] = acc;
    }
    free(all);
}

/* Energy loss L = (1/B) sum_c (E_c - T_c)^2 over structures (per
 * configuration, quadratic; Sec. II.A) and its gradient with respect to
 * every MLP parameter: dL/dtheta = sum_c (2/B)(E_c - T_c) sum_{i in c}
 * dE_i/dtheta.  Needs a list holding every atom's row.  Returns L.         */
double nnref_energy_loss_grad(const ref_params *P, const ref_model *M, const ref_system *sys,
                              const ref_nlist *nl, const double *targets, double *E_struct,
                              double *dparams, int64_t n_params) {
    const int64_t D = nnref_descriptor_dim(P->n_species, P->n_rad, P->n_theta, P->n_rs_ang);
    int64_t N = sys->n_atoms;
    int B = sys->n_structs;
    double *G = malloc(sizeof(double) * (size_t)(N * D + 1));
    nnref_descriptors(P, sys, nl, G, NULL);
    double *E = malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    nnref_mlp(M, N, sys->species, G, D, E, NULL);
    double L = 0.0;
    for (int c = 0; c < B; ++c) {
        double acc = 0.0;
        for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a) acc += E[a];
        E_struct[c] = acc;
        L += (acc - targets[c]) * (acc - targets[c]);
    }
    L /= B;
    memset(dparams, 0, sizeof(double) * (size_t)n_params);
    for (int c = 0; c < B; ++c) {
        double w = 2.0 / B * (E_struct[c] - targets[c]);
        for (int64_t a = sys->atom_ptr[c]; a < sys->atom_ptr[c + 1]; ++a)
            (void)mlp_atom(M, sys->species[a], G + a * D, NULL, dparams, w);
    }
    free(E);
    free(G);
    return L;
}

int nnref_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
