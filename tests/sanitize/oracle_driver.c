/* Runs the FP64 oracle (nnref.c, compiled into this file) on small inputs
 * under AddressSanitizer and UndefinedBehaviorSanitizer: neighbor lists
 * (brute force and cell-binned, compared entry for entry), descriptors with
 * the Jacobian, the MLP, energies and forces, the descriptor tangent and the
 * force-loss weight gradient, for a triclinic periodic cell and a cluster.
 * Exit status 0 and no sanitizer report = pass. */
#include "../../oracle/nnref.c"

#include <stdio.h>

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run(int periodic) {
    const int N = 24, S = 2, D_rad = 6, NT = 4, NR = 3;
    double pos[24 * 3], cell[9] = {6.0, 0.0, 0.0, 0.7, 5.6, 0.0, -0.4, 0.5, 6.3};
    int32_t species[24];
    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) pos[3 * i + k] = 6.0 * urand() - (periodic ? 1.0 : 0.0);
        species[i] = (int32_t)(urand() * S);
    }
    int64_t atom_ptr[2] = {0, N};
    uint8_t pbc[3] = {(uint8_t)periodic, (uint8_t)periodic, (uint8_t)periodic};
    ref_system sys = {N, 1, pos, species, atom_ptr, cell, pbc};
    const double rc = 3.8;
    int64_t off_b[25], off_c[25];
    int64_t nnz = nnref_neighbors_brute(&sys, rc, 0, NULL, N, 0, off_b, NULL, NULL);
    int32_t *nb_b = malloc(sizeof(int32_t) * (size_t)(nnz + 1)), *sh_b = malloc(sizeof(int32_t) * 3 * (size_t)(nnz + 1));
    int32_t *nb_c = malloc(sizeof(int32_t) * (size_t)(nnz + 1)), *sh_c = malloc(sizeof(int32_t) * 3 * (size_t)(nnz + 1));
    nnref_neighbors_brute(&sys, rc, 0, NULL, N, nnz, off_b, nb_b, sh_b);
    int64_t nnz_c = nnref_neighbors_cells(&sys, rc, NULL, N, nnz, off_c, nb_c, sh_c);
    if (nnz_c != nnz) return 1;
    for (int64_t e = 0; e < nnz; ++e)
        if (nb_b[e] != nb_c[e] || sh_b[3 * e] != sh_c[3 * e] || sh_b[3 * e + 2] != sh_c[3 * e + 2]) return 2;
    double rs_rad[6], th[4], rs_ang[3];
    for (int k = 0; k < D_rad; ++k) rs_rad[k] = 0.5 + k * (rc - 0.5) / (D_rad - 1);
    for (int k = 0; k < NT; ++k) th[k] = (k + 0.5) * 3.141592653589793 / NT;
    for (int k = 0; k < NR; ++k) rs_ang[k] = 0.5 + k * (rc - 0.5) / (NR - 1);
    ref_params P = {S, rc, D_rad, 4.0, rs_rad, NT, th, NR, 3.0, rs_ang, 6.0, 1e-3, 0, NULL, NULL, NULL};
    ref_nlist nl = {N, NULL, off_b, nb_b, sh_b};
    const int64_t D = nnref_descriptor_dim(S, D_rad, NT, NR);
    double *G = calloc((size_t)(N * D), sizeof(double));
    double *dG = calloc((size_t)(nnz * D * 3 + 1), sizeof(double));
    nnref_descriptors(&P, &sys, &nl, G, dG);
    /* a 2-species MLP D -> 5 -> 4 -> 1 (tanh) */
    int32_t n_layers[2] = {3, 3}, arch[2 * (REF_MAX_LAYERS + 1)] = {0}, act[2 * REF_MAX_LAYERS] = {0};
    int64_t poff[2];
    int64_t np = 0;
    for (int s = 0; s < 2; ++s) {
        int32_t *w = arch + s * (REF_MAX_LAYERS + 1);
        w[0] = (int32_t)D;
        w[1] = 5;
        w[2] = 4;
        w[3] = 1;
        act[s * REF_MAX_LAYERS + 0] = ACT_TANH;
        act[s * REF_MAX_LAYERS + 1] = ACT_GAUSSIAN;
        act[s * REF_MAX_LAYERS + 2] = ACT_LINEAR;
        poff[s] = np;
        for (int l = 1; l <= 3; ++l) np += (int64_t)w[l] * w[l - 1] + w[l];
    }
    double *params = malloc(sizeof(double) * (size_t)np);
    for (int64_t k = 0; k < np; ++k) params[k] = 0.3 * (urand() - 0.5);
    ref_model M = {2, n_layers, arch, act, params, poff};
    double E[24], Ea[24], lam[24 * 64], F[24 * 3], Es[1], v[24 * 3];
    if (D > 64) return 3;
    nnref_mlp(&M, N, species, G, D, E, lam);
    nnref_energy_forces(&P, &M, &sys, &nl, Es, Ea, F);
    for (int i = 0; i < 3 * N; ++i) v[i] = urand() - 0.5;
    double *u = calloc((size_t)(N * D), sizeof(double));
    nnref_descriptor_tangent(&P, &sys, &nl, v, u);
    double *dp = calloc((size_t)np, sizeof(double));
    double gE[1] = {0.7};
    nnref_force_loss_grad(&P, &M, &sys, &nl, gE, v, dp, np);
    double T[1] = {0.1};
    nnref_energy_loss_grad(&P, &M, &sys, &nl, T, Es, dp, np);
    double fsum[3] = {0, 0, 0};
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < 3; ++k) fsum[k] += F[3 * i + k];
    printf("%s: %lld entries, D %lld, E %.6f, |sum F| %.2e\n", periodic ? "periodic" : "cluster", (long long)nnz,
           (long long)D, Es[0], fabs(fsum[0]) + fabs(fsum[1]) + fabs(fsum[2]));
    free(nb_b); free(sh_b); free(nb_c); free(sh_c); free(G); free(dG); free(params); free(u); free(dp);
    return 0;
}

int main(void) {
    int rc = run(1);
    if (rc) return rc;
    return run(0);
}
