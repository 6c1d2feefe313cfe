/* Host-side paths of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer: descriptor sizes, workspace sizes for the
 * fused, layer-by-layer and charge-equilibration models, and every argument
 * check that returns before anything is enqueued (fake device pointers,
 * never dereferenced on the host; no GPU is needed).  Exit status 0 and no
 * sanitizer report = pass. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "nnpot.h"

#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "failed: %s (line %d): %s\n", #cond, __LINE__, nn_last_error()); \
      return 1;                                                         \
    }                                                                   \
  } while (0)

static void* fake(uintptr_t k) { return (void*)(0x100000u * k); }

int main(void) {
  double rs_rad[16], th[8], rs_ang[4];
  for (int k = 0; k < 16; ++k) rs_rad[k] = 0.5 + 0.25 * k;
  for (int k = 0; k < 8; ++k) th[k] = (k + 0.5) * 3.14159265358979 / 8;
  for (int k = 0; k < 4; ++k) rs_ang[k] = 0.5 + k;
  nn_mbp_params p;
  memset(&p, 0, sizeof p);
  p.n_species = 2; p.rc = 4.6; p.n_rad = 16; p.eta_rad = 16; p.rs_rad = rs_rad; p.n_theta = 8; p.theta_s = th;
  p.n_rs_ang = 4; p.eta_ang = 12; p.rs_ang = rs_ang; p.zeta = 50; p.eps = 1e-3; p.kind = NN_DESC_MBP;
  const int64_t D = nn_descriptor_dim(&p);
  CHECK(D == 16 * 2 + 8 * 4 * 3);
  nn_mbp_params bad = p;
  bad.n_theta = 5;
  CHECK(nn_descriptor_dim(&bad) == -1);
  bad = p;
  bad.zeta = 2.5;
  CHECK(nn_descriptor_dim(&bad) == -1);
  CHECK(nn_jacobian_stride(&p) > 0);
  /* models: fused (64, 32), layer by layer (per species), charge equilibration (3 outputs) */
  nn_model m[3];
  memset(m, 0, sizeof m);
  const int widths[3][2][5] = {{{(int)D, 64, 32, 1, 0}, {(int)D, 64, 32, 1, 0}},
                               {{(int)D, 48, 1, 0, 0}, {(int)D, 40, 24, 16, 1}},
                               {{(int)D, 15, 15, 3, 0}, {(int)D, 15, 15, 3, 0}}};
  const int nl_[3][2] = {{3, 3}, {2, 4}, {3, 3}};
  for (int k = 0; k < 3; ++k) {
    m[k].n_species = 2;
    for (int s = 0; s < 2; ++s) {
      m[k].mlp[s].n_layers = nl_[k][s];
      for (int l = 0; l <= nl_[k][s]; ++l) m[k].mlp[s].width[l] = widths[k][s][l];
      for (int l = 0; l < nl_[k][s]; ++l) {
        m[k].mlp[s].act[l] = l + 1 < nl_[k][s] ? NN_ACT_GAUSSIAN : NN_ACT_LINEAR;
        m[k].mlp[s].W[l] = (const float*)fake(20 + 2 * l);
        m[k].mlp[s].b[l] = (const float*)fake(21 + 2 * l);
      }
    }
  }
  size_t ws[3];
  for (int k = 0; k < 3; ++k) CHECK(nn_workspace_size(1000, 40, 20000, &p, &m[k], 0, 0, &ws[k]) == NN_OK);
  CHECK(ws[1] > ws[0] / 4 && ws[2] > 0);
  size_t wsj = 0;
  CHECK(nn_workspace_size(1000, 40, 20000, &p, &m[0], NN_STORE_JACOBIAN, (size_t)1 << 40, &wsj) == NN_OK);
  CHECK(wsj > ws[0]);
  CHECK(nn_workspace_size(-1, 1, 0, &p, NULL, 0, 0, &wsj) == NN_E_INVALID);
  /* argument checks that return before any launch */
  nn_system sys = {1000, 40, (const double*)fake(1), (const int32_t*)fake(2), (const int64_t*)fake(3),
                   (const double*)fake(4), (const uint8_t*)fake(5)};
  nn_nlist nl = {20000, (int64_t*)fake(6), (int32_t*)fake(7), (int8_t*)fake(8), (int32_t*)fake(9),
                 (double*)fake(10), (int64_t*)fake(11), NULL, 4.6};
  double* E = (double*)fake(12);
  float* F = (float*)fake(13);
  void* w = fake(14);
  CHECK(nn_energy_forces(&sys, &nl, &p, &m[0], 0, 0, E, NULL, F, w, ws[0] - 1, NULL) == NN_E_WORKSPACE);
  CHECK(nn_energy_forces(&sys, &nl, &p, &m[0], NN_BF16_MLP | NN_BF16X3_MLP, 0, E, NULL, F, w, ws[0], NULL) ==
        NN_E_INVALID);
  CHECK(nn_energy_forces(&sys, &nl, &p, &m[1], NN_BF16X3_MLP, 0, E, NULL, F, w, ws[1], NULL) == NN_E_UNSUPPORTED);
  CHECK(nn_energy_forces(&sys, &nl, &p, &m[2], 0, 0, E, NULL, F, w, ws[2], NULL) == NN_E_INVALID);  /* 3 outputs */
  CHECK(nn_energy_forces(&sys, &nl, &p, &m[0], 0, 0, NULL, NULL, F, w, ws[0], NULL) == NN_E_INVALID);
  nn_nlist short_nl = nl;
  short_nl.radius = 4.0;
  CHECK(nn_energy_forces(&sys, &short_nl, &p, &m[0], 0, 0, E, NULL, F, w, ws[0], NULL) == NN_E_INVALID);
  CHECK(nn_energy_forces_noalloc(&sys, &nl, &p, &m[0], NN_STORE_JACOBIAN, E, NULL, F, NULL) == NN_E_INVALID);
  nn_system big = sys;
  big.n_atoms = 1000000;
  CHECK(nn_energy_forces_noalloc(&big, &nl, &p, &m[0], 0, E, NULL, F, NULL) == NN_E_WORKSPACE);
  double sigma[2] = {1.0, -1.0};
  nn_qeq_params qp = {sigma, 14.4};
  CHECK(nn_energy_forces_qeq(&sys, &nl, &p, &m[2], &qp, E, E, NULL, F, w, ws[2], NULL) == NN_E_INVALID);
  CHECK(nn_energy_forces_qeq(&sys, &nl, &p, &m[0], &qp, E, E, NULL, F, w, ws[0], NULL) == NN_E_INVALID);
  CHECK(nn_energy_forces_grad(&sys, &nl, &p, &m[0], 0, NULL, NULL, NULL, NULL, NULL, NULL, w, ws[0], NULL) ==
        NN_E_INVALID);
  CHECK(nn_energy_forces_grad(&sys, &nl, &p, &m[0], 0, E, F, NULL, F, NULL, NULL, w, ws[0], NULL) ==
        NN_E_UNSUPPORTED);
  CHECK(nn_build_neighbors(&sys, 4.6, 0.5, &nl, w, 8, NULL) == NN_E_WORKSPACE);
  CHECK(nn_build_neighbors(NULL, 4.6, 0.0, &nl, w, 8, NULL) == NN_E_INVALID);
  nn_langevin lp = {0.0, 0.0, 0.0};
  CHECK(nn_md_langevin(&sys, (double*)fake(1), (double*)fake(15), (const double*)fake(16), &nl, 4.6, 0.0, &p, &m[0],
                       0, &lp, NULL, 3, E, F, w, ws[0], NULL) == NN_E_INVALID);
  nn_loss_params lsp = {7, 0, 0, 1.0, 1.0};
  double L1[1];
  CHECK(nn_loss(&sys, &lsp, E, E, NULL, NULL, L1, E, NULL, w, ws[0], NULL) == NN_E_INVALID);
  CHECK(nn_timing(0) == NN_OK);
  double ms[NN_STAGE_COUNT];
  int64_t n[NN_STAGE_COUNT];
  CHECK(nn_timing_read(ms, n) == NN_OK);
  nn_autotune_reset();
  printf("abi host paths: workspace %zu / %zu / %zu bytes\n", ws[0], ws[1], ws[2]);
  return 0;
}
