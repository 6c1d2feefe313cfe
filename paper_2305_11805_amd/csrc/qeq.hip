// Charge equilibration of Sec. II.B on the device, one structure per block.
//
// The network gives each atom the coefficients of a second-order expansion of
// its energy in its charge: E0_i, chi_i, J_i.  With Gaussian charges of width
// sigma (per species) the electrostatic energy is a quadratic form, and the
// charges minimise
//   E(q) = sum_i E0_i + chi . q + q^T A q / 2,
//   A_ij = k_e erf(r_ij / (sqrt(2) gamma_ij)) / r_ij  (i != j),
//   A_ii = J_i + k_e / (sigma_i sqrt(pi)),   gamma_ij^2 = sigma_i^2 + sigma_j^2,
// subject to sum_i q_i = Q (the structure's total charge): q = y + mu z with
// A y = -chi, A z = 1 and mu = (Q - sum y) / sum z, every atom at chemical
// potential dE/dq_i = mu, and E = sum E0 + chi . q / 2 + mu Q / 2.
//
// The block assembles A in LDS in FP64, factors it by Cholesky (A is the
// Coulomb matrix of Gaussian charges, positive definite, plus the
// hardnesses on the diagonal; a pivot <= 0 is reported), solves both right
// sides, and writes the charges, the energy and the output seeds (1, q,
// q^2 / 2) with which the network's backward pass gives the forces at fixed
// charges (the minimum makes the derivative of the solve drop out).  The
// Coulomb part of the forces is a second pass over the pairs.  Every sum has
// a fixed order, so results are the same on every run.
#include <math.h>

#include "common.h"

namespace nnp {

constexpr int kQeqThreads = 256;
constexpr int kQeqLd = kQeqMax + 1;  // padded row stride of A in LDS

__device__ __forceinline__ bool qeq_struct_ok(const QeqArgs& a, int c, int64_t a0, int64_t n) {
  const uint8_t* pb = a.pbc + 3 * (int64_t)c;
  return n <= kQeqMax && pb[0] == 0 && pb[1] == 0 && pb[2] == 0;
}

// Fixed-order FP64 sum of v over the block (v per thread; result to all).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = kQeqThreads / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kQeqThreads) k_qeq_solve(QeqArgs a) {
  __shared__ double A[kQeqMax * kQeqLd];
  __shared__ double x[kQeqMax][3];
  __shared__ double y[kQeqMax], z[kQeqMax], chi[kQeqMax];
  __shared__ double sh[kQeqThreads];
  __shared__ int bad;
  const int c = blockIdx.x, t = threadIdx.x;
  const int64_t a0 = a.atom_ptr[c], a1 = a.atom_ptr[c + 1];
  const int64_t n64 = a1 - a0;
  if (n64 <= 0) {
    if (t == 0) a.E_struct[c] = 0.0;
    return;
  }
  if (!qeq_struct_ok(a, c, a0, n64)) {
    for (int64_t i = a0 + t; i < a1; i += kQeqThreads) {
      a.q[i] = 0.0;
      a.seed[3 * i] = 1.f;
      a.seed[3 * i + 1] = 0.f;
      a.seed[3 * i + 2] = 0.f;
    }
    if (t == 0) {
      a.E_struct[c] = 0.0;
      atomicOr((unsigned long long*)&a.meta[kMetaErr], (unsigned long long)kErrQeq);
    }
    return;
  }
  const int n = (int)n64;
  if (t == 0) bad = 0;
  for (int i = t; i < n; i += kQeqThreads) {
    for (int k = 0; k < 3; ++k) x[i][k] = a.pos[3 * (a0 + i) + k];
    chi[i] = (double)a.out[3 * (a0 + i) + 1];
  }
  __syncthreads();
  // A, lower triangle and diagonal (the factorization reads only those)
  const double rsqpi = 0.56418958354775628;  // 1 / sqrt(pi)
  for (int e = t; e < n * n; e += kQeqThreads) {
    const int i = e / n, j = e % n;
    if (j > i) continue;
    const int si = a.species[a0 + i];
    const double sgi = a.sigma[si];
    double v;
    if (i == j) {
      v = (double)a.out[3 * (a0 + i) + 2] + a.ke * rsqpi / sgi;
    } else {
      const double sgj = a.sigma[a.species[a0 + j]];
      const double dx = x[i][0] - x[j][0], dy = x[i][1] - x[j][1], dz = x[i][2] - x[j][2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double g = sqrt(2.0 * (sgi * sgi + sgj * sgj));
      v = a.ke * erf(r / g) / r;
    }
    A[i * kQeqLd + j] = v;
  }
  __syncthreads();
  // Cholesky, A = L L^T in place (lower triangle), column by column
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      const double d = A[j * kQeqLd + j];
      if (!(d > 0.0)) bad = 1;
      A[j * kQeqLd + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double ljj = A[j * kQeqLd + j];
    for (int i = j + 1 + t; i < n; i += kQeqThreads) A[i * kQeqLd + j] /= ljj;
    __syncthreads();
    const int m = n - j - 1;  // trailing (i, k), j < k <= i < n
    for (int e = t; e < m * m; e += kQeqThreads) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) A[i * kQeqLd + k] -= A[i * kQeqLd + j] * A[k * kQeqLd + j];
    }
    __syncthreads();
  }
  // L u = b (b = -chi and 1), then L^T v = u, both right sides at once
  for (int i = t; i < n; i += kQeqThreads) {
    y[i] = -chi[i];
    z[i] = 1.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double ljj = A[j * kQeqLd + j];
    const double yj = y[j] / ljj, zj = z[j] / ljj;
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += kQeqThreads) {
      const double l = A[i * kQeqLd + j];
      y[i] -= l * yj;
      z[i] -= l * zj;
    }
    if (t == 0) {
      y[j] = yj;
      z[j] = zj;
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = A[j * kQeqLd + j];
    const double yj = y[j] / ljj, zj = z[j] / ljj;
    __syncthreads();
    for (int i = t; i < j; i += kQeqThreads) {
      const double l = A[j * kQeqLd + i];  // (L^T)_ij = L_ji
      y[i] -= l * yj;
      z[i] -= l * zj;
    }
    if (t == 0) {
      y[j] = yj;
      z[j] = zj;
    }
    __syncthreads();
  }
  double sy = 0.0, sz = 0.0;
  for (int i = t; i < n; i += kQeqThreads) {
    sy += y[i];
    sz += z[i];
  }
  sy = block_sum(sy, sh);
  sz = block_sum(sz, sh);
  const double Q = a.total[c];
  const double mu = (Q - sy) / sz;
  double e0 = 0.0, cq = 0.0;
  for (int i = t; i < n; i += kQeqThreads) {
    const double qi = bad ? 0.0 : y[i] + mu * z[i];
    const int64_t g = a0 + i;
    a.q[g] = qi;
    a.seed[3 * g] = 1.f;
    a.seed[3 * g + 1] = (float)qi;
    a.seed[3 * g + 2] = (float)(0.5 * qi * qi);
    e0 += (double)a.out[3 * g];
    cq += chi[i] * qi;
  }
  e0 = block_sum(e0, sh);
  cq = block_sum(cq, sh);
  if (t == 0) {
    a.E_struct[c] = bad ? 0.0 : e0 + 0.5 * cq + 0.5 * mu * Q;
    if (bad) atomicOr((unsigned long long*)&a.meta[kMetaErr], (unsigned long long)kErrQeq);
  }
}

// F_i += -sum_{j != i} k_e q_i q_j f'(r_ij) (x_i - x_j) / r_ij with
// f(r) = erf(r / g) / r, g = sqrt(2 (sigma_i^2 + sigma_j^2)); FP64, j in order.
__global__ void __launch_bounds__(kQeqThreads) k_qeq_coulomb(QeqArgs a, float* __restrict__ F) {
  const int c = blockIdx.x;
  const int64_t a0 = a.atom_ptr[c], a1 = a.atom_ptr[c + 1];
  if (a1 - a0 <= 0 || !qeq_struct_ok(a, c, a0, a1 - a0)) return;
  const double tsqpi = 1.1283791670955126;  // 2 / sqrt(pi)
  for (int64_t i = a0 + threadIdx.x; i < a1; i += kQeqThreads) {
    const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
    const double si = a.sigma[a.species[i]], qi = a.q[i];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int64_t j = a0; j < a1; ++j) {
      if (j == i) continue;
      const double dx = xi - a.pos[3 * j], dy = yi - a.pos[3 * j + 1], dz = zi - a.pos[3 * j + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double sj = a.sigma[a.species[j]];
      const double g = sqrt(2.0 * (si * si + sj * sj));
      const double u = r / g;
      const double fp = tsqpi * exp(-u * u) / (g * r) - erf(u) / (r * r);
      const double s = a.ke * qi * a.q[j] * fp / r;
      fx -= s * dx;
      fy -= s * dy;
      fz -= s * dz;
    }
    F[3 * i] += (float)fx;
    F[3 * i + 1] += (float)fy;
    F[3 * i + 2] += (float)fz;
  }
}

void launch_qeq_solve(const QeqArgs& a, hipStream_t s) {
  if (a.B == 0) return;
  hipLaunchKernelGGL(k_qeq_solve, dim3((unsigned)a.B), dim3(kQeqThreads), 0, s, a);
}

void launch_qeq_coulomb(const QeqArgs& a, float* F, hipStream_t s) {
  if (a.B == 0 || a.N == 0) return;
  hipLaunchKernelGGL(k_qeq_coulomb, dim3((unsigned)a.B), dim3(kQeqThreads), 0, s, a, F);
}

}  // namespace nnp
