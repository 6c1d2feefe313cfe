// Langevin dynamics driven by the potential: the repeated evaluation of
// Table II (Sec. III.B), integrated with the BAOAB splitting of the Langevin
// equation (Leimkuhler and Matthews, 2013).  One step from x, v and the
// forces F(x):
//   B  v += (dt/2) F / m
//   A  x += (dt/2) v
//   O  v  = c1 v + c2 sqrt(kT / m) xi,   c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2)
//   A  x += (dt/2) v
//   (list update and F, E at the new x)
//   B  v += (dt/2) F / m
// The second B of a step and the first B of the next use the same forces, so
// between steps they are one kick of dt.  Positions and velocities are FP64
// (the positions are FP64 inputs of the potential), forces FP32.  Units:
// Angstrom, fs, eV, amu.
#include "common.h"

namespace nnp {

// (eV / Angstrom) / amu in Angstrom / fs^2
constexpr double kAccel = 1.602176634e-19 / 1.66053906660e-27 / 1e10;  // eV / amu in Angstrom^2 / fs^2 (SI values)

__global__ void __launch_bounds__(256) k_md_update(int64_t N, int mode, double* __restrict__ pos,
                                                   double* __restrict__ vel, const double* __restrict__ inv_mass,
                                                   const float* __restrict__ F, const float* __restrict__ noise,
                                                   double dt, double c1, double c2_sqrt_kT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double a = inv_mass[i] * kAccel;
  const double kick = (mode == kMdKickDrift ? dt : 0.5 * dt) * a;
  double v[3], x[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = vel[3 * i + k] + kick * (double)F[3 * i + k];
    x[k] = pos[3 * i + k];
  }
  if (mode != kMdKick) {
    const double sigma = c2_sqrt_kT * sqrt(a);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k] += 0.5 * dt * v[k];
      v[k] = c1 * v[k] + (noise ? sigma * (double)noise[3 * i + k] : 0.0);
      x[k] += 0.5 * dt * v[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) pos[3 * i + k] = x[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) vel[3 * i + k] = v[k];
}

void launch_md_update(int64_t N, int mode, double* pos, double* vel, const double* inv_mass, const float* F,
                      const float* noise, double dt, double c1, double c2_sqrt_kT, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_md_update, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, mode, pos, vel, inv_mass,
                     F, noise, dt, c1, c2_sqrt_kT);
}

}  // namespace nnp
