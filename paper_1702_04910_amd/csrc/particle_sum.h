// Per-particle sums of force and torque records (Eqs. MEM_TotForce/TotTorque,
// PSM_TotForce/TotTorque) in a fixed order, and the rigid-body step that
// follows the last sum of a rigid-body cycle.  Shared by the reduction kernel
// and the MEM link kernel, which sums its own link forces per chunk: each
// workgroup stores the sum of its chunks, and finish_sums_kernel (the next
// launch; for the link sums, the one after the last sweep of a rigid-body
// step) adds a particle's chunk sums in a fixed order.
#pragma once

#include "common.h"
#include "kernels.h"

namespace lbm {

// ------------------------------------------------------------------------ rigid body
// Forward Euler with dt = n_sub (the number of sweeps per rigid-body step):
//   F_tot = F_h + (rho_p - 1) V g + V f_ext,  U += dt F_tot/m,  X += dt U_old,
//   Omega += dt T/I,  with V = pi D^3/6, m = rho_p V, I = m D^2/10.
// The hydrodynamic force is the average of the n_sub sweeps (Sec. 2.2.4).
__device__ inline void rigid_update(int p, const InstDev* __restrict__ insts, const PartDev& P, unsigned* err) {
  const InstDev& I = insts[P.inst[p]];
  const double dt = (double)I.n_sub;
  double F[3], T[3];
  for (int k = 0; k < 3; ++k) {
    F[k] = P.Facc[3 * p + k] / dt;
    T[k] = P.Tacc[3 * p + k] / dt;
    P.F[3 * p + k] = F[k];
    P.T[3 * p + k] = T[k];
    P.Facc[3 * p + k] = 0.0;
    P.Tacc[3 * p + k] = 0.0;
    P.Xold[3 * p + k] = P.X[3 * p + k];
  }
  bool bad = false;
  for (int k = 0; k < 3; ++k) bad |= !isfinite(F[k]) || !isfinite(T[k]);
  if (!P.fixed[p]) {
    const double D = P.D[p];
    const double V = M_PI * (D * D * D) / 6.0;
    const double m = P.rho[p] * V;
    const double inertia = m * D * D / 10.0;
    const double L[3] = {(double)I.nx, (double)I.ny, (double)I.nz};
    double Un[3], Xn[3], On[3];
    for (int k = 0; k < 3; ++k) {
      const double ftot = (F[k] + (P.rho[p] - 1.0) * V * I.grav[k]) + V * I.fext[k];
      const double u_old = P.U[3 * p + k];
      Un[k] = u_old + dt * ftot / m;
      double x = P.X[3 * p + k] + dt * u_old;
      if (x >= L[k]) x -= L[k];
      if (x < 0.0) x += L[k];
      Xn[k] = x;
      On[k] = P.Om[3 * p + k] + dt * T[k] / inertia;
      // a step of a cell or more (or a non-finite one) leaves the bounds the
      // remap assumes (bounding boxes start at floor(X - R - 2), the cells
      // uncovered since the last remap lie within one cell of the box)
      bad |= !(fabs(dt * u_old) < 1.0) || !isfinite(Un[k]) || !isfinite(On[k]);
    }
    // an unstable step is reported and not taken: the particle keeps a
    // finite position inside the box, so every index derived from it stays
    // in bounds until the caller sees LBMPS_EUNSTABLE
    if (!bad)
      for (int k = 0; k < 3; ++k) {
        P.U[3 * p + k] = Un[k];
        P.X[3 * p + k] = Xn[k];
        P.Om[3 * p + k] = On[k];
      }
  }
  if (bad) atomicOr(err, (unsigned)ERR_UNSTABLE);
}

// Sum of the per-thread 6-vectors acc over the workgroup: a butterfly over the
// 64 lanes of each wave, then the waves in order.  Every thread gets the sum.
__device__ __forceinline__ void block_sum6(const double (&acc)[6], double (&s)[6]) {
  __shared__ double wsum[SUM_THREADS / 64][6];
  double v[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double x = acc[k];
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    v[k] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) wsum[wave][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = 0;
  for (int w = 0; w < SUM_THREADS / 64; ++w)
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] += wsum[w][k];
  __syncthreads();  // wsum may be reused
}

// Workgroup kb's chunk sum s of list position j, kept for finish_sums_kernel
// (partial rows are nb wide).
__device__ __forceinline__ void store_chunk_sum(int j, int kb, int nb, const double (&s)[6],
                                                double* __restrict__ partial) {
  if (threadIdx.x == 0) {
    double* mine = partial + ((long long)j * nb + kb) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) mine[k] = s[k];
  }
}

}  // namespace lbm
