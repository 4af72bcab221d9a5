// Per-particle sums of force and torque records (Eqs. MEM_TotForce/TotTorque,
// PSM_TotForce/TotTorque) in a fixed order, and the rigid-body step that
// follows the last sum of a rigid-body cycle.  Shared by the reduction kernel
// and the MEM link kernel, which sums its own link forces.
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
    for (int k = 0; k < 3; ++k) {
      const double ftot = (F[k] + (P.rho[p] - 1.0) * V * I.grav[k]) + V * I.fext[k];
      const double u_old = P.U[3 * p + k];
      P.U[3 * p + k] = u_old + dt * ftot / m;
      double x = P.X[3 * p + k] + dt * u_old;
      if (x >= L[k]) x -= L[k];
      if (x < 0.0) x += L[k];
      P.X[3 * p + k] = x;
      P.Om[3 * p + k] = P.Om[3 * p + k] + dt * T[k] / inertia;
      bad |= !isfinite(P.U[3 * p + k]) || fabs(dt * u_old) >= 1.0;
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

// Called by every thread of the parts_n workgroups (index kb < parts_n) that
// hold a chunk sum s of particle p (list position j).  With one workgroup the
// sum goes straight to Facc/Tacc; otherwise each stores its sum in
// partial[(j * nb + kb) * 6 ..], and the one that arrives last at arrivals[j]
// adds all of them in workgroup order and resets the counter.  With insts !=
// nullptr the finishing thread then takes the rigid-body step.
__device__ __forceinline__ void finish_particle_sum(int j, int p, const double (&s)[6], int parts_n, int kb, int nb,
                                                    double* __restrict__ partial, unsigned* __restrict__ arrivals,
                                                    const PartDev& parts, const InstDev* __restrict__ insts,
                                                    unsigned* err) {
  if (parts_n == 1) {
    if (threadIdx.x == 0) {
      for (int k = 0; k < 3; ++k) {
        parts.Facc[3 * p + k] += s[k];
        parts.Tacc[3 * p + k] += s[3 + k];
      }
      if (insts) rigid_update(p, insts, parts, err);
    }
    return;
  }
  __shared__ int last;
  if (threadIdx.x == 0) {
    double* mine = partial + ((long long)j * nb + kb) * 6;
    for (int k = 0; k < 6; ++k) mine[k] = s[k];
    __threadfence();
    last = atomicAdd(&arrivals[j], 1u) == (unsigned)(parts_n - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // every chunk sum is loaded at once (one double per thread), then added in order
  __shared__ double ps[SUM_THREADS];
  constexpr int PER = SUM_THREADS / 6;  // chunk sums per round
  double tot[6] = {0, 0, 0, 0, 0, 0};
  for (int k0 = 0; k0 < parts_n; k0 += PER) {
    const int n = min(PER, parts_n - k0);
    if ((int)threadIdx.x < 6 * n)
      ps[threadIdx.x] = __hip_atomic_load(partial + ((long long)j * nb + k0) * 6 + threadIdx.x, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int k = 0; k < 6; ++k) tot[k] += ps[6 * i + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      parts.Facc[3 * p + k] += tot[k];
      parts.Tacc[3 * p + k] += tot[3 + k];
    }
    arrivals[j] = 0;
    if (insts) rigid_update(p, insts, parts, err);
  }
}

}  // namespace lbm
