// Particle-side kernels: device-wide exclusive scan used to compact the
// per-bounding-box record lists, the per-particle force/torque reduction
// (Eqs. MEM_TotForce/TotTorque and PSM_TotForce/TotTorque) and the explicit
// Euler rigid-body update (Sec. 4.1).
#include "common.h"
#include "kernels.h"

namespace lbm {

// ------------------------------------------------------------------------ scan
// One workgroup of 1024 threads walks the array in tiles of 8192 entries:
// a coalesced load into LDS, a scan of 8 consecutive entries per thread, a
// wave-shuffle scan of the thread sums and a 16-entry scan of the wave sums,
// then a coalesced store.  Integer sums: the result is exact and independent
// of scheduling.
constexpr int SCAN_TILE = 8192;

__global__ __launch_bounds__(1024) void scan_kernel(const int* __restrict__ totals, int* __restrict__ offsets, int m,
                                                    int side, int nlist, int* __restrict__ begin,
                                                    int* __restrict__ end, int* __restrict__ count, int cap,
                                                    unsigned* err, unsigned err_bit) {
  __shared__ int tile[SCAN_TILE];
  __shared__ long long wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  long long carry = 0;
  for (int base = 0; base < m; base += SCAN_TILE) {
    const int n = min(SCAN_TILE, m - base);
    for (int i = t; i < SCAN_TILE; i += 1024) tile[i] = i < n ? totals[base + i] : 0;
    __syncthreads();
    int v[8];
    long long s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = tile[8 * t + k];
      s += v[k];
    }
    long long x = s;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
      long long z = lane < 16 ? wsum[lane] : 0;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const long long y = __shfl_up(z, off, 64);
        if (lane >= off) z += y;
      }
      if (lane < 16) wsum[lane] = z;
    }
    __syncthreads();
    long long run = carry + (x - s) + (w > 0 ? wsum[w - 1] : 0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      tile[8 * t + k] = (int)run;
      run += v[k];
    }
    carry += wsum[15];
    __syncthreads();
    for (int i = t; i < n; i += 1024) offsets[base + i] = tile[i];
    __syncthreads();
  }
  const long long total = carry;
  if (t == 0) {
    *count = (int)(total < cap ? total : cap);
    if (total > cap) atomicOr(err, err_bit);
  }
  __syncthreads();
  for (int j = t; j < nlist; j += 1024) {
    const int b0 = offsets[j * side];
    const int e0 = offsets[j * side + side - 1] + totals[j * side + side - 1];
    begin[j] = min(b0, cap);
    end[j] = min(e0, cap);
  }
}

hipError_t launch_scan(const int* totals, int* offsets, int m, int side, int nlist, int* begin, int* end, int* count,
                       int cap, unsigned* err, unsigned err_bit, hipStream_t st) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, totals, offsets, m, side, nlist, begin, end, count, cap,
                     err, err_bit);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ reduction
// Workgroup j sums the records [base + begin[j], base + end[j]) (6 components,
// component k of record i at out[k * ostride + i]) in a
// fixed order: strided per-thread partial sums, a butterfly over the 64 lanes of
// each wave, then the waves in order.  The result is added to Facc/Tacc.
constexpr int RED_THREADS = 256;  // fixed: the summation order must not depend on the particle count
__global__ __launch_bounds__(RED_THREADS) void reduce_kernel(const int* __restrict__ list, const int* __restrict__ begin,
                                                     const int* __restrict__ end, int base,
                                                     const double* __restrict__ out, long long ostride,
                                                     PartDev parts) {
  const int j = blockIdx.x;
  const int p = list[j];
  const int b = base + begin[j], e = base + end[j];
  double acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
  for (int i = b + (int)threadIdx.x; i < e; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += out[k * ostride + i];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double v = acc[k];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    acc[k] = v;
  }
  __shared__ double wsum[RED_THREADS / 64][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) wsum[wave][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) / 64;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int w = 0; w < nw; ++w)
      for (int k = 0; k < 6; ++k) s[k] += wsum[w][k];
    for (int k = 0; k < 3; ++k) {
      parts.Facc[3 * p + k] += s[k];
      parts.Tacc[3 * p + k] += s[3 + k];
    }
  }
}

hipError_t launch_reduce(const int* list, int nlist, const int* begin, const int* end, int base, const double* out,
                         long long ostride, PartDev parts, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(nlist), dim3(RED_THREADS), 0, st, list, begin, end, base, out, ostride,
                     parts);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ rigid body
// Forward Euler with dt = n_sub (the number of sweeps per rigid-body step):
//   F_tot = F_h + (rho_p - 1) V g + V f_ext,  U += dt F_tot/m,  X += dt U_old,
//   Omega += dt T/I,  with V = pi D^3/6, m = rho_p V, I = m D^2/10.
// The hydrodynamic force is the average of the n_sub sweeps (Sec. 2.2.4).
__global__ void rigid_kernel(const int* __restrict__ list, int nlist, const InstDev* __restrict__ insts, PartDev P,
                             unsigned* err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlist) return;
  const int p = list[j];
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

hipError_t launch_rigid(const int* list, int nlist, const InstDev* insts, PartDev parts, unsigned* err,
                        hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(rigid_kernel, dim3((nlist + 127) / 128), dim3(128), 0, st, list, nlist, insts, parts, err);
  return hipGetLastError();
}

}  // namespace lbm
