// Particle-side kernels: device-wide exclusive scan used to compact the
// per-bounding-box record lists, the per-particle force/torque reduction
// (Eqs. MEM_TotForce/TotTorque and PSM_TotForce/TotTorque) and the explicit
// Euler rigid-body update (Sec. 4.1).
#include "common.h"
#include "kernels.h"
#include "particle_sum.h"

namespace lbm {

// ------------------------------------------------------------------------ scan
// One workgroup of 1024 threads walks the array in tiles of 8192 entries:
// a coalesced load into LDS, a scan of 8 consecutive entries per thread, a
// wave-shuffle scan of the thread sums and a 16-entry scan of the wave sums,
// then a coalesced store.  Integer sums: the result is exact and independent
// of scheduling.
constexpr int SCAN_TILE = 8192;

__device__ void scan_body(const int* __restrict__ totals, int* __restrict__ offsets, int m, int side, int nlist,
                          int* __restrict__ begin, int* __restrict__ end, int* __restrict__ count, int cap,
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
  __syncthreads();
}

__global__ __launch_bounds__(1024) void scan_kernel(const int* __restrict__ totals, int* __restrict__ offsets, int m,
                                                    int side, int nlist, int* __restrict__ begin,
                                                    int* __restrict__ end, int* __restrict__ count, int cap,
                                                    unsigned* err, unsigned err_bit) {
  scan_body(totals, offsets, m, side, nlist, begin, end, count, cap, err, err_bit);
}

__global__ __launch_bounds__(1024) void scan2_kernel(const int* __restrict__ totals, int* __restrict__ offsets, int m,
                                                     int side, int nlist, int* __restrict__ begin,
                                                     int* __restrict__ end, int* __restrict__ count, int cap,
                                                     unsigned err_bit, const int* __restrict__ totals2,
                                                     int* __restrict__ offsets2, int m2, int side2, int nlist2,
                                                     int* __restrict__ begin2, int* __restrict__ end2,
                                                     int* __restrict__ count2, int cap2, unsigned err_bit2,
                                                     unsigned* err) {
  // the two scans are independent: one workgroup each, running side by side
  if (blockIdx.x == 0)
    scan_body(totals, offsets, m, side, nlist, begin, end, count, cap, err, err_bit);
  else
    scan_body(totals2, offsets2, m2, side2, nlist2, begin2, end2, count2, cap2, err, err_bit2);
}

hipError_t launch_scan(const int* totals, int* offsets, int m, int side, int nlist, int* begin, int* end, int* count,
                       int cap, unsigned* err, unsigned err_bit, hipStream_t st) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, totals, offsets, m, side, nlist, begin, end, count, cap,
                     err, err_bit);
  return hipGetLastError();
}

hipError_t launch_scan2(const int* totals, int* offsets, int m, int side, int nlist, int* begin, int* end, int* count,
                        int cap, unsigned err_bit, const int* totals2, int* offsets2, int m2, int side2, int nlist2,
                        int* begin2, int* end2, int* count2, int cap2, unsigned err_bit2, unsigned* err,
                        hipStream_t st) {
  hipLaunchKernelGGL(scan2_kernel, dim3(2), dim3(1024), 0, st, totals, offsets, m, side, nlist, begin, end, count, cap,
                     err_bit, totals2, offsets2, m2, side2, nlist2, begin2, end2, count2, cap2, err_bit2, err);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ reduction
// The records [base + begin[j], base + end[j]) of particle list[j] (6
// components, component k of record i at out[k * ostride + i]) are cut into
// chunks of RED_CHUNK consecutive records; workgroup (k, j) sums chunks k,
// k + gridDim.x, ... in a fixed order (strided per-thread sums, then
// block_sum6) and stores the result; finish_sums_kernel adds the workgroup
// sums in a fixed order.  The order depends only on the record count, so results
// repeat bit for bit.
__global__ __launch_bounds__(SUM_THREADS) void reduce_kernel(const int* __restrict__ begin,
                                                     const int* __restrict__ end, int base,
                                                     const double* __restrict__ out, long long ostride,
                                                     double* __restrict__ partial) {
  const int j = blockIdx.y, kb = blockIdx.x, nb = gridDim.x;
  const int b = base + begin[j], e = base + end[j];
  const int nch = (e - b + RED_CHUNK - 1) / RED_CHUNK;
  if (kb >= nch) return;  // no records for this workgroup; it takes no part
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int ch = kb; ch < nch; ch += nb) {
    const int cb = b + ch * RED_CHUNK, ce = min(e, cb + RED_CHUNK);
    double acc[6] = {0, 0, 0, 0, 0, 0}, t[6];
#pragma unroll 4
    for (int i = cb + (int)threadIdx.x; i < ce; i += SUM_THREADS) {
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] += out[k * ostride + i];
    }
    block_sum6(acc, t);
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] += t[k];
  }
  store_chunk_sum(j, kb, nb, s, partial);
}

// One wave per particle: the min(ceil(n / chunk), width) chunk sums of list
// position j (n = end[j] - begin[j] records) in each of nsets sets (set s at
// partial + s * set_stride; the MEM link sums of the n_sub sweeps of one
// rigid-body step): lane l loads chunks l, l + 64, ... (all loads of a lane in
// flight together) and adds them in that order, then a butterfly over the 64
// lanes forms the set's total, which is added to Facc/Tacc, set after set.
// The order depends only on the chunk count.  With insts != nullptr the
// rigid-body step follows.
constexpr int FIN_WAVES = 4;
__global__ __launch_bounds__(64 * FIN_WAVES) void finish_sums_kernel(const int* __restrict__ list, int nlist,
                                                                     const int* __restrict__ begin,
                                                                     const int* __restrict__ end, int chunk,
                                                                     int width, const double* __restrict__ partial,
                                                                     int nsets, long long set_stride,
                                                                     PartDev parts, const InstDev* __restrict__ insts,
                                                                     unsigned* err) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * FIN_WAVES + w;
  if (j >= nlist) return;  // whole wave
  const int p = list[j];  // requested with the record range, used after the sums
  const int n = end[j] - begin[j];
  const int parts_n = min((n + chunk - 1) / chunk, width);
  for (int s = 0; s < nsets; ++s) {
    double tot[6] = {0, 0, 0, 0, 0, 0};
    for (int i = lane; i < parts_n; i += 64) {
      const double* src = partial + s * set_stride + ((long long)j * width + i) * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) tot[k] += src[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
      for (int m = 32; m >= 1; m >>= 1) tot[k] += __shfl_xor(tot[k], m, 64);
    if (lane == 0 && parts_n > 0)
      for (int k = 0; k < 3; ++k) {
        parts.Facc[3 * p + k] += tot[k];
        parts.Tacc[3 * p + k] += tot[3 + k];
      }
  }
  if (lane == 0 && insts) rigid_update(p, insts, parts, err);
}

hipError_t launch_finish_sums(const int* list, int nlist, const int* begin, const int* end, int chunk, int width,
                              const double* partial, int nsets, long long set_stride, PartDev parts,
                              const InstDev* rigid_insts, unsigned* err, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(finish_sums_kernel, dim3((nlist + FIN_WAVES - 1) / FIN_WAVES), dim3(64 * FIN_WAVES), 0, st, list,
                     nlist, begin, end, chunk, width, partial, nsets, set_stride, parts, rigid_insts, err);
  return hipGetLastError();
}

hipError_t launch_reduce(const int* list, int nlist, const int* begin, const int* end, int base, const double* out,
                         long long ostride, PartDev parts, int nchunk_blocks, double* partial,
                         const InstDev* rigid_insts, unsigned* err, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(nchunk_blocks, nlist), dim3(SUM_THREADS), 0, st, begin, end, base, out,
                     ostride, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish_sums(list, nlist, begin, end, RED_CHUNK, nchunk_blocks, partial, 1, 0, parts, rigid_insts, err,
                            st);
}

}  // namespace lbm
