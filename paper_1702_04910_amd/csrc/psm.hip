// Partially saturated cells coupling (Sec. 2.3): supersampled solid volume
// fractions (Sec. 2.3.2), the (cell, particle) overlap list, and the PSM
// collision of the overlapped cells (Eqs. PSM, PSM_B1/B2, PSM_M1..M3,
// LBM_Collide_PSM) with the per-pair force and torque terms of
// Eqs. PSM_TotForce/TotTorque.
//
// Geometry conventions: cell centres at index + 1/2, minimum-image
// displacements, a sample point is inside when ((dx*dx + dy*dy) + dz*dz) <= R^2
// evaluated without fused multiply-add, sample points at the centres of an
// n^3 sub-cell grid.  The recursive count classifies octree blocks of sample
// points by their farthest and nearest sample point; both counts are exact
// integers and equal.
#include <algorithm>
#include <climits>

#include "bbox.h"
#include "common.h"
#include "kernels.h"
#include "particle_sum.h"
#include "psm_cell.h"

namespace lbm {


// ((x^2 + y^2) + z^2), each operation rounded on its own (no fused multiply-add).
__device__ __forceinline__ double sq3(double x, double y, double z) {
#pragma clang fp contract(off)
  return (x * x + y * y) + z * z;
}

__device__ __forceinline__ double sample_off(int a, int n) { return __dadd_rn(__ddiv_rn((double)a + 0.5, (double)n), -0.5); }

// Whole-block classification: 1 all inside, -1 all outside, 0 mixed.
__device__ __forceinline__ int classify(const double (&lo)[3], const double (&hi)[3], double R2) {
  double f[3], nr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = fabs(lo[k]), b = fabs(hi[k]);
    f[k] = a > b ? a : b;
    nr[k] = (lo[k] <= 0.0 && 0.0 <= hi[k]) ? 0.0 : (a < b ? a : b);
  }
  if (sq3(f[0], f[1], f[2]) <= R2) return 1;
  if (sq3(nr[0], nr[1], nr[2]) > R2) return -1;
  return 0;
}

// Per-wave LDS table for the cell being counted: the sample offsets along one
// axis and the squared sample coordinates (d_k + o_a)^2 along each axis.
struct WaveTab {
  double off[64];
  double sq[3][64];
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Fill the table for centre displacement dc (lane a < n writes entry a).
__device__ __forceinline__ void wave_table(const double dc[3], int n, WaveTab& T) {
  const int lane = threadIdx.x & 63;
  wave_sync_lds();  // previous readers are done
  if (lane < n) {
    const double o = sample_off(lane, n);
    T.off[lane] = o;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x = __dadd_rn(dc[k], o);
      T.sq[k][lane] = __dmul_rn(x, x);
    }
  }
  wave_sync_lds();
}

// Octree count over the block of m^3 sample points (m = 2^L) starting at
// (a0, b0, c0), without a stack: the points are walked in Morton order
// (bit 3i of the code -> a, 3i+1 -> b, 3i+2 -> c), and at each position the
// largest aligned sub-block that starts there is classified by its farthest
// and nearest point; a decided sub-block is counted whole and skipped, an
// undecided one is split by retrying one level lower.
__device__ int count_recursive_block(const double dc[3], double R2, const WaveTab& T, int a0, int b0, int c0, int L) {
  const int total = 1 << (3 * L);
  int cnt = 0;
  int i = 0;
  while (i < total) {
    int l = i == 0 ? L : min(L, __builtin_ctz(i) / 3);
    int a = a0, b = b0, c = c0;
    for (int bit = 0; bit < L; ++bit) {
      a += ((i >> (3 * bit)) & 1) << bit;
      b += ((i >> (3 * bit + 1)) & 1) << bit;
      c += ((i >> (3 * bit + 2)) & 1) << bit;
    }
    for (;;) {
      if (l == 0) {
        cnt += __dadd_rn(__dadd_rn(T.sq[0][a], T.sq[1][b]), T.sq[2][c]) <= R2 ? 1 : 0;
        i += 1;
        break;
      }
      const int h = 1 << l;
      double lo[3], hi[3];
      lo[0] = __dadd_rn(dc[0], T.off[a]); hi[0] = __dadd_rn(dc[0], T.off[a + h - 1]);
      lo[1] = __dadd_rn(dc[1], T.off[b]); hi[1] = __dadd_rn(dc[1], T.off[b + h - 1]);
      lo[2] = __dadd_rn(dc[2], T.off[c]); hi[2] = __dadd_rn(dc[2], T.off[c + h - 1]);
      const int cl = classify(lo, hi, R2);
      if (cl != 0) {
        if (cl == 1) cnt += h * h * h;
        i += 1 << (3 * l);
        break;
      }
      --l;
    }
  }
  return cnt;
}

// Sample count of one cut cell, computed by a whole wave: the flat estimator
// gives each lane (a, b) columns of n points along z; the recursive one gives
// each lane one of the 64 octree blocks of (n/4)^3 points (or the flat loop
// for n < 4).  Squared coordinates come from the wave's table, so every point
// test is ((x^2 + y^2) + z^2 <= R^2) with the same roundings as a direct
// evaluation, and both return the exact serial count.
__device__ int wave_count(const double dc[3], double R2, int n, int mode, WaveTab& T) {
  const int lane = threadIdx.x & 63;
  wave_table(dc, n, T);
  int cnt = 0;
  if (mode == EPS_RECURSIVE && n >= 4) {
    const int m = n / 4, L = __builtin_ctz(m);
    cnt = count_recursive_block(dc, R2, T, (lane & 3) * m, ((lane >> 2) & 3) * m, (lane >> 4) * m, L);
  } else {
    // Along z the coordinates dz + o_c increase with c, so their squares fall
    // on [0, k0) (negative coordinates) and rise on [k0, n), and a column's
    // inside points form a suffix of the first range and a prefix of the
    // second: two bisections count them with the exact point tests.
    const int k0 = __popcll(__ballot(lane < n && __dadd_rn(dc[2], T.off[lane]) < 0.0));
    for (int ab = lane; ab < n * n; ab += 64) {
      const double sab = __dadd_rn(T.sq[0][ab % n], T.sq[1][ab / n]);
      int first = k0;  // first inside point of [0, k0)
      if (k0 > 0 && __dadd_rn(sab, T.sq[2][k0 - 1]) <= R2) {
        if (__dadd_rn(sab, T.sq[2][0]) <= R2) {
          first = 0;
        } else {
          int l = 0, h = k0 - 1;  // l outside, h inside
          while (h - l > 1) {
            const int mid = (l + h) >> 1;
            if (__dadd_rn(sab, T.sq[2][mid]) <= R2) h = mid; else l = mid;
          }
          first = h;
        }
      }
      int last = k0;  // one past the last inside point of [k0, n)
      if (k0 < n && __dadd_rn(sab, T.sq[2][k0]) <= R2) {
        if (__dadd_rn(sab, T.sq[2][n - 1]) <= R2) {
          last = n;
        } else {
          int l = k0, h = n - 1;  // l inside, h outside
          while (h - l > 1) {
            const int mid = (l + h) >> 1;
            if (__dadd_rn(sab, T.sq[2][mid]) <= R2) l = mid; else h = mid;
          }
          last = l + 1;
        }
      }
      cnt += (k0 - first) + (last - k0);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  return cnt;
}

// Bounding box of particle p: `side` cells per axis starting at floor(X - R - 2).
__device__ __forceinline__ void bbox_lo(const PartDev& P, int p, int (&lo)[3]) {
  const double R = 0.5 * P.D[p];
#pragma unroll
  for (int k = 0; k < 3; ++k) lo[k] = (int)floor(P.X[3 * p + k] - R - 2.0);
}

__device__ __forceinline__ void centre_disp(const InstDev& I, const PartDev& P, int p, int i, int j, int k,
                                            double (&d)[3]) {
  d[0] = min_image(((double)i + 0.5) - P.X[3 * p + 0], (double)I.nx);
  d[1] = min_image(((double)j + 0.5) - P.X[3 * p + 1], (double)I.ny);
  d[2] = min_image(((double)k + 0.5) - P.X[3 * p + 2], (double)I.nz);
}

// Closed-form estimators of Sec. 2.3.2 other than supersampling.  Edge
// intersection: the covered length of the cell's twelve edges over 12 (axis by
// axis; the two other coordinates at (-,-), (+,-), (-,+), (+,+) half-cells).
__device__ double eps_edge(const double (&d)[3], double R2) {
#pragma clang fp contract(off)
  double total = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double yb = __dadd_rn(d[b], (k & 1) ? 0.5 : -0.5);
      const double zc = __dadd_rn(d[c], (k & 2) ? 0.5 : -0.5);
      const double h2 = __dadd_rn(R2, -__dadd_rn(__dmul_rn(yb, yb), __dmul_rn(zc, zc)));
      if (h2 > 0.0) {
        const double h = sqrt(h2);
        const double lo = fmax(__dadd_rn(d[a], -0.5), -h);
        const double hi = fmin(__dadd_rn(d[a], 0.5), h);
        total = __dadd_rn(total, fmax(0.0, __dadd_rn(hi, -lo)));
      }
    }
  }
  return fmin(1.0, __ddiv_rn(total, 12.0));
}

// Surface distance: 1/2 - (|d| - R), clamped to [0, 1].
__device__ double eps_distance(const double (&d)[3], double R) {
  const double r = sqrt(sq3(d[0], d[1], d[2]));
  return fmin(1.0, fmax(0.0, __dadd_rn(0.5, -__dadd_rn(r, -R))));
}

// Stage 1 of the solid fractions, grid (units, nlist): every bounding-box cell
// of the unit is classified by its farthest and nearest sample point.  Cells
// entirely inside get the full count n^3, entirely outside 0, cut cells the
// marker -1; totals[unit] receives the number of cut cells.  Slots end up
// holding sample counts out of n^3 for every estimator (the learned one
// rounds its prediction to a count).
__global__ __launch_bounds__(256) void psm_classify_kernel(const int* __restrict__ list, int side, int nsplit,
                                                           const InstDev* __restrict__ insts, PartDev P,
                                                           int* __restrict__ slots, int* __restrict__ totals) {
  __shared__ int sh[256];
  const int j = blockIdx.y;
  const int p = list[j];
  const InstDev& I = insts[P.inst[p]];
  int lo[3];
  bbox_lo(P, p, lo);
  const double R = 0.5 * P.D[p];
  const double R2 = __dmul_rn(R, R);
  const int n = I.eps_n;
  const double o0 = sample_off(0, n), o1 = sample_off(n - 1, n);
  const int ext = bbox_extent(P, p, side);
  const int qs = (int)blockDim.x / ext, rs = (int)blockDim.x % ext;
  for (int ub = blockIdx.x; ub < side * nsplit; ub += gridDim.x) {
    const Unit U = unit_of(ub, side, nsplit);
    const int ncu = unit_cells(U, ext);
    const int k = wrap_near(lo[2] + U.z, I.nz);
    const double dz = min_image(((double)k + 0.5) - P.X[3 * p + 2], (double)I.nz);
    int ncut = 0;
    BBOX_FOR_CELLS_STRIDED(c, (int)threadIdx.x, ncu, (int)blockDim.x, qs, rs, U.y0, ext, dy, dx) {
      const int i = wrap_near(lo[0] + dx, I.nx), jj = wrap_near(lo[1] + dy, I.ny);
      const double dc[3] = {min_image(((double)i + 0.5) - P.X[3 * p + 0], (double)I.nx),
                            min_image(((double)jj + 0.5) - P.X[3 * p + 1], (double)I.ny), dz};
      double blo[3], bhi[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        blo[q] = __dadd_rn(dc[q], o0);
        bhi[q] = __dadd_rn(dc[q], o1);
      }
      const int cl = classify(blo, bhi, R2);
      int v = cl == 1 ? n * n * n : (cl == 0 ? -1 : 0);
      if (I.eps_mode >= EPS_EDGE) {  // closed forms: evaluated here, counts out of n^3
        const double e = I.eps_mode == EPS_EDGE ? eps_edge(dc, R2) : eps_distance(dc, R);
        v = (int)rint(e * ((double)n * n * n));
      }
      slots[slot_index(j, side, U.z, dy, dx)] = v;
      ncut += v < 0 ? 1 : 0;
    }
    int total;
    block_excl_scan256(ncut, sh, &total);
    if (threadIdx.x == 0) totals[j * (side * nsplit) + ub] = total;
  }
}

// Exclusive prefix count of a 0/1 flag over the 256 threads of a workgroup
// (thread order) and its total, from the waves' ballots.
__device__ __forceinline__ int block_flag_scan256(bool f, int* sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long m = __ballot(f);
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) sh[w] = __popcll(m);
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int s = sh[k];
    before += k < w ? s : 0;
    all += s;
  }
  *total = all;
  __syncthreads();  // sh is reused by the next round
  return before + below;
}

// The cells of a unit in rounds of 256 consecutive cells, thread t taking cell
// c = 256 r + t of round r (coalesced reads of the slots and writes of the
// lists); the (row, column) cursor (dy, dx) steps by 256 cells per round.
// Every thread runs every round (the rounds hold workgroup scans); in_unit
// says whether its cell exists.
#define UNIT_ROUNDS(c0, ncu, y0, ext, dy, dx, in_unit)                                            \
  for (int c0 = 0, dy = (y0) + (int)threadIdx.x / (ext), dx = (int)threadIdx.x % (ext), in_unit = 0; \
       c0 < (ncu) && ((in_unit = c0 + (int)threadIdx.x < (ncu)), true);                            \
       c0 += 256, dx += 256 % (ext), dy += 256 / (ext), (dx >= (ext) ? (dx -= (ext), ++dy) : 0))

// Stage 1b: the cut cells of each unit, in cell order, at the unit's scanned
// offset: slot index, particle and centre displacement.
__global__ __launch_bounds__(256) void psm_cut_fill_kernel(const int* __restrict__ list, int side, int nsplit,
                                                           const InstDev* __restrict__ insts, PartDev P,
                                                           const int* __restrict__ slots,
                                                           const int* __restrict__ offsets, CutDev cuts, int cap) {
  __shared__ int sh[256];
  const int j = blockIdx.y;
  const int p = list[j];
  const InstDev& I = insts[P.inst[p]];
  int lo[3];
  bbox_lo(P, p, lo);
  const int ext = bbox_extent(P, p, side);
  for (int ub = blockIdx.x; ub < side * nsplit; ub += gridDim.x) {
    const Unit U = unit_of(ub, side, nsplit);
    const int ncu = unit_cells(U, ext);
    int base = offsets[j * (side * nsplit) + ub];
    UNIT_ROUNDS(c0, ncu, U.y0, ext, dy, dx, in_unit) {
      const long long si = slot_index(j, side, U.z, dy, dx);
      const bool cut = in_unit && slots[si] < 0;
      int total;
      const int pos = base + block_flag_scan256(cut, sh, &total);
      if (cut && pos < cap) {
        const int i = wrap_near(lo[0] + dx, I.nx), jj = wrap_near(lo[1] + dy, I.ny), k = wrap_near(lo[2] + U.z, I.nz);
        double dc[3];
        centre_disp(I, P, p, i, jj, k, dc);
        cuts.slot[pos] = si;
        cuts.p[pos] = p;
        cuts.use[pos] = 0;
        cuts.d[3 * pos] = dc[0];
        cuts.d[3 * pos + 1] = dc[1];
        cuts.d[3 * pos + 2] = dc[2];
      }
      base += total;
    }
  }
}

// Stage 2 (supersampling): one wave per cut cell.  With the learned estimator
// only cells whose radius lies outside the trained range are evaluated here
// (fallback, flat sampling).
__global__ __launch_bounds__(256) void psm_cut_exact_kernel(const InstDev* __restrict__ insts, PartDev P,
                                                            int* __restrict__ slots, CutDev cuts, int cap,
                                                            double rmin, double rmax) {
  __shared__ WaveTab tab[4];
  const int n_cut = min(*cuts.count, cap);
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < n_cut; t += nw) {
    const int p = cuts.p[t];
    const InstDev& I = insts[P.inst[p]];
    const double R = 0.5 * P.D[p];
    const bool learned = I.eps_mode == EPS_LEARNED;
    if (learned && R >= rmin && R <= rmax) continue;
    const double dc[3] = {cuts.d[3 * t], cuts.d[3 * t + 1], cuts.d[3 * t + 2]};
    const int n = I.eps_n;
    const int cnt = wave_count(dc, __dmul_rn(R, R), n, learned ? EPS_FLAT : I.eps_mode, tab[threadIdx.x >> 6]);
    if ((threadIdx.x & 63) == 0) slots[cuts.slot[t]] = cnt;
  }
}

// Stage 2 (learned): features of every cut cell; `use` flags the cells of
// learned-estimator instances whose radius is inside the trained range.
__global__ void psm_cut_features_kernel(const InstDev* __restrict__ insts, PartDev P, CutDev cuts, int cap,
                                        double rmin, double rmax, float* __restrict__ X) {
  const int n_cut = min(*cuts.count, cap);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cut) return;
  const int p = cuts.p[t];
  const InstDev& I = insts[P.inst[p]];
  const double R = 0.5 * P.D[p];
  const bool use = I.eps_mode == EPS_LEARNED && R >= rmin && R <= rmax;
  cuts.use[t] = use ? 1 : 0;
  const double d[3] = {cuts.d[3 * t], cuts.d[3 * t + 1], cuts.d[3 * t + 2]};
  float x[8];
  eps_features(d, R, x);
#pragma unroll
  for (int k = 0; k < 8; ++k) X[8LL * t + k] = x[k];
}

// The network's eps (clamped to [0, 1]) as the nearest count out of n^3.
__global__ void psm_cut_scatter_kernel(const InstDev* __restrict__ insts, PartDev P, CutDev cuts, int cap,
                                       const float* __restrict__ y, int* __restrict__ slots) {
  const int n_cut = min(*cuts.count, cap);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_cut || !cuts.use[t]) return;
  const int n = insts[P.inst[cuts.p[t]]].eps_n;
  slots[cuts.slot[t]] = (int)rintf(y[t] * (float)(n * n * n));
}

// Stage 3: number of cells with eps > 0 (count > 0) per work unit.
__global__ __launch_bounds__(256) void psm_unit_totals_kernel(const int* __restrict__ list, int side, int nsplit,
                                                              PartDev P, const int* __restrict__ slots,
                                                              int* __restrict__ totals) {
  __shared__ int sh[256];
  const int j = blockIdx.y;
  const int ext = bbox_extent(P, list[j], side);
  const int qs = (int)blockDim.x / ext, rs = (int)blockDim.x % ext;
  for (int ub = blockIdx.x; ub < side * nsplit; ub += gridDim.x) {
    const Unit U = unit_of(ub, side, nsplit);
    const int ncu = unit_cells(U, ext);
    int local = 0;
    BBOX_FOR_CELLS_STRIDED(c, (int)threadIdx.x, ncu, (int)blockDim.x, qs, rs, U.y0, ext, dy, dx)
      local += slots[slot_index(j, side, U.z, dy, dx)] > 0 ? 1 : 0;
    int total;
    block_excl_scan256(local, sh, &total);
    if (threadIdx.x == 0) totals[j * (side * nsplit) + ub] = total;
  }
}

// Labels for training samples (R, dx, dy, dz): exact eps by flat n^3
// supersampling, one wave per sample.
__global__ __launch_bounds__(256) void psm_label_kernel(const double* __restrict__ rd, long long ns, int n,
                                                        float* __restrict__ eps) {
  __shared__ WaveTab tab[4];
  const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long t = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < ns; t += nw) {
    const double R = rd[4 * t];
    const double dc[3] = {rd[4 * t + 1], rd[4 * t + 2], rd[4 * t + 3]};
    const int cnt = wave_count(dc, __dmul_rn(R, R), n, EPS_FLAT, tab[threadIdx.x >> 6]);
    if ((threadIdx.x & 63) == 0) eps[t] = (float)((double)cnt / ((double)n * n * n));
  }
}

// Error judge of the learned estimator: every `stride`-th cut cell that used
// the network is recounted exactly; stats[0] += |error|, stats[1] = max |error|
// (ordered as bits of a non-negative double), stats[2] += 1.
__global__ __launch_bounds__(256) void psm_judge_kernel(const InstDev* __restrict__ insts, PartDev P,
                                                        const int* __restrict__ slots, CutDev cuts, int cap,
                                                        int stride, double* __restrict__ stats) {
  __shared__ WaveTab tab[4];
  const int n_cut = min(*cuts.count, cap);
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; (long long)k * stride < n_cut; k += nw) {
    const int t = k * stride;
    if (!cuts.use[t]) continue;
    const int p = cuts.p[t];
    const InstDev& I = insts[P.inst[p]];
    const double R = 0.5 * P.D[p];
    const double dc[3] = {cuts.d[3 * t], cuts.d[3 * t + 1], cuts.d[3 * t + 2]};
    const int n = I.eps_n;
    const int cnt = wave_count(dc, __dmul_rn(R, R), n, EPS_FLAT, tab[threadIdx.x >> 6]);
    if ((threadIdx.x & 63) == 0) {
      const double e = fabs((double)(slots[cuts.slot[t]] - cnt) / ((double)n * n * n));
      atomicAdd(&stats[0], e);
      atomicMax((unsigned long long*)&stats[1], (unsigned long long)__double_as_longlong(e));
      atomicAdd(&stats[2], 1.0);
    }
  }
}

hipError_t launch_psm_classify(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                               int* slots, int* totals, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(psm_classify_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts,
                     parts, slots, totals);
  return hipGetLastError();
}

hipError_t launch_psm_cut_fill(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                               const int* slots, const int* offsets, CutDev cuts, int cap, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(psm_cut_fill_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts,
                     parts, slots, offsets, cuts, cap);
  return hipGetLastError();
}

hipError_t launch_psm_cut_exact(const InstDev* insts, PartDev parts, int* slots, CutDev cuts, int cap, double rmin,
                                double rmax, hipStream_t st) {
  hipLaunchKernelGGL(psm_cut_exact_kernel, dim3(2048), dim3(256), 0, st, insts, parts, slots, cuts, cap, rmin, rmax);
  return hipGetLastError();
}

hipError_t launch_psm_cut_features(const InstDev* insts, PartDev parts, CutDev cuts, int cap, double rmin,
                                   double rmax, float* X, hipStream_t st) {
  hipLaunchKernelGGL(psm_cut_features_kernel, dim3((cap + 255) / 256), dim3(256), 0, st, insts, parts, cuts, cap,
                     rmin, rmax, X);
  return hipGetLastError();
}

hipError_t launch_psm_cut_scatter(const InstDev* insts, PartDev parts, CutDev cuts, int cap, const float* y,
                                  int* slots, hipStream_t st) {
  hipLaunchKernelGGL(psm_cut_scatter_kernel, dim3((cap + 255) / 256), dim3(256), 0, st, insts, parts, cuts, cap, y,
                     slots);
  return hipGetLastError();
}

hipError_t launch_psm_unit_totals(const int* list, int nlist, int side, int nsplit, PartDev parts, const int* slots,
                                  int* totals, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(psm_unit_totals_kernel, grid, dim3(256), 0, st, list, side, nsplit, parts, slots, totals);
  return hipGetLastError();
}

hipError_t launch_psm_label(const double* rd, long long ns, int n, float* eps, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<long long>((ns + 3) / 4, 65536);
  hipLaunchKernelGGL(psm_label_kernel, dim3(grid), dim3(256), 0, st, rd, ns, n, eps);
  return hipGetLastError();
}

hipError_t launch_psm_judge(const InstDev* insts, PartDev parts, const int* slots, CutDev cuts, int cap, int stride,
                            double* stats, hipStream_t st) {
  hipLaunchKernelGGL(psm_judge_kernel, dim3(1024), dim3(256), 0, st, insts, parts, slots, cuts, cap, stride, stats);
  return hipGetLastError();
}

// Writes the overlap pairs of each unit in cell order (per-thread contiguous chunks).
__global__ __launch_bounds__(256) void psm_fill_kernel(const int* __restrict__ list, int side, int nsplit,
                                                       const InstDev* __restrict__ insts, PartDev P,
                                                       const int* __restrict__ slots, const int* __restrict__ offsets,
                                                       int cap, PairDev pairs) {
  __shared__ int sh[256];
  const int j = blockIdx.y;
  const int p = list[j];
  const InstDev& I = insts[P.inst[p]];
  int lo[3];
  bbox_lo(P, p, lo);
  const int n = I.eps_n;
  const double nn = (double)n * (double)n * (double)n;
  const double t = I.tau - 0.5;
  const int ext = bbox_extent(P, p, side);
  for (int ub = blockIdx.x; ub < side * nsplit; ub += gridDim.x) {
    const Unit U = unit_of(ub, side, nsplit);
    const int ncu = unit_cells(U, ext);
    int base = offsets[j * (side * nsplit) + ub];
    UNIT_ROUNDS(c0, ncu, U.y0, ext, dy, dx, in_unit) {
      const int v = in_unit ? slots[slot_index(j, side, U.z, dy, dx)] : 0;
      int total;
      const int pos = base + block_flag_scan256(v > 0, sh, &total);
      base += total;
      if (v > 0 && pos < cap) {
        const int i = wrap_near(lo[0] + dx, I.nx), jj = wrap_near(lo[1] + dy, I.ny), k = wrap_near(lo[2] + U.z, I.nz);
        const double eps = (double)v / nn;
        pairs.cell[pos] = (k * I.ny + jj) * I.nx + i;
        pairs.p[pos] = p;
        pairs.eps[pos] = eps;
        pairs.B[pos] = I.psm_b == 1 ? eps : eps * t / ((1.0 - eps) + t);
        pairs.next[pos] = -1;
      }
    }
  }
}

hipError_t launch_psm_fill(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                           const int* slots, const int* offsets, int cap, PairDev pairs, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(psm_fill_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts, parts,
                     slots, offsets, cap, pairs);
  return hipGetLastError();
}

// stage 0: reset the cell map entries of the listed pairs; stage 1: each cell's
// leader is its smallest pair index; stage 2: the other pairs of a cell are
// chained behind the leader (order fixed later by sorting).
__global__ void psm_cellmap_kernel(int stage, const int* __restrict__ count, int cap,
                                   const InstDev* __restrict__ insts, PartDev P, PairDev pairs,
                                   int* __restrict__ cellmap) {
  const int n = min(*count, cap);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int p = pairs.p[i];
    int* cm = cellmap + insts[P.inst[p]].cellmap_off;
    const int c = pairs.cell[i];
    if (stage == 0) {
      cm[c] = INT_MAX;
    } else if (stage == 1) {
      atomicMin(&cm[c], i);
    } else {
      const int L = cm[c];
      if (L != i) pairs.next[i] = atomicExch(&pairs.next[L], i);
    }
  }
}

hipError_t launch_psm_cellmap(int stage, const int* count, int cap, const InstDev* insts, PartDev parts,
                              PairDev pairs, int* cellmap, hipStream_t st) {
  hipLaunchKernelGGL(psm_cellmap_kernel, dim3(1024), dim3(256), 0, st, stage, count, cap, insts, parts, pairs,
                     cellmap);
  return hipGetLastError();
}

// Overlapped cells, visited through their leader pairs in pair order (the
// list is ordered by particle, slab and row, so neighbouring lanes touch
// neighbouring cells and share cache lines).  The post-collision values are
// pushed into dst, or with stage != nullptr stored at stage[stage_at(L, q)]
// (whole cache lines; the next sweep pushes them).  With 16-bit storage they are
// rounded stochastically (keyed by cell and direction), like the overlapped
// cells that the sweep collides inline.  MULTI = false: the cells with a
// single pair, with the solid operator M fixed at compile time (0: per
// instance) -- the common case, compiled for four waves per SIMD where the
// storage is below 8 bytes and M is fixed; MULTI = true: the cells shared by
// several particles.
template <typename S, int M, bool MULTI>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MULTI || M == 0 || sizeof(S) == 8 ? 1 : 4))) void psm_collide_kernel(
    const int* __restrict__ count, int cap, const InstDev* __restrict__ insts, PartDev P, PairDev pairs,
    const int* __restrict__ cellmap, const S* __restrict__ src, S* __restrict__ dst, S* __restrict__ stage,
    long long sstride) {
  using R = typename CompOf<S>::type;
  const int npairs = min(*count, cap);
  for (int L = blockIdx.x * blockDim.x + threadIdx.x; L < npairs; L += gridDim.x * blockDim.x) {
    if ((pairs.next[L] >= 0) != MULTI) continue;  // a single pair's cell has no chain
    const int p0 = pairs.p[L];
    const InstDev& I = insts[P.inst[p0]];
    const int c = pairs.cell[L];
    if (cellmap[I.cellmap_off + c] != L) continue;  // not the cell's leader
    const S* s = src + I.pdf_off;
    S* d = dst + I.pdf_off;
    R g[Q], out[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = Codec<S>::ld(s[pdf_at(c, q)]);
    psm_cell_collide<M, !MULTI, R>(g, out, I, P, pairs, L, c);
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = StochasticRound<S>::apply(out[q], (uint32_t)c * Q + q);
    if (stage) {  // the sweep pushes them
#pragma unroll
      for (int q = 0; q < Q; ++q) stage[stage_at(L, q)] = Codec<S>::st(out[q]);
      continue;
    }
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const int x = c % nx, yz = c / nx, y = yz % ny, z = yz / ny;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int xa = wrapi(x + cx(q), nx), ya = wrapi(y + cy(q), ny), za = wrapi(z + cz(q), nz);
      d[pdf_at(((long long)za * ny + ya) * nx + xa, q)] = Codec<S>::st(out[q]);
    }
  }
}

// Cells of a single pair visited per particle: workgroup (k, j) takes the
// chunks k, k + gridDim.x, ... of RED_CHUNK pairs of list position j's pair
// range, each thread the pairs cb + t, cb + t + SUM_THREADS, ... of a chunk --
// the order in which reduce_kernel reads force records.  A thread adds the
// force/torque terms of its single-pair cells, computed here and kept in
// registers, and the records of its pairs in shared cells (written before by
// the shared-cell launch); the chunk sums are those reduce_kernel would form
// from a complete record array, bit for bit, without writing and reading the
// 48-byte record of every pair.  finish_sums_kernel adds them per particle.
// Built for three waves per SIMD where the storage is below 8 bytes and M is
// fixed (~136 registers): capped at four it spills, and took ~3 % longer.
template <typename S, int M>
__global__ __launch_bounds__(SUM_THREADS)
__attribute__((amdgpu_waves_per_eu(M == 0 || sizeof(S) == 8 ? 1 : 3))) void psm_collide_sum_kernel(
    const int* __restrict__ list, const int* __restrict__ begin, const int* __restrict__ end,
    const InstDev* __restrict__ insts, PartDev P, PairDev pairs, const int* __restrict__ cellmap,
    const S* __restrict__ src, S* __restrict__ dst, S* __restrict__ stage, long long sstride,
    double* __restrict__ partial) {
  using R = typename CompOf<S>::type;
  const int j = blockIdx.y, kb = blockIdx.x, nb = gridDim.x;
  const int b = begin[j], e = end[j];
  const int nch = (e - b + RED_CHUNK - 1) / RED_CHUNK;
  if (kb >= nch) return;  // no pairs for this workgroup; it takes no part
  const InstDev& I = insts[P.inst[list[j]]];
  const S* s = src + I.pdf_off;
  S* d = dst + I.pdf_off;
  double sum[6] = {0, 0, 0, 0, 0, 0};
  for (int ch = kb; ch < nch; ch += nb) {
    const int cb = b + ch * RED_CHUNK, ce = min(e, cb + RED_CHUNK);
    double acc[6] = {0, 0, 0, 0, 0, 0}, t[6];
    for (int L = cb + (int)threadIdx.x; L < ce; L += SUM_THREADS) {
      const int c = pairs.cell[L];
      double ft[6];
      if (pairs.next[L] < 0 && cellmap[I.cellmap_off + c] == L) {  // the cell's only pair
        R g[Q], out[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) g[q] = Codec<S>::ld(s[pdf_at(c, q)]);
        psm_cell_collide<M, true, R, true>(g, out, I, P, pairs, L, c, ft);
#pragma unroll
        for (int q = 0; q < Q; ++q) out[q] = StochasticRound<S>::apply(out[q], (uint32_t)c * Q + q);
        if (stage) {
#pragma unroll
          for (int q = 0; q < Q; ++q) stage[stage_at(L, q)] = Codec<S>::st(out[q]);
        } else {
          const int nx = I.nx, ny = I.ny, nz = I.nz;
          const int x = c % nx, yz = c / nx, y = yz % ny, z = yz / ny;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int xa = wrapi(x + cx(q), nx), ya = wrapi(y + cy(q), ny), za = wrapi(z + cz(q), nz);
            d[pdf_at(((long long)za * ny + ya) * nx + xa, q)] = Codec<S>::st(out[q]);
          }
        }
      } else {  // a pair of a shared cell: its record
#pragma unroll
        for (int k = 0; k < 6; ++k) ft[k] = pairs.out[k * pairs.ostride + L];
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] += ft[k];
    }
    block_sum6(acc, t);
#pragma unroll
    for (int k = 0; k < 6; ++k) sum[k] += t[k];
  }
  store_chunk_sum(j, kb, nb, sum, partial);
}

#define LBM_DISPATCH(prec, CALL)                          \
  switch (prec) {                                         \
    case PREC_FP64: { using S = double; CALL; } break;    \
    case PREC_FP32: { using S = float; CALL; } break;     \
    case PREC_FP16: { using S = _Float16; CALL; } break;  \
    case PREC_BF16: { using S = __bf16; CALL; } break;    \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t launch_psm_collide(int prec, int psm_m, const int* count, int cap, const InstDev* insts, PartDev parts,
                              PairDev pairs, const int* cellmap, const void* src, void* dst, void* stage,
                              long long sstride, bool shared_only, hipStream_t st, const PsmSums* sums) {
  const int grid = 2048;
#define PSM_COLLIDE(MM, MULTI)                                                                                      \
  LBM_DISPATCH(prec, hipLaunchKernelGGL((psm_collide_kernel<S, MM, MULTI>), dim3(grid), dim3(256), 0, st, count, cap, \
                                        insts, parts, pairs, cellmap, (const S*)src, (S*)dst, (S*)stage, sstride))
  if (sums && !shared_only) {
    if (sums->nlist <= 0) return hipSuccess;
    PSM_COLLIDE(0, true);  // shared cells first: their records are summed below
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(sums->width, sums->nlist);
#define PSM_SUM(MM)                                                                                                \
  LBM_DISPATCH(prec, hipLaunchKernelGGL((psm_collide_sum_kernel<S, MM>), g2, dim3(SUM_THREADS), 0, st, sums->list,  \
                                        sums->begin, sums->end, insts, parts, pairs, cellmap, (const S*)src,       \
                                        (S*)dst, (S*)stage, sstride, sums->partial))
    switch (psm_m) {
      case 1: PSM_SUM(1); break;
      case 2: PSM_SUM(2); break;
      case 3: PSM_SUM(3); break;
      default: PSM_SUM(0); break;
    }
#undef PSM_SUM
    return hipGetLastError();
  }
  if (!shared_only) {
    switch (psm_m) {
      case 1: PSM_COLLIDE(1, false); break;
      case 2: PSM_COLLIDE(2, false); break;
      case 3: PSM_COLLIDE(3, false); break;
      default: PSM_COLLIDE(0, false); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  PSM_COLLIDE(0, true);
#undef PSM_COLLIDE
  return hipGetLastError();
}

// Eq. MacVel_PSM for the overlapped cells of instance `inst` within [c0, c0 + n):
// u = (1 - B)(U + f_ext/2) + sum_s B_s v_s, written over the fluid velocity in out.
template <typename S>
__global__ void psm_fields_kernel(const int* __restrict__ count, int cap, const InstDev* __restrict__ insts,
                                  PartDev P, PairDev pairs, const int* __restrict__ cellmap,
                                  const S* __restrict__ buf, int inst, long long c0, long long n,
                                  double* __restrict__ out) {
  const int npairs = min(*count, cap);
  for (int L = blockIdx.x * blockDim.x + threadIdx.x; L < npairs; L += gridDim.x * blockDim.x) {
    const int p0 = pairs.p[L];
    if (P.inst[p0] != inst) continue;
    const InstDev& I = insts[inst];
    const int c = pairs.cell[L];
    if (c < c0 || c >= c0 + n) continue;
    if (cellmap[I.cellmap_off + c] != L) continue;
    int mem[KMAX];
    const int k = gather_members(pairs, L, mem);
    const long long N = I.ncell;
    const S* s = buf + I.pdf_off;
    double jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const double gq = (double)Codec<S>::ld(s[pdf_at(c, q)]);
      jx += cx(q) * gq;
      jy += cy(q) * gq;
      jz += cz(q) * gq;
    }
    double Bs[KMAX], Bsum = 0;
    for (int m = 0; m < k; ++m) {
      Bs[m] = pairs.B[mem[m]];
      Bsum += Bs[m];
    }
    if (Bsum > 1.0) {
      for (int m = 0; m < k; ++m) Bs[m] = Bs[m] * (1.0 / Bsum);
      Bsum = 0.0;
      for (int m = 0; m < k; ++m) Bsum += Bs[m];
    }
    const int x = c % I.nx, yz = c / I.nx, y = yz % I.ny, z = yz / I.ny;
    double u[3] = {(1.0 - Bsum) * (jx + 0.5 * I.fext[0]), (1.0 - Bsum) * (jy + 0.5 * I.fext[1]),
                   (1.0 - Bsum) * (jz + 0.5 * I.fext[2])};
    for (int m = 0; m < k; ++m) {
      const int pm = pairs.p[mem[m]];
      double r[3];
      r[0] = min_image(((double)x + 0.5) - P.X[3 * pm + 0], (double)I.nx);
      r[1] = min_image(((double)y + 0.5) - P.X[3 * pm + 1], (double)I.ny);
      r[2] = min_image(((double)z + 0.5) - P.X[3 * pm + 2], (double)I.nz);
      const double* Up = P.U + 3 * pm;
      const double* Wp = P.Om + 3 * pm;
      u[0] += Bs[m] * (Up[0] + (Wp[1] * r[2] - Wp[2] * r[1]));
      u[1] += Bs[m] * (Up[1] + (Wp[2] * r[0] - Wp[0] * r[2]));
      u[2] += Bs[m] * (Up[2] + (Wp[0] * r[1] - Wp[1] * r[0]));
    }
    const long long i = c - c0;
    out[n + i] = u[0];
    out[2 * n + i] = u[1];
    out[3 * n + i] = u[2];
  }
}

hipError_t launch_psm_fields(int prec, const int* count, int cap, const InstDev* insts, PartDev parts, PairDev pairs,
                             const int* cellmap, const void* buf, int inst, long long c0, long long n, double* out,
                             hipStream_t st) {
  LBM_DISPATCH(prec, hipLaunchKernelGGL(psm_fields_kernel<S>, dim3(512), dim3(256), 0, st, count, cap, insts, parts,
                                        pairs, cellmap, (const S*)buf, inst, c0, n, out));
  return hipGetLastError();
}

}  // namespace lbm
