// Launchers of the lbmps device kernels (internal interface between the
// kernel translation units and the C-ABI layer).
#pragma once

#include "common.h"

namespace lbm {

// Workgroups along x for the per-unit bounding-box kernels (grid y = particle
// list): about 8192 in all, each looping over units x, x + grid, ...
inline int unit_grid(int units, int nlist) {
  const int g = nlist > 0 ? (8192 + nlist - 1) / nlist : 1;
  return units < g ? units : g;
}

// ---- sweep.hip
// sweep_flags: bit 0 non-temporal loads; bit 1 collide PSM cells inside the
// sweep; bit 2 collide them in the separate overlap kernel after the sweep;
// bit 3 the sweep compiled for six waves per SIMD (4- and 2-byte storage);
// bit 4 collide them in the overlap kernel before the sweep into a staging
// array that the sweep pushes (none of bits 1, 2, 4: chosen from the expected
// share of overlapped cells); bits 5-6 cap the sweep workgroups resident per
// CU (0 no cap, 1 three, 2 two; 3 is invalid) by reserving LDS; bit 7 every
// sweep thread handles two x-adjacent cells (needs even nx; not used with bit 3
// or while the sweep handles overlapped cells, bits 1 and 4); bit 8 four
// x-adjacent cells per thread in 8-byte words (2-byte storage, nx a multiple
// of 4; not with bits 3 or 7; not used while the sweep handles overlapped
// cells).  Results never depend on them.
enum {
  SWEEP_NT_LOADS = 1, SWEEP_PSM_FUSED = 2, SWEEP_PSM_SEPARATE = 4, SWEEP_OCC6 = 8, SWEEP_PSM_STAGED = 16,
  SWEEP_WG_CAP_SHIFT = 5, SWEEP_WG_CAP_MASK = 3 << SWEEP_WG_CAP_SHIFT, SWEEP_CELL_PAIRS = 128, SWEEP_CELL_QUADS = 256,
  SWEEP_FLAGS_ALL = 511,
  SWEEP_PSM_MODES = SWEEP_PSM_FUSED | SWEEP_PSM_SEPARATE | SWEEP_PSM_STAGED
};
constexpr int LDS_PER_CU = 160 * 1024;
// LDS a sweep workgroup reserves: what its staging needs, raised under a cap
// so that only (4 - cap) workgroups fit on one CU.
inline size_t sweep_lds_bytes(size_t need, int flags) {
  const int cap = (flags & SWEEP_WG_CAP_MASK) >> SWEEP_WG_CAP_SHIFT;
  if (cap == 0) return need;
  const size_t floor = (size_t)LDS_PER_CU / (size_t)(5 - cap) + 256;
  return need > floor ? need : floor;
}
// psm_mode: 0 no PSM cells (or they are re-collided afterwards), 1 single-particle cells inline (shared ones are
// re-collided afterwards), 2 staged (stage[stage_at(leader pair, q)], written by launch_psm_collide).
hipError_t launch_sweep(int prec, const InstDev* insts, const int4* tiles, int ntiles, int grid, int block,
                        int max_tile_cells, int flags, int psm_mode, const void* src, void* dst, const int* cellmap,
                        PairDev pairs, PartDev parts, const void* stage, long long sstride, hipStream_t st);
// Collide-and-push of the first min(*count, cap) cells of the MEM refill list (rcell, rpart) from src to dst, with
// the sweep's arithmetic: repairs a sweep that ran while those cells were being refilled.
hipError_t launch_resweep_cells(int prec, const int* count, int cap, const int* rcell, const int* rpart,
                                const InstDev* insts, PartDev parts, const void* src, void* dst, hipStream_t st);
constexpr int SWEEP_LDS_LIMIT = 64 * 1024;  // bytes of LDS staging per sweep workgroup
hipError_t launch_init_eq(int prec, void* buf, long long N, double rho, const double u[3], hipStream_t st);
hipError_t launch_to_f64(int prec, const void* a, int q, long long c0, double* b, long long n, hipStream_t st);
hipError_t launch_from_f64(int prec, const double* a, void* b, int q, long long c0, long long n, hipStream_t st);
hipError_t launch_fields(int prec, const void* buf, long long N, long long c0, long long n, const int* owner,
                         const double f[3], double* out, hipStream_t st);

// ---- particles.hip
// Exclusive scan of `totals` (length m) into `offsets`; writes the grand total to
// *count and, for each of the nlist bounding boxes of `side` slabs, its record range
// [begin, end).  Sets err_bit in *err when the total exceeds cap.
hipError_t launch_scan(const int* totals, int* offsets, int m, int side, int nlist, int* begin, int* end, int* count,
                       int cap, unsigned* err, unsigned err_bit, hipStream_t st);
// Two independent scans in one launch (second array: *2 arguments).
hipError_t launch_scan2(const int* totals, int* offsets, int m, int side, int nlist, int* begin, int* end, int* count,
                        int cap, unsigned err_bit, const int* totals2, int* offsets2, int m2, int side2, int nlist2,
                        int* begin2, int* end2, int* count2, int cap2, unsigned err_bit2, unsigned* err,
                        hipStream_t st);
// Per-particle sum of 6-double records [begin[j], end[j]) (+ base) into Facc/Tacc of particle list[j]:
// nchunk_blocks workgroups per particle over chunks of RED_CHUNK records store their sums in partial
// (nlist * nchunk_blocks * 6 doubles), then launch_finish_sums adds them.
constexpr int RED_CHUNK = 1024;
constexpr int SUM_THREADS = 256;  // workgroup size of the summing kernels (one link per thread and chunk)
hipError_t launch_reduce(const int* list, int nlist, const int* begin, const int* end, int base, const double* out,
                         long long ostride, PartDev parts, int nchunk_blocks, double* partial,
                         const InstDev* rigid_insts, unsigned* err, hipStream_t st);
// Adds the min(ceil((end[j] - begin[j]) / chunk), width) chunk sums of list position j (rows of partial are
// width wide) in a fixed order to Facc/Tacc of particle list[j], for each of nsets sets (set s at
// partial + s * set_stride doubles), set after set; with rigid_insts != nullptr each particle's explicit Euler
// rigid-body step (averaging Facc over n_sub sweeps) follows.
hipError_t launch_finish_sums(const int* list, int nlist, const int* begin, const int* end, int chunk, int width,
                              const double* partial, int nsets, long long set_stride, PartDev parts,
                              const InstDev* rigid_insts, unsigned* err, hipStream_t st);

// ---- mem.hip
hipError_t launch_mem_unmap(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                            int* owner, hipStream_t st);
hipError_t launch_mem_map(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                          int* owner, hipStream_t st);
// Link masks per cell and per-unit link counts; with `uncovered`, also the
// uncovered cells (bit 0) and their per-unit counts in totals2.
hipError_t launch_mem_count(bool uncovered, const int* list, int nlist, int side, int nsplit, const InstDev* insts,
                            PartDev parts, const int* owner, int* slots, int* totals, int* totals2, hipStream_t st);
// Link list at the scanned offsets; with rcell, also the refill list at offsets2.
hipError_t launch_mem_fill_links(const int* list, int nlist, int side, int nsplit, const InstDev* insts,
                                 PartDev parts, int* owner, const int* slots, const int* offsets, int base, int cap,
                                 LinkDev links, const int* offsets2, int cap2, int* rcell, int* rpart,
                                 hipStream_t st);
hipError_t launch_mem_refill(int prec, const int* count, int cap, const int* rcell, const int* rpart,
                             const InstDev* insts, PartDev parts, const int* owner, void* buf, hipStream_t st);
// Link rules of the wall links [0, n_wall) and of the particle links [n_wall + lbeg[j], n_wall + lend[j]) of
// list[j].  Each particle's link force and torque chunk sums go to set `set` of partial (width workgroups per
// particle, nlist * width * 6 doubles per set); after the last sweep of a rigid-body step, launch_finish_sums
// over all sets (SUM_THREADS records per chunk, set_stride nlist * width * 6) adds them to Facc/Tacc.
// Wall groups: WALL_REC doubles each, the wall velocity (3), WALL_KIND (0 a
// velocity wall, bounce-back with that velocity; 1 an outflow) and WALL_RHO_OUT.
// Outflow links read the pre-collision PDFs of their fluid cell from src.
constexpr int WALL_REC = 8, WALL_KIND = 3, WALL_RHO_OUT = 4, WALL_GROUPS = 16;
hipError_t launch_links_bc(int prec, int n_wall, const int* list, int nlist, const int* lbeg, const int* lend,
                           int width, LinkDev links, const double* wall_v, const InstDev* insts, PartDev parts,
                           const void* src, void* buf, double* partial, int set, hipStream_t st);

// ---- psm.hip
hipError_t launch_psm_classify(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                               int* slots, int* totals, hipStream_t st);
hipError_t launch_psm_cut_fill(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                               const int* slots, const int* offsets, CutDev cuts, int cap, hipStream_t st);
hipError_t launch_psm_cut_exact(const InstDev* insts, PartDev parts, int* slots, CutDev cuts, int cap, double rmin,
                                double rmax, hipStream_t st);
hipError_t launch_psm_cut_features(const InstDev* insts, PartDev parts, CutDev cuts, int cap, double rmin,
                                   double rmax, float* X, hipStream_t st);
hipError_t launch_psm_cut_scatter(const InstDev* insts, PartDev parts, CutDev cuts, int cap, const float* y,
                                  int* slots, hipStream_t st);
hipError_t launch_psm_unit_totals(const int* list, int nlist, int side, int nsplit, PartDev parts, const int* slots,
                                  int* totals, hipStream_t st);
hipError_t launch_psm_label(const double* rd, long long ns, int n, float* eps, hipStream_t st);
hipError_t launch_psm_judge(const InstDev* insts, PartDev parts, const int* slots, CutDev cuts, int cap, int stride,
                            double* stats, hipStream_t st);
hipError_t launch_psm_fill(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                           const int* slots, const int* offsets, int cap, PairDev pairs, hipStream_t st);
hipError_t launch_psm_cellmap(int stage, const int* count, int cap, const InstDev* insts, PartDev parts,
                              PairDev pairs, int* cellmap, hipStream_t st);
// Collision of every overlapped cell (two launches: single-pair cells unless shared_only, then shared cells),
// pushed into dst or,
// with stage != nullptr, stored per leader pair for the sweep that follows.  psm_m: the solid operator shared by
// every PSM instance (1..3), or 0 when they differ.
// With sums (and not shared_only): the shared cells first, then the single-pair cells per particle (list
// positions [0, nlist) with pair ranges [begin[j], end[j])), which also store the force/torque chunk sums of
// every pair of the range (width chunk rows per particle, as launch_reduce) in partial, for launch_finish_sums
// with chunk RED_CHUNK; no reduce launch is needed.
struct PsmSums {
  const int* list;
  int nlist;
  const int *begin, *end;
  int width;
  double* partial;
};
hipError_t launch_psm_collide(int prec, int psm_m, const int* count, int cap, const InstDev* insts, PartDev parts,
                              PairDev pairs, const int* cellmap, const void* src, void* dst, void* stage,
                              long long sstride, bool shared_only, hipStream_t st, const PsmSums* sums = nullptr);
hipError_t launch_psm_fields(int prec, const int* count, int cap, const InstDev* insts, PartDev parts, PairDev pairs,
                             const int* cellmap, const void* buf, int inst, long long c0, long long n, double* out,
                             hipStream_t st);

// ---- mlp.hip
int mlp_nparam();
hipError_t launch_mlp_features(const double* rd, long long n, int n_inputs, float* X, hipStream_t st);
hipError_t launch_mlp_infer(const float* P, const float* X, long long n, float* y, hipStream_t st);
hipError_t launch_mlp_infer_count(const float* P, const float* X, const int* count, long long cap, float* y,
                                  hipStream_t st);
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, long long n, long long b0, long long mult,
                           long long add, int batch, float* partial, hipStream_t st);
hipError_t launch_mlp_reduce_adam(float* P, const float* partial, int ntiles, float* grad, float* m, float* v,
                                  int do_adam, float lr, float b1, float b2, float eps, int step, hipStream_t st);

}  // namespace lbm
