// C-ABI layer of lbmps: workspace layout, validation, and the host-side
// schedule of one LBM time step (Alg. 1 for MEM, Alg. 2 for PSM):
//
//   sweep (collide + push, every instance)            -- sweep.hip
//   PSM overlapped cells: solid operator, re-push      -- psm.hip
//   link rule + link force (MEM particles, walls)      -- mem.hip
//   per-particle force/torque sums                      -- particles.hip
//   every n_sub sweeps: rigid-body step, then remap with refill and new links
//   (MEM) / new solid fractions (PSM).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbmps.h"
#include "common.h"
#include "kernels.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t storage_size(int prec) {
  switch (prec) {
    case PREC_FP64: return 8;
    case PREC_FP32: return 4;
    case PREC_FP16:
    case PREC_BF16: return 2;
  }
  return 0;
}

struct Layout {
  bool ok = false;
  std::string err;
  int n = 0, prec = 0, side = 0, ptotal = 0, mem_nsub = 0, psm_nsub = 0;
  int psm_m = -1;  // solid operator shared by the PSM instances, 0 if they differ
  size_t ssz = 0;
  std::vector<long long> pdf_off, owner_off, cellmap_off, ncell;
  std::vector<int> part_begin;
  long long pdf_elems = 0, owner_elems = 0, cellmap_elems = 0;
  int link_cap = 0, wall_cap = 0, pair_cap = 0, refill_cap = 0, cut_cap = 0;
  int red_blocks = 1;   // reduction workgroups per particle
  int link_blocks = 1;  // link-kernel workgroups per particle
  bool learned = false;  // some instance estimates eps_s with the network
  long long slot_elems = 0;
  int box_total = 0;  // ptotal * side * side: work units at the finest split
  long long chunk = 0;
  // byte offsets
  size_t o_bufA, o_bufB, o_owner, o_cellmap, o_inst, o_parts, o_plists, o_slots, o_totals, o_offsets, o_totals2, o_offsets2, o_ranges, o_red, o_redm, o_stage,
      o_counts, o_links, o_wallv, o_pairs, o_refill, o_scratch, o_tiles, o_cuts, o_cutx, o_mlp, o_judge, total;
  int ntiles = 0;
  int max_tile_cells = 0;
};

// The four-cells-per-thread sweep (bit 8): 2-byte storage, whole 8-byte words per row.
static bool quads_ok(int flags, int precision, int nx) {
  if (!(flags & SWEEP_CELL_QUADS)) return true;
  return (precision == LBMPS_FP16_DEV || precision == LBMPS_BF16_DEV) && nx % 4 == 0 &&
         !(flags & (SWEEP_OCC6 | SWEEP_CELL_PAIRS));
}

bool valid_cfg(const lbmps_config& c, std::string& err) {
  if (c.nx < 1 || c.ny < 1 || c.nz < 1) { err = "box dimensions must be positive"; return false; }
  if ((long long)c.nx * c.ny * c.nz >= (1LL << 31)) { err = "box too large (>= 2^31 cells)"; return false; }
  if (c.collision != LBMPS_BGK && c.collision != LBMPS_TRT) { err = "collision must be BGK or TRT"; return false; }
  if (c.coupling < LBMPS_NONE || c.coupling > LBMPS_PSM) { err = "unknown coupling"; return false; }
  if (c.coupling == LBMPS_PSM && (c.psm_m < 1 || c.psm_m > 3 || c.psm_b < 1 || c.psm_b > 2)) {
    err = "psm_m must be 1..3 and psm_b 1..2"; return false;
  }
  if (c.precision < LBMPS_FP64 || c.precision > LBMPS_BF16_DEV) { err = "unknown precision"; return false; }
  if (!(c.nu > 0.0) || !std::isfinite(c.nu)) { err = "nu must be positive"; return false; }
  if (c.max_particles < 0) { err = "max_particles must be >= 0"; return false; }
  if (c.max_particles > 0 && !(c.max_diameter > 0.0)) { err = "max_diameter must be positive"; return false; }
  if (c.max_particles > 0 && std::ceil(c.max_diameter) + 6 > 64) {
    err = "max_diameter must be <= 58 cells (bounding boxes of at most 64 cells per axis)"; return false;
  }
  if (c.max_particles > 0 && c.max_diameter + 6 > std::min(c.nx, std::min(c.ny, c.nz))) {
    err = "max_diameter + 6 exceeds the smallest box dimension"; return false;
  }
  const int en = c.eps_n ? c.eps_n : 8;
  if (en < 1 || en > 64) { err = "eps_n must be 1..64"; return false; }
  if (c.eps_mode == LBMPS_EPS_RECURSIVE && (en & (en - 1))) { err = "recursive supersampling needs eps_n = 2^k"; return false; }
  if (c.eps_mode < 0 || c.eps_mode > 4) { err = "unknown eps_mode"; return false; }
  if (c.block_threads < 0 || c.block_threads > 256 || (c.block_threads % 64)) { err = "block_threads must be a multiple of 64, <= 256"; return false; }
  if (c.sweep_flags & ~SWEEP_FLAGS_ALL) { err = "unknown sweep_flags bits"; return false; }
  if ((c.sweep_flags & SWEEP_WG_CAP_MASK) == SWEEP_WG_CAP_MASK) { err = "sweep_flags: workgroup cap 3 is invalid"; return false; }
  if ((c.sweep_flags & SWEEP_CELL_PAIRS) && (c.nx & 1)) { err = "sweep_flags: cell pairs need an even nx"; return false; }
  if (!quads_ok(c.sweep_flags, c.precision, c.nx)) {
    err = "sweep_flags: cell quads need FP16/BF16 storage, nx a multiple of 4, and neither bit 3 nor bit 7"; return false;
  }
  if (__builtin_popcount(c.sweep_flags & SWEEP_PSM_MODES) > 1) {
    err = "sweep_flags: the PSM modes (fused, separate, staged) are exclusive"; return false;
  }
  if (c.n_sub < 0) { err = "n_sub must be >= 0"; return false; }
  if (c.refill != LBMPS_REFILL_EXTRAPOLATE && c.refill != LBMPS_REFILL_EQUILIBRIUM) { err = "unknown refill"; return false; }
  if (10LL * (long long)storage_size(c.precision) * c.nx > SWEEP_LDS_LIMIT) {
    err = "nx too large for the LDS-staged sweep (10 * nx * element size must be <= 64 KiB)"; return false;
  }
  return true;
}

int eff_nsub(const lbmps_config& c) {
  if (c.coupling == LBMPS_MEM_BB || c.coupling == LBMPS_MEM_CLI) return c.n_sub ? c.n_sub : 2;
  return c.n_sub ? c.n_sub : 1;
}

// Rows per sweep tile: by default about one PDF block (256 cells) per tile for
// 4- and 8-byte storage and two blocks for 2-byte storage (measured optima),
// bounded by the LDS staging limit (10 shifted planes).
int eff_tile_rows(const lbmps_config& c) {
  const int s = (int)storage_size(c.precision);
  const int max_rows = std::max(1, SWEEP_LDS_LIMIT / (10 * s * c.nx));
  if (c.tile_rows > 0) return std::min(c.tile_rows, max_rows);
  const int target = s == 2 ? 2 * PDF_BLOCK : PDF_BLOCK;
  return std::max(1, std::min(max_rows, target / c.nx));
}

Layout make_layout(int n, const lbmps_config* cfgs) {
  Layout L;
  if (n < 1 || !cfgs) { L.err = "need at least one configuration"; return L; }
  L.n = n;
  L.prec = cfgs[0].precision;
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!valid_cfg(cfgs[i], L.err)) return L;
    if (cfgs[i].precision != L.prec) { L.err = "all instances of a batch must share the precision"; return L; }
    const bool mem = cfgs[i].coupling == LBMPS_MEM_BB || cfgs[i].coupling == LBMPS_MEM_CLI;
    if (mem) {
      if (L.mem_nsub && L.mem_nsub != eff_nsub(cfgs[i])) { L.err = "MEM instances of a batch must share n_sub"; return L; }
      L.mem_nsub = eff_nsub(cfgs[i]);
    }
    if (cfgs[i].coupling == LBMPS_PSM) {
      if (L.psm_nsub && L.psm_nsub != eff_nsub(cfgs[i])) { L.err = "PSM instances of a batch must share n_sub"; return L; }
      L.psm_nsub = eff_nsub(cfgs[i]);
      L.psm_m = (L.psm_m < 0 || L.psm_m == cfgs[i].psm_m) ? cfgs[i].psm_m : 0;
    }
    if (cfgs[i].max_particles > 0) dmax = std::max(dmax, cfgs[i].max_diameter);
  }
  L.ssz = storage_size(L.prec);
  L.side = (int)std::ceil(dmax) + 6;
  long long pdf = 0, own = 0, cm = 0;
  double rmax = 0.5 * dmax;
  long long pairs = 0, links = 0, refill = 0, walls = 0, cuts = 0;
  long long cmax = 0;
  for (int i = 0; i < n; ++i) {
    const lbmps_config& c = cfgs[i];
    const long long N = (long long)c.nx * c.ny * c.nz;
    L.ncell.push_back(N);
    L.pdf_off.push_back(pdf);
    pdf += pdf_elems(N);
    L.owner_off.push_back(own);
    own += (N + 63) / 64 * 64;
    if (c.coupling == LBMPS_PSM) {
      L.cellmap_off.push_back(cm);
      cm += (N + 63) / 64 * 64;
    } else {
      L.cellmap_off.push_back(-1);
    }
    L.part_begin.push_back(L.ptotal);
    L.ptotal += c.max_particles;
    const long long sd = L.side;
    const long long lp = 40 * sd * sd, pp = (long long)std::ceil(4.2 * std::pow(rmax + 1.8, 3));
    links += (long long)c.max_particles * lp;
    pairs += (long long)c.max_particles * pp;
    if (c.max_particles > 0 && c.coupling == LBMPS_PSM)
      L.red_blocks = (int)std::max<long long>(L.red_blocks, (pp + RED_CHUNK - 1) / RED_CHUNK);
    if (c.max_particles > 0 && c.coupling != LBMPS_PSM)
      L.link_blocks = (int)std::max<long long>(L.link_blocks, (lp + SUM_THREADS - 1) / SUM_THREADS);
    if (c.coupling == LBMPS_PSM) {
      // cells cut by a sphere surface lie within sqrt(3)/2 of it: a shell of
      // volume below 8 pi (R + 1)^2
      cuts += (long long)c.max_particles * (long long)std::ceil(8.0 * M_PI * (rmax + 1.0) * (rmax + 1.0));
      if (c.eps_mode == LBMPS_EPS_LEARNED) L.learned = true;
    }
    refill += (long long)c.max_particles * 6 * sd * sd;
    walls += c.wall_link_cap > 0 ? c.wall_link_cap
                                 : 10LL * ((long long)c.nx * c.ny + (long long)c.ny * c.nz + (long long)c.nz * c.nx);
    cmax = std::max(cmax, N);
    L.ntiles += (c.ny * c.nz + eff_tile_rows(c) - 1) / eff_tile_rows(c);
    L.max_tile_cells = std::max(L.max_tile_cells, eff_tile_rows(c) * c.nx);
  }
  if (links + walls >= (1LL << 31) || pairs >= (1LL << 31) || cuts >= (1LL << 31)) {
    L.err = "list capacities exceed 2^31"; return L;
  }
  L.pdf_elems = pdf;
  L.owner_elems = own;
  L.cellmap_elems = cm;
  L.link_cap = (int)links;
  L.wall_cap = (int)walls;
  L.pair_cap = (int)pairs;
  L.refill_cap = (int)refill;
  L.cut_cap = (int)cuts;
  L.slot_elems = (long long)L.ptotal * L.side * L.side * L.side;
  L.box_total = L.ptotal * L.side * L.side;
  L.chunk = std::min<long long>(cmax, 1LL << 22);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  L.o_bufA = take(L.pdf_elems * L.ssz);
  L.o_bufB = take(L.pdf_elems * L.ssz);
  L.o_owner = take(L.owner_elems * 4);
  L.o_cellmap = take(L.cellmap_elems * 4);
  L.o_inst = take(sizeof(InstDev) * n);
  L.o_parts = take((size_t)L.ptotal * (3 * 9 + 2 + 6) * 8 + (size_t)L.ptotal * 2 * 4);
  L.o_plists = take((size_t)L.ptotal * 2 * 4);
  L.o_slots = take((size_t)L.slot_elems * 4);
  L.o_totals = take((size_t)L.box_total * 4);
  L.o_offsets = take((size_t)L.box_total * 4);
  L.o_totals2 = take((size_t)L.box_total * 4);
  L.o_offsets2 = take((size_t)L.box_total * 4);
  L.o_ranges = take((size_t)L.ptotal * 8 * 4);
  L.o_red = take((size_t)L.ptotal * L.red_blocks * 6 * 8);
  // MEM link sums of every sweep of a rigid-body step, added up after its last
  L.o_redm = take((size_t)L.ptotal * L.link_blocks * 6 * 8 * std::max(1, L.mem_nsub));
  L.o_counts = take(16 * 4);
  L.o_links = take((size_t)(L.link_cap + L.wall_cap) * (5 * 4 + 8) + 2 * ALIGN);
  L.o_wallv = take((size_t)n * WALL_GROUPS * WALL_REC * 8);
  L.o_pairs = take((size_t)L.pair_cap * (3 * 4 + 2 * 8 + 6 * 8) + 2 * ALIGN);
  L.o_refill = take((size_t)L.refill_cap * 2 * 4);
  L.o_scratch = take((size_t)L.chunk * 4 * 8);
  L.o_tiles = take((size_t)L.ntiles * sizeof(int4));
  L.o_cuts = take((size_t)L.cut_cap * (8 + 4 + 4 + 24) + 4 * ALIGN);
  L.o_cutx = take(L.learned ? (size_t)L.cut_cap * (8 + 1) * 4 : 0);
  L.o_mlp = take((size_t)mlp_nparam() * 4);
  L.o_judge = take(4 * 8);  // own aligned block: the judge updates it with 8-byte atomics
  // post-collision values of overlapped cells, per leader pair (staged PSM mode)
  L.o_stage = take(L.cellmap_elems > 0 ? (size_t)Q * L.pair_cap * L.ssz : 0);
  L.total = o;
  L.ok = true;
  return L;
}

}  // namespace

// PSM cells: collided by the overlap kernel after the sweep (which then
// overwrites their pushes), inside the sweep, or by the overlap kernel before
// the sweep into a staging array that the sweep pushes.
enum { PSM_SEPARATE = 0, PSM_FUSED = 1, PSM_STAGED = 2 };

constexpr size_t TIMING_EVENTS = 4096;  // HIP events of the timing pool (start/stop pairs)

struct lbmps_ctx {
  hipStream_t st = nullptr;
  int device = -1;        // current device at creation (the workspace's)
  bool in_order = false;  // every step's work on st: no second stream (lbmps_step_noalloc)
  Layout L;
  std::vector<lbmps_config> cfg;
  std::vector<InstDev> inst_h;
  char* ws = nullptr;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buf[cur] holds the canonical PDFs
  int* owner = nullptr;
  int* cellmap = nullptr;
  InstDev* inst_d = nullptr;
  int4* tiles_d = nullptr;
  int ntiles = 0, grid = 0, block = 256;
  PartDev parts{};
  int* plist_d = nullptr;  // [0, n_mem) MEM particles, then PSM particles
  std::vector<int> n_active;
  std::vector<int> fixed_h;  // per global particle
  std::vector<int> coupling_of_part;
  int n_mem = 0, n_psm = 0;
  bool mem_moving = false, psm_moving = false;
  int* slots = nullptr;
  int* totals = nullptr;
  int* offsets = nullptr;
  int* totals2 = nullptr;  // second per-unit count (refill cells of the MEM remap)
  int* offsets2 = nullptr;
  double* red_partial = nullptr;  // per-chunk force/torque sums (PSM overlap records)
  double* red_mem = nullptr;      // per-chunk MEM link sums, one set per sweep of a rigid-body step
  int *lbeg = nullptr, *lend = nullptr, *pbeg = nullptr, *pend = nullptr, *rbeg = nullptr, *rend = nullptr,
      *cbeg = nullptr, *cend = nullptr;
  int* counts = nullptr;  // [0] links, [1] pairs, [2] refill, [4] error bits (unsigned)
  LinkDev links{};
  int n_wall = 0;
  std::vector<int> wall_groups;  // per instance
  double* wall_v = nullptr;
  PairDev pairs{};
  int* rcell = nullptr;
  int* rpart = nullptr;
  CutDev cuts{};
  float* cut_x = nullptr;  // features [cut_cap][8], then outputs [cut_cap]
  float* mlp_p = nullptr;  // network parameters (learned eps_s)
  double* judge = nullptr; // error statistics of lbmps_eps_judge
  bool mlp_set = false;
  double mlp_rmin = 0.0, mlp_rmax = -1.0;
  bool psm_exact = true;           // some PSM cut cell needs supersampling
  int psm_mode = PSM_SEPARATE;      // how the sweep and the overlap kernel share the PSM cells
  void* stage = nullptr;            // staged post-collision values (PSM_STAGED)
  std::vector<double> diam_h;      // per global particle
  double* scratch = nullptr;
  long long sweeps = 0;
  bool have_psm = false, have_links_inst = false;
  // MEM remap or PSM list rebuild overlapped with the next sweep: it runs on
  // `side` (forked after the rigid-body step, joined right after that sweep;
  // a MEM remap is followed by a re-sweep of its refilled cells)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool join_pending = false;
  bool join_resweep = false;  // the forked work holds a MEM remap: re-sweep its refilled cells
  bool join_lists = false;    // the forked work holds a PSM rebuild: the next sweep reads no list
  // captured step graph (one period of sweeps), invalidated when lists change
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_period = 0, graph_cur = -1;
  // optional timing of sweep-kernel launches (HIP events on the stream): every
  // timing_stride-th launch after set_timing
  bool timing = false;
  int timing_stride = 1;
  long long timing_seq = 0;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t ev_used = 0;
  double sweep_ms = 0.0;
  long long sweep_launches = 0;
  std::string last;
};

namespace {

// tau from Eq. Viscosity (nu = (tau - 1/2)/3), lambda_+ = -1/tau and, for TRT,
// lambda_- from the magic parameter (Eq. MEM_TRT); BGK: lambda_- = lambda_+.
void set_relaxation(InstDev& I, const lbmps_config& cf) {
  I.tau = 3.0 * cf.nu + 0.5;
  I.mag = cf.magic > 0 ? cf.magic : 3.0 / 16.0;
  I.lam_p = -1.0 / I.tau;
  if (cf.collision == LBMPS_TRT) {
    const double inv_m = I.mag / (0.5 + 1.0 / I.lam_p) - 0.5;
    I.lam_m = 1.0 / inv_m;
  } else {
    I.lam_m = I.lam_p;
  }
}

lbmps_status fail(lbmps_ctx* c, lbmps_status s, const std::string& msg) {
  if (c) c->last = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                                       \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(ctx, LBMPS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

unsigned* err_word(lbmps_ctx* c) { return (unsigned*)(c->counts + 4); }

lbmps_status check_device_errors(lbmps_ctx* c) {
  unsigned e = 0;
  HIPCHK(c, hipMemcpyAsync(&e, err_word(c), sizeof(unsigned), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (e & ERR_UNSTABLE)
    return fail(c, LBMPS_EUNSTABLE, "unstable rigid-body step (a particle would move >= 1 cell or its state is not finite); not taken");
  if (e & ERR_LINK_CAP) return fail(c, LBMPS_ENOMEM, "boundary-link capacity exceeded");
  if (e & ERR_PAIR_CAP) return fail(c, LBMPS_ENOMEM, "overlap-pair capacity exceeded");
  if (e & ERR_REFILL_CAP) return fail(c, LBMPS_ENOMEM, "refill-list capacity exceeded");
  if (e & ERR_CUT_CAP) return fail(c, LBMPS_ENOMEM, "cut-cell list capacity exceeded");
  return LBMPS_OK;
}

// Row ranges per bounding-box slab: enough work units (>= ~2048) to fill the GPU.
// Row splits per bounding-box slab so that about `target` work units exist.
// In order, many small units keep the short remap and rebuild latency low;
// beside a sweep (side stream) fewer, fuller workgroups take fewer of the
// sweep's CU slots and still finish well within it.  The split does not
// change the cell order of any list.
int nsplit_for(int nlist, int side, int target = 2048) {
  if (nlist <= 0) return 1;
  const int want = (target + nlist * side - 1) / (nlist * side);
  return std::max(1, std::min(side, want));
}
int split_target(const lbmps_ctx* c, hipStream_t st) { return st == c->st ? 2048 : 256; }

int* mem_list(lbmps_ctx* c) { return c->plist_d; }

// Whether any current PSM particle needs supersampled cut cells (an exact
// estimator, or the learned one outside its radius range), and how PSM cells
// are collided.  Inline collision raises the sweep's register count, which
// lowers its occupancy: slower than the other two modes, used only when
// sweep_flags asks for it.  The separate pass after the sweep rewrites the
// pushes of the overlapped cells as scattered partial cache lines; the staged
// mode writes them as whole lines but makes the sweep read one cell-map entry
// per cell.  Measured on 2000 spheres in 512^3 (4.3 % of the cells overlapped)
// staging saves ~0.4 ms per sweep; with one sphere in 14 M cells the cell-map
// reads cost more than they save.  Without a mode in sweep_flags, staging is
// chosen when the current PSM spheres (bounding spheres of diameter D + 2)
// cover at least 1 % of the PSM cells.
void update_psm_exact(lbmps_ctx* c) {
  c->psm_exact = false;
  for (int k = 0; k < c->L.n; ++k) {
    if (c->cfg[k].coupling != LBMPS_PSM) continue;
    const int b = c->L.part_begin[k];
    for (int i = 0; i < c->n_active[k]; ++i) {
      const double R = 0.5 * c->diam_h[b + i];
      const int em = c->cfg[k].eps_mode;
      if (em == LBMPS_EPS_FLAT || em == LBMPS_EPS_RECURSIVE ||
          (em == LBMPS_EPS_LEARNED && (!c->mlp_set || R < c->mlp_rmin || R > c->mlp_rmax)))
        c->psm_exact = true;
    }
  }
  const int fl = c->cfg[0].sweep_flags;
  if (fl & SWEEP_PSM_FUSED) {
    c->psm_mode = PSM_FUSED;
  } else if (fl & SWEEP_PSM_STAGED) {
    c->psm_mode = PSM_STAGED;
  } else if (fl & SWEEP_PSM_SEPARATE) {
    c->psm_mode = PSM_SEPARATE;
  } else {
    double vol = 0.0, cells = 0.0;
    for (int k = 0; k < c->L.n; ++k) {
      if (c->cfg[k].coupling != LBMPS_PSM) continue;
      cells += (double)c->L.ncell[k];
      const int b = c->L.part_begin[k];
      for (int i = 0; i < c->n_active[k]; ++i) {
        const double D = c->diam_h[b + i] + 2.0;
        vol += M_PI / 6.0 * D * D * D;
      }
    }
    c->psm_mode = (cells > 0 && vol >= 0.01 * cells) ? PSM_STAGED : PSM_SEPARATE;
  }
}

int* psm_list(lbmps_ctx* c) { return c->plist_d + c->n_mem; }

// Rebuild links of every MEM particle (after mapping); refill first when `refill`.
lbmps_status rebuild_mem(lbmps_ctx* c, bool refill, hipStream_t st) {
  const Layout& L = c->L;
  if (c->n_mem == 0) return LBMPS_OK;
  unsigned* err = err_word(c);
  const int ns = nsplit_for(c->n_mem, L.side, split_target(c, st));
  const int units = L.side * ns;
  // one pass counts links and uncovered cells, one launch scans both, one
  // pass writes both lists; the refill only reads the owner field, so it can
  // follow the link list
  HIPCHK(c, launch_mem_count(refill, mem_list(c), c->n_mem, L.side, ns, c->inst_d, c->parts, c->owner,
                             c->slots, c->totals, c->totals2, st));
  if (refill)
    HIPCHK(c, launch_scan2(c->totals, c->offsets, c->n_mem * units, units, c->n_mem, c->lbeg, c->lend, c->counts + 0,
                           L.link_cap, ERR_LINK_CAP, c->totals2, c->offsets2, c->n_mem * units, units, c->n_mem,
                           c->rbeg, c->rend, c->counts + 2, L.refill_cap, ERR_REFILL_CAP, err, st));
  else
    HIPCHK(c, launch_scan(c->totals, c->offsets, c->n_mem * units, units, c->n_mem, c->lbeg, c->lend, c->counts + 0,
                          L.link_cap, err, ERR_LINK_CAP, st));
  HIPCHK(c, launch_mem_fill_links(mem_list(c), c->n_mem, L.side, ns, c->inst_d, c->parts, c->owner, c->slots,
                                  c->offsets, c->n_wall, L.link_cap, c->links, c->offsets2, L.refill_cap,
                                  refill ? c->rcell : nullptr, c->rpart, st));
  if (refill)
    HIPCHK(c, launch_mem_refill(L.prec, c->counts + 2, L.refill_cap, c->rcell, c->rpart, c->inst_d, c->parts, c->owner,
                                c->buf[c->cur], st));
  return LBMPS_OK;
}

lbmps_status remap_mem(lbmps_ctx* c, hipStream_t st) {
  const int ns = nsplit_for(c->n_mem, c->L.side, split_target(c, st));
  HIPCHK(c, launch_mem_unmap(mem_list(c), c->n_mem, c->L.side, ns, c->inst_d, c->parts, c->owner, st));
  HIPCHK(c, launch_mem_map(mem_list(c), c->n_mem, c->L.side, ns, c->inst_d, c->parts, c->owner, st));
  return rebuild_mem(c, true, st);
}

__global__ void fill_int_kernel(int* a, long long n, int v);

// Solid fractions and overlap lists of every PSM particle (Sec. 2.3.2):
// classify bounding-box cells, evaluate the cut ones (supersampling, or the
// network inside its radius range), count per work unit, scan, fill, and link
// the pairs of shared cells.  Kernel launches only (graph capturable).
lbmps_status rebuild_psm(lbmps_ctx* c, hipStream_t st) {
  const Layout& L = c->L;
  if (c->n_psm == 0) return LBMPS_OK;
  unsigned* err = err_word(c);
  const int ns = nsplit_for(c->n_psm, L.side, split_target(c, st));
  const int units = L.side * ns;
  HIPCHK(c, launch_psm_cellmap(0, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs, c->cellmap, st));
  HIPCHK(c, launch_psm_classify(psm_list(c), c->n_psm, L.side, ns, c->inst_d, c->parts, c->slots, c->totals, st));
  HIPCHK(c, launch_scan(c->totals, c->offsets, c->n_psm * units, units, c->n_psm, c->cbeg, c->cend, c->cuts.count,
                        L.cut_cap, err, ERR_CUT_CAP, st));
  HIPCHK(c, launch_psm_cut_fill(psm_list(c), c->n_psm, L.side, ns, c->inst_d, c->parts, c->slots, c->offsets,
                                c->cuts, L.cut_cap, st));
  const double rmin = c->mlp_set ? c->mlp_rmin : 0.0, rmax = c->mlp_set ? c->mlp_rmax : -1.0;
  if (L.learned && c->mlp_set) {
    float* y = c->cut_x + (size_t)L.cut_cap * 8;
    HIPCHK(c, launch_psm_cut_features(c->inst_d, c->parts, c->cuts, L.cut_cap, rmin, rmax, c->cut_x, st));
    HIPCHK(c, launch_mlp_infer_count(c->mlp_p, c->cut_x, c->cuts.count, L.cut_cap, y, st));
    HIPCHK(c, launch_psm_cut_scatter(c->inst_d, c->parts, c->cuts, L.cut_cap, y, c->slots, st));
  }
  if (c->psm_exact)
    HIPCHK(c, launch_psm_cut_exact(c->inst_d, c->parts, c->slots, c->cuts, L.cut_cap, rmin, rmax, st));
  HIPCHK(c, launch_psm_unit_totals(psm_list(c), c->n_psm, L.side, ns, c->parts, c->slots, c->totals, st));
  HIPCHK(c, launch_scan(c->totals, c->offsets, c->n_psm * units, units, c->n_psm, c->pbeg, c->pend, c->counts + 1,
                        L.pair_cap, err, ERR_PAIR_CAP, st));
  HIPCHK(c, launch_psm_fill(psm_list(c), c->n_psm, L.side, ns, c->inst_d, c->parts, c->slots, c->offsets, L.pair_cap,
                            c->pairs, st));
  HIPCHK(c, launch_psm_cellmap(1, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs, c->cellmap, st));
  HIPCHK(c, launch_psm_cellmap(2, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs, c->cellmap, st));
  return LBMPS_OK;
}

__global__ void fill_int_kernel(int* a, long long n, int v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
__global__ void reset_owner_kernel(int* a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && a[i] > OWN_FLUID) a[i] = OWN_FLUID;
}

lbmps_status fill_int(lbmps_ctx* c, int* a, long long n, int v) {
  if (n <= 0) return LBMPS_OK;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->st, a, n, v);
  HIPCHK(c, hipGetLastError());
  return LBMPS_OK;
}

// Accumulate the elapsed time of every recorded (start, stop) event pair.
lbmps_status harvest_timing(lbmps_ctx* c) {
  if (c->ev_used == 0) return LBMPS_OK;
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (size_t k = 0; k < c->ev_used; k += 2) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
    c->sweep_ms += ms;
    c->sweep_launches++;
  }
  c->ev_used = 0;
  return LBMPS_OK;
}

void drop_graph(lbmps_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_cur = -1;
}

lbmps_status check_inst(lbmps_ctx* c, int inst) {
  if (!c) return LBMPS_EINVAL;
  if (inst < 0 || inst >= c->L.n) return fail(c, LBMPS_EINVAL, "instance index out of range");
  return LBMPS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of lbmps_step_noalloc: the per-chunk force and torque sums of the
// overlap records and of the boundary links.  One copy per GPU, held until the
// process ends and shared by every call on that GPU.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[LBMPS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[SCRATCH_DEVICES] = {};

// Device address of `scratch` on the current device `dev`.
lbmps_status scratch_address(lbmps_ctx* c, int dev, void** out) {
  if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(c, LBMPS_EDEVICE, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, LBMPS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return LBMPS_OK;
}

}  // namespace

extern "C" {

void lbmps_velocities(int32_t c[19][3]) {
  for (int q = 0; q < 19; ++q) {
    c[q][0] = cx(q);
    c[q][1] = cy(q);
    c[q][2] = cz(q);
  }
}

size_t lbmps_workspace_bytes(const lbmps_config* cfg) { return lbmps_batch_workspace_bytes(1, cfg); }

size_t lbmps_batch_workspace_bytes(int32_t n, const lbmps_config* cfgs) {
  Layout L = make_layout(n, cfgs);
  return L.ok ? L.total : 0;
}

lbmps_status lbmps_create(const lbmps_config* cfg, void* ws, size_t bytes, void* stream, lbmps_ctx** out) {
  return lbmps_batch_create(1, cfg, ws, bytes, stream, out);
}

lbmps_status lbmps_batch_create(int32_t n, const lbmps_config* cfgs, void* ws, size_t bytes, void* stream,
                                lbmps_ctx** out) {
  if (!out) return LBMPS_EINVAL;
  *out = nullptr;
  Layout L = make_layout(n, cfgs);
  if (!L.ok) return LBMPS_EINVAL;
  if (!ws || bytes < L.total) return LBMPS_ENOMEM;
  lbmps_ctx* c = new lbmps_ctx();
  c->st = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
  c->L = L;
  c->cfg.assign(cfgs, cfgs + n);
  char* w = (char*)ws;
  c->ws = w;
  c->buf[0] = w + L.o_bufA;
  c->buf[1] = w + L.o_bufB;
  c->owner = (int*)(w + L.o_owner);
  c->cellmap = (int*)(w + L.o_cellmap);
  c->inst_d = (InstDev*)(w + L.o_inst);
  c->tiles_d = (int4*)(w + L.o_tiles);
  {
    double* d = (double*)(w + L.o_parts);
    const size_t P = L.ptotal;
    c->parts.X = d; d += 3 * P;
    c->parts.U = d; d += 3 * P;
    c->parts.Om = d; d += 3 * P;
    c->parts.F = d; d += 3 * P;
    c->parts.T = d; d += 3 * P;
    c->parts.Facc = d; d += 3 * P;
    c->parts.Tacc = d; d += 3 * P;
    c->parts.Xold = d; d += 3 * P;
    d += 3 * P;  // spare
    c->parts.D = d; d += P;
    c->parts.rho = d; d += P;
    d += 6 * P;
    int* ip = (int*)d;
    c->parts.fixed = ip; ip += P;
    c->parts.inst = ip;
  }
  c->plist_d = (int*)(w + L.o_plists);
  c->slots = (int*)(w + L.o_slots);
  c->totals = (int*)(w + L.o_totals);
  c->offsets = (int*)(w + L.o_offsets);
  c->totals2 = (int*)(w + L.o_totals2);
  c->offsets2 = (int*)(w + L.o_offsets2);
  {
    int* r = (int*)(w + L.o_ranges);
    const int P = L.ptotal;
    c->lbeg = r; c->lend = r + P; c->pbeg = r + 2 * P; c->pend = r + 3 * P; c->rbeg = r + 4 * P; c->rend = r + 5 * P;
    c->cbeg = r + 6 * P; c->cend = r + 7 * P;
  }
  c->counts = (int*)(w + L.o_counts);
  c->red_partial = (double*)(w + L.o_red);
  c->red_mem = (double*)(w + L.o_redm);
  {
    const size_t nl = (size_t)L.link_cap + L.wall_cap;
    char* b = w + L.o_links;
    c->links.cell = (int*)b; b += nl * 4;
    c->links.q = (int*)b; b += nl * 4;
    c->links.p = (int*)b; b += nl * 4;
    c->links.inst = (int*)b; b += nl * 4;
    c->links.cli_ok = (int*)b; b += nl * 4;
    b = w + L.o_links + align_up(nl * 20);
    c->links.delta = (double*)b;
  }
  c->wall_v = (double*)(w + L.o_wallv);
  {
    const size_t np = L.pair_cap;
    char* b = w + L.o_pairs;
    c->pairs.cell = (int*)b; b += np * 4;
    c->pairs.p = (int*)b; b += np * 4;
    c->pairs.next = (int*)b; b += np * 4;
    b = w + L.o_pairs + align_up(np * 12);
    c->pairs.eps = (double*)b; b += np * 8;
    c->pairs.B = (double*)b; b += np * 8;
    c->pairs.out = (double*)b;
    c->pairs.ostride = (long long)np;
  }
  c->rcell = (int*)(w + L.o_refill);
  c->rpart = c->rcell + L.refill_cap;
  c->scratch = (double*)(w + L.o_scratch);
  {
    const size_t nc = L.cut_cap;
    char* b = w + L.o_cuts;
    c->cuts.slot = (long long*)b; b += align_up(nc * 8);
    c->cuts.d = (double*)b; b += align_up(nc * 24);
    c->cuts.p = (int*)b; b += align_up(nc * 4);
    c->cuts.use = (int*)b;
    c->cuts.count = c->counts + 3;
    c->cuts.err = err_word(c);
    c->cut_x = L.learned ? (float*)(w + L.o_cutx) : nullptr;
    c->mlp_p = (float*)(w + L.o_mlp);
    c->judge = (double*)(w + L.o_judge);
    c->stage = w + L.o_stage;
  }

  // instance table and sweep tiles
  std::vector<int4> tiles;
  for (int i = 0; i < n; ++i) {
    const lbmps_config& cf = cfgs[i];
    InstDev I{};
    I.nx = cf.nx; I.ny = cf.ny; I.nz = cf.nz;
    I.coupling = cf.coupling;
    I.collision = cf.collision;
    I.psm_m = cf.psm_m; I.psm_b = cf.psm_b;
    I.n_sub = eff_nsub(cf);
    I.ncell = L.ncell[i];
    I.pdf_off = L.pdf_off[i];
    I.owner_off = L.owner_off[i];
    I.cellmap_off = L.cellmap_off[i];
    set_relaxation(I, cf);
    for (int k = 0; k < 3; ++k) { I.fext[k] = cf.f_ext[k]; I.grav[k] = cf.gravity[k]; }
    I.part_begin = L.part_begin[i];
    I.part_count = 0;
    I.eps_n = cf.eps_n ? cf.eps_n : 8;
    I.eps_mode = cf.eps_mode;
    I.refill = cf.refill;
    c->inst_h.push_back(I);
    const int tr = eff_tile_rows(cf);
    const int rows = cf.ny * cf.nz;
    for (int r0 = 0; r0 < rows; r0 += tr) tiles.push_back(make_int4(i, r0, std::min(tr, rows - r0), 0));
    if (cf.coupling == LBMPS_PSM) c->have_psm = true;
  }
  c->ntiles = (int)tiles.size();
  c->block = cfgs[0].block_threads ? cfgs[0].block_threads : 256;
  c->grid = cfgs[0].grid_blocks > 0 ? std::min(cfgs[0].grid_blocks, c->ntiles) : c->ntiles;
  c->n_active.assign(n, 0);
  c->wall_groups.assign(n, 0);
  c->fixed_h.assign(L.ptotal, 1);
  c->diam_h.assign(L.ptotal, 0.0);
  c->coupling_of_part.assign(L.ptotal, 0);
  lbmps_status s = LBMPS_OK;
  auto bail = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) { s = LBMPS_EDEVICE; c->last = std::string(what) + ": " + hipGetErrorString(e); }
  };
  bail(hipMemcpyAsync(c->inst_d, c->inst_h.data(), sizeof(InstDev) * n, hipMemcpyHostToDevice, c->st), "copy instances");
  bail(hipMemcpyAsync(c->tiles_d, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, c->st), "copy tiles");
  bail(hipMemsetAsync(c->counts, 0, 16 * 4, c->st), "clear counters");
  bail(hipMemsetAsync(w + L.o_parts, 0, L.o_plists - L.o_parts, c->st), "clear particles");
  if (s == LBMPS_OK) s = fill_int(c, c->owner, L.owner_elems, OWN_FLUID);
  if (s == LBMPS_OK) s = fill_int(c, c->cellmap, L.cellmap_elems, 0x7fffffff);
  if (s == LBMPS_OK) {
    const double u0[3] = {0, 0, 0};
    for (int i = 0; i < n && s == LBMPS_OK; ++i) {
      hipError_t e = launch_init_eq(L.prec, (char*)c->buf[0] + L.pdf_off[i] * L.ssz, L.ncell[i], 1.0, u0, c->st);
      bail(e, "init");
    }
  }
  if (s == LBMPS_OK) bail(hipStreamSynchronize(c->st), "synchronise");
  if (s != LBMPS_OK) {
    *out = c;  // keep the context so that lbmps_last_error can be read
    return s;
  }
  *out = c;
  return LBMPS_OK;
}

void lbmps_destroy(lbmps_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipEventDestroy(c->fork_ev);
    (void)hipEventDestroy(c->join_ev);
    (void)hipStreamDestroy(c->side);
  }
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

int32_t lbmps_particle_base(const lbmps_ctx* c, int32_t inst) {
  if (!c || inst < 0 || inst >= c->L.n) return -1;
  return c->L.part_begin[inst];
}

lbmps_status lbmps_init_equilibrium(lbmps_ctx* c, int32_t inst, double rho, const double u[3]) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!u || !std::isfinite(rho) || !std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2]))
    return fail(c, LBMPS_EINVAL, "non-finite initial state");
  HIPCHK(c, launch_init_eq(c->L.prec, (char*)c->buf[c->cur] + c->L.pdf_off[inst] * c->L.ssz, c->L.ncell[inst], rho, u,
                           c->st));
  return LBMPS_OK;
}

}  // extern "C"

namespace {

// One more group of static wall cells of instance `inst` (kind 0: velocity
// wall with v_wall; 1: outflow with rho_out); every wall link of every
// instance is rebuilt on the host from the owner fields.
lbmps_status add_wall_group(lbmps_ctx* c, int32_t inst, const uint8_t* mask, const double v_wall[3], int kind,
                            double rho_out) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!mask || !v_wall) return fail(c, LBMPS_EINVAL, "null argument");
  if (c->n_mem + c->n_psm > 0) return fail(c, LBMPS_ESTATE, "set static walls before any particles");
  if (!std::isfinite(v_wall[0]) || !std::isfinite(v_wall[1]) || !std::isfinite(v_wall[2]))
    return fail(c, LBMPS_EINVAL, "non-finite wall velocity");
  drop_graph(c);
  if (c->wall_groups[inst] >= WALL_GROUPS) return fail(c, LBMPS_EINVAL, "at most 16 wall groups per instance");
  const lbmps_config& cf = c->cfg[inst];
  const int nx = cf.nx, ny = cf.ny, nz = cf.nz;
  const long long N = c->L.ncell[inst];
  // host owner copy of this instance
  std::vector<int> own(N);
  HIPCHK(c, hipMemcpyAsync(own.data(), c->owner + c->L.owner_off[inst], N * 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const int gid = inst * WALL_GROUPS + c->wall_groups[inst];
  for (long long i = 0; i < N; ++i)
    if (mask[i]) own[i] = -2 - gid;
  // rebuild every wall link of every instance from the host owner fields
  std::vector<int> lc, lq, lp, li;
  for (int k = 0; k < c->L.n; ++k) {
    const lbmps_config& ck = c->cfg[k];
    std::vector<int> ok;
    const std::vector<int>* o = &own;
    if (k != inst) {
      if (c->wall_groups[k] == 0) continue;
      ok.resize(c->L.ncell[k]);
      HIPCHK(c, hipMemcpy(ok.data(), c->owner + c->L.owner_off[k], c->L.ncell[k] * 4, hipMemcpyDeviceToHost));
      o = &ok;
    }
    for (int z = 0; z < ck.nz; ++z)
      for (int y = 0; y < ck.ny; ++y)
        for (int x = 0; x < ck.nx; ++x) {
          const int cell = (z * ck.ny + y) * ck.nx + x;
          if (!own_is_fluid((*o)[cell])) continue;
          for (int q = 1; q < 19; ++q) {
            const int xi = (x + cx(q) + ck.nx) % ck.nx, yi = (y + cy(q) + ck.ny) % ck.ny, zi = (z + cz(q) + ck.nz) % ck.nz;
            const int nb = (*o)[(zi * ck.ny + yi) * ck.nx + xi];
            if (nb <= -2) {
              lc.push_back(cell); lq.push_back(q); lp.push_back(nb); li.push_back(k);
            }
          }
        }
  }
  (void)nx; (void)ny; (void)nz;
  if ((long long)lc.size() > c->L.wall_cap) return fail(c, LBMPS_ENOMEM, "wall_link_cap exceeded");
  c->wall_groups[inst]++;
  double rec[WALL_REC] = {v_wall[0], v_wall[1], v_wall[2], (double)kind, rho_out, 0.0, 0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(c->wall_v + WALL_REC * gid, rec, sizeof(rec), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->owner + c->L.owner_off[inst], own.data(), N * 4, hipMemcpyHostToDevice, c->st));
  const size_t nl = lc.size();
  std::vector<int> zeros(nl, 0);
  std::vector<double> half(nl, 0.5);
  if (nl) {
    HIPCHK(c, hipMemcpyAsync(c->links.cell, lc.data(), nl * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->links.q, lq.data(), nl * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->links.p, lp.data(), nl * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->links.inst, li.data(), nl * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->links.cli_ok, zeros.data(), nl * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->links.delta, half.data(), nl * 8, hipMemcpyHostToDevice, c->st));
  }
  c->n_wall = (int)nl;
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LBMPS_OK;
}

}  // namespace

extern "C" {

lbmps_status lbmps_set_static_solid(lbmps_ctx* c, int32_t inst, const uint8_t* mask, const double v_wall[3]) {
  return add_wall_group(c, inst, mask, v_wall, 0, 1.0);
}

lbmps_status lbmps_set_outflow(lbmps_ctx* c, int32_t inst, const uint8_t* mask, double rho_out) {
  if (!c) return LBMPS_EINVAL;
  if (!std::isfinite(rho_out) || !(rho_out > 0.0)) return fail(c, LBMPS_EINVAL, "rho_out must be positive");
  const double zero[3] = {0.0, 0.0, 0.0};
  return add_wall_group(c, inst, mask, zero, 1, rho_out);
}

lbmps_status lbmps_set_viscosity(lbmps_ctx* c, int32_t inst, double nu) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!(nu > 0.0) || !std::isfinite(nu)) return fail(c, LBMPS_EINVAL, "nu must be positive");
  drop_graph(c);
  c->cfg[inst].nu = nu;
  set_relaxation(c->inst_h[inst], c->cfg[inst]);
  HIPCHK(c, hipMemcpyAsync(c->inst_d + inst, &c->inst_h[inst], sizeof(InstDev), hipMemcpyHostToDevice, c->st));
  // the B2 weights of the overlap pairs depend on tau
  if (c->cfg[inst].coupling == LBMPS_PSM && c->n_psm) {
    s = rebuild_psm(c, c->st);
    if (s) return s;
  }
  return check_device_errors(c);
}

lbmps_status lbmps_set_gravity(lbmps_ctx* c, int32_t inst, const double g[3]) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!g || !std::isfinite(g[0]) || !std::isfinite(g[1]) || !std::isfinite(g[2]))
    return fail(c, LBMPS_EINVAL, "non-finite gravity");
  drop_graph(c);
  for (int k = 0; k < 3; ++k) {
    c->cfg[inst].gravity[k] = g[k];
    c->inst_h[inst].grav[k] = g[k];
  }
  HIPCHK(c, hipMemcpyAsync(c->inst_d + inst, &c->inst_h[inst], sizeof(InstDev), hipMemcpyHostToDevice, c->st));
  return check_device_errors(c);
}

lbmps_status lbmps_set_particles(lbmps_ctx* c, int32_t inst, int32_t n, const lbmps_particle* hp) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  drop_graph(c);
  const lbmps_config& cf = c->cfg[inst];
  if (n < 0 || n > cf.max_particles) return fail(c, LBMPS_EINVAL, "particle count exceeds max_particles");
  if (n > 0 && !hp) return fail(c, LBMPS_EINVAL, "null particle array");
  if (n > 0 && cf.coupling == LBMPS_PSM && cf.eps_mode == LBMPS_EPS_LEARNED && !c->mlp_set)
    return fail(c, LBMPS_ESTATE, "learned eps_s: call lbmps_set_eps_model before setting particles");
  const int mind = std::min(cf.nx, std::min(cf.ny, cf.nz));
  const double L3[3] = {(double)cf.nx, (double)cf.ny, (double)cf.nz};
  const int P = c->L.ptotal;
  const int base = c->L.part_begin[inst];
  std::vector<double> X(3 * n), U(3 * n), Om(3 * n), D(n), rho(n);
  std::vector<int> fixed(n), pinst(n, inst);
  for (int i = 0; i < n; ++i) {
    const lbmps_particle& p = hp[i];
    bool fin = std::isfinite(p.D) && std::isfinite(p.rho_p);
    for (int k = 0; k < 3; ++k) fin = fin && std::isfinite(p.X[k]) && std::isfinite(p.U[k]) && std::isfinite(p.Omega[k]);
    if (!fin) return fail(c, LBMPS_EINVAL, "non-finite particle value");
    if (!(p.D > 0) || p.D > cf.max_diameter || p.D + 6 > mind) return fail(c, LBMPS_EINVAL, "invalid particle diameter");
    if (!(p.rho_p > 0)) return fail(c, LBMPS_EINVAL, "particle density must be positive");
    for (int k = 0; k < 3; ++k) {
      double x = std::fmod(p.X[k], L3[k]);
      if (x < 0) x += L3[k];
      if (x >= L3[k]) x -= L3[k];
      X[3 * i + k] = x;
      U[3 * i + k] = p.U[k];
      Om[3 * i + k] = p.Omega[k];
    }
    D[i] = p.D;
    rho[i] = p.rho_p;
    fixed[i] = p.fixed ? 1 : 0;
  }
  (void)P;
  HIPCHK(c, hipStreamSynchronize(c->st));
  HIPCHK(c, hipMemcpy(c->parts.X + 3 * base, X.data(), 24 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.Xold + 3 * base, X.data(), 24 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.U + 3 * base, U.data(), 24 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.Om + 3 * base, Om.data(), 24 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.D + base, D.data(), 8 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.rho + base, rho.data(), 8 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.fixed + base, fixed.data(), 4 * n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->parts.inst + base, pinst.data(), 4 * n, hipMemcpyHostToDevice));
  std::vector<double> z(3 * std::max(n, 1), 0.0);
  if (n) {
    HIPCHK(c, hipMemcpy(c->parts.F + 3 * base, z.data(), 24 * n, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->parts.T + 3 * base, z.data(), 24 * n, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->parts.Facc + 3 * base, z.data(), 24 * n, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->parts.Tacc + 3 * base, z.data(), 24 * n, hipMemcpyHostToDevice));
  }
  c->n_active[inst] = n;
  for (int i = 0; i < n; ++i) {
    c->fixed_h[base + i] = fixed[i];
    c->diam_h[base + i] = D[i];
    c->coupling_of_part[base + i] = cf.coupling;
  }
  c->inst_h[inst].part_count = n;
  HIPCHK(c, hipMemcpy(c->inst_d + inst, &c->inst_h[inst], sizeof(InstDev), hipMemcpyHostToDevice));
  // particle lists: MEM particles first, then PSM, in global index order
  std::vector<int> lm, lps;
  c->mem_moving = c->psm_moving = false;
  for (int k = 0; k < c->L.n; ++k) {
    const int b = c->L.part_begin[k];
    const int cp = c->cfg[k].coupling;
    for (int i = 0; i < c->n_active[k]; ++i) {
      if (cp == LBMPS_MEM_BB || cp == LBMPS_MEM_CLI) {
        lm.push_back(b + i);
        if (!c->fixed_h[b + i]) c->mem_moving = true;
      } else if (cp == LBMPS_PSM) {
        lps.push_back(b + i);
        if (!c->fixed_h[b + i]) c->psm_moving = true;
      }
    }
  }
  c->n_mem = (int)lm.size();
  c->n_psm = (int)lps.size();
  update_psm_exact(c);
  std::vector<int> all(lm);
  all.insert(all.end(), lps.begin(), lps.end());
  if (!all.empty()) HIPCHK(c, hipMemcpy(c->plist_d, all.data(), 4 * all.size(), hipMemcpyHostToDevice));
  // mapping
  if (cf.coupling == LBMPS_MEM_BB || cf.coupling == LBMPS_MEM_CLI) {
    hipLaunchKernelGGL(reset_owner_kernel, dim3((unsigned)((c->L.ncell[inst] + 255) / 256)), dim3(256), 0, c->st,
                       c->owner + c->L.owner_off[inst], c->L.ncell[inst]);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, launch_mem_map(mem_list(c), c->n_mem, c->L.side, nsplit_for(c->n_mem, c->L.side), c->inst_d, c->parts,
                             c->owner, c->st));
    s = rebuild_mem(c, false, c->st);
    if (s) return s;
  } else if (cf.coupling == LBMPS_PSM) {
    s = rebuild_psm(c, c->st);
    if (s) return s;
  }
  return check_device_errors(c);
}

// Side stream and events of the overlapped MEM remap, created on first use
// (default priority).  False when they cannot be created: the remap then
// runs in order on the context's stream.
static bool ensure_side_stream(lbmps_ctx* c) {
  if (c->side) return true;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
  // both streams are on one device: no system-scope fence (cache writeback) is needed
  const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipEventCreateWithFlags(&a, fl) != hipSuccess || hipEventCreateWithFlags(&b, fl) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    (void)hipStreamDestroy(s);
    return false;
  }
  c->side = s;
  c->fork_ev = a;
  c->join_ev = b;
  return true;
}

// A stream under graph capture keeps all work on itself (no fork).
static bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

static lbmps_status step_sweeps(lbmps_ctx* c, int32_t n);

lbmps_status lbmps_step(lbmps_ctx* c, int32_t n) {
  if (!c) return LBMPS_EINVAL;
  if (n < 0) return fail(c, LBMPS_EINVAL, "negative step count");
  const Layout& L = c->L;
  if (L.mem_nsub && (n % L.mem_nsub)) return fail(c, LBMPS_EINVAL, "MEM steps must be a multiple of n_sub");
  if (L.psm_nsub && (n % L.psm_nsub)) return fail(c, LBMPS_EINVAL, "PSM steps must be a multiple of n_sub");
  lbmps_status r = step_sweeps(c, n);
  if (c->join_pending) {  // only after an error: the forked remap still joins the stream
    (void)hipStreamWaitEvent(c->st, c->join_ev, 0);
    c->join_pending = false;
  }
  return r;
}

lbmps_status lbmps_step_noalloc(lbmps_ctx* c, int32_t n) {
  if (!c) return LBMPS_EINVAL;
  if (n < 0) return fail(c, LBMPS_EINVAL, "negative step count");
  const Layout& L = c->L;
  if (L.mem_nsub && (n % L.mem_nsub)) return fail(c, LBMPS_EINVAL, "MEM steps must be a multiple of n_sub");
  if (L.psm_nsub && (n % L.psm_nsub)) return fail(c, LBMPS_EINVAL, "PSM steps must be a multiple of n_sub");
  if (c->timing) return fail(c, LBMPS_ESTATE, "switch timing off before lbmps_step_noalloc");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(c, LBMPS_ESTATE, "lbmps_step_noalloc: the context's device must be current");
  // chunk sums of the overlap records (rows of red_blocks per PSM particle),
  // then n_sub sets of link chunk sums (rows of link_blocks per MEM particle)
  const size_t psm_bytes = align_up((size_t)c->n_psm * L.red_blocks * 6 * 8);
  const size_t mem_bytes = (size_t)c->n_mem * L.link_blocks * 6 * 8 * std::max(1, L.mem_nsub);
  if (psm_bytes + mem_bytes > LBMPS_NOALLOC_SCRATCH_BYTES)
    return fail(c, LBMPS_ENOMEM, "lbmps_step_noalloc: the context needs " + std::to_string(psm_bytes + mem_bytes) +
                                     " bytes of scratch, more than the " +
                                     std::to_string((size_t)LBMPS_NOALLOC_SCRATCH_BYTES) + " available");
  void* base = nullptr;
  lbmps_status s = scratch_address(c, dev, &base);
  if (s) return s;
  double* const own_partial = c->red_partial;
  double* const own_mem = c->red_mem;
  c->red_partial = (double*)base;
  c->red_mem = (double*)((char*)base + psm_bytes);
  c->in_order = true;
  s = step_sweeps(c, n);
  c->in_order = false;
  c->red_partial = own_partial;
  c->red_mem = own_mem;
  return s;
}

// Per-particle PSM force/torque of the sweep: the chunk sums the overlap kernel
// formed (chunked) or a reduction of the per-pair records (inline mode), then
// the fixed-order finishing sum, with the rigid-body step when insts is given.
static hipError_t psm_sums(lbmps_ctx* c, bool chunked, const InstDev* insts, hipStream_t st) {
  const Layout& L = c->L;
  if (chunked)
    return launch_finish_sums(psm_list(c), c->n_psm, c->pbeg, c->pend, RED_CHUNK, L.red_blocks, c->red_partial, 1, 0,
                              c->parts, insts, err_word(c), st);
  return launch_reduce(psm_list(c), c->n_psm, c->pbeg, c->pend, 0, c->pairs.out, c->pairs.ostride, c->parts,
                       L.red_blocks, c->red_partial, insts, err_word(c), st);
}

static lbmps_status step_sweeps(lbmps_ctx* c, int32_t n) {
  const Layout& L = c->L;
  unsigned* err = err_word(c);
  for (int s = 0; s < n; ++s) {
    void* src = c->buf[c->cur];
    void* dst = c->buf[1 - c->cur];
    // a sweep beside which the PSM lists are being rebuilt reads none of them:
    // it leaves every overlapped cell to the overlap kernel after the join
    // (all modes give the same bits)
    const bool lists_pending = c->join_pending && c->join_lists;
    const int pm = c->n_psm && !lists_pending ? c->psm_mode : PSM_SEPARATE;
    // outside the inline mode the overlap kernel also forms the chunk sums of
    // the force/torque terms (no record round trip); finish_sums adds them
    const PsmSums sums{psm_list(c), c->n_psm, c->pbeg, c->pend, L.red_blocks, c->red_partial};
    const PsmSums* psum = pm == PSM_FUSED ? nullptr : &sums;
    if (pm == PSM_STAGED)  // overlapped cells first, from the same pre-collision values
      HIPCHK(c, launch_psm_collide(L.prec, L.psm_m, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs,
                                   c->cellmap, src, dst, c->stage, L.pair_cap, false, c->st, psum));
    const bool timed = c->timing && (c->timing_seq++ % c->timing_stride) == 0;
    if (timed) {
      if (c->ev_used + 2 > c->ev.size()) {  // every event of the pool is recorded: read them out
        lbmps_status r = harvest_timing(c);
        if (r) return r;
      }
      HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->st));
    }
    HIPCHK(c, launch_sweep(L.prec, c->inst_d, c->tiles_d, c->ntiles, c->grid, c->block, L.max_tile_cells,
                           c->cfg[0].sweep_flags, pm == PSM_FUSED ? 1 : pm == PSM_STAGED ? 2 : 0, src, dst,
                           pm != PSM_SEPARATE ? c->cellmap : nullptr, c->pairs, c->parts, c->stage, L.pair_cap,
                           c->st));
    if (timed) {
      HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->st));
      c->ev_used += 2;
    }
    // the reduction that completes a rigid-body step also takes it
    const bool psm_rb = c->n_psm && ((c->sweeps + 1) % L.psm_nsub) == 0;
    const bool mem_rb = c->n_mem && ((c->sweeps + 1) % L.mem_nsub) == 0;
    if (c->join_pending) {  // the work forked after the previous rigid-body step
      HIPCHK(c, hipStreamWaitEvent(c->st, c->join_ev, 0));
      c->join_pending = false;
      if (c->join_resweep)  // a MEM remap has refilled cells of src since the sweep read them
        HIPCHK(c, launch_resweep_cells(L.prec, c->counts + 2, L.refill_cap, c->rcell, c->rpart, c->inst_d, c->parts,
                                       src, dst, c->st));
    }
    if (c->n_psm) {
      if (pm != PSM_STAGED)  // after the sweep: every overlapped cell, or (inline mode) the shared ones
        HIPCHK(c, launch_psm_collide(L.prec, L.psm_m, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs,
                                     c->cellmap, src, dst, nullptr, 0, pm == PSM_FUSED, c->st, psum));
      if (!psm_rb)  // the rigid-body sweep's sum goes with the rebuild, below
        HIPCHK(c, psm_sums(c, psum != nullptr, nullptr, c->st));
    }
    if (c->n_mem || c->n_wall) {
      // the link sums of the sweeps of a rigid-body step wait in their own sets
      // and are added up (in sweep order) after the last one, below
      const int set = c->n_mem ? (int)(c->sweeps % L.mem_nsub) : 0;
      HIPCHK(c, launch_links_bc(L.prec, c->n_wall, mem_list(c), c->n_mem, c->lbeg, c->lend, L.link_blocks, c->links,
                                c->wall_v, c->inst_d, c->parts, src, dst, c->red_mem, set, c->st));
    }
    c->cur = 1 - c->cur;
    c->sweeps++;
    // The PSM rebuild and the MEM remap after a rigid-body step, with another
    // sweep to come in this call, run on the side stream (one after the
    // other: their list stages share work arrays) beside that sweep: the sweep
    // reads no PSM list (it leaves the PSM cells to the overlap kernel after
    // the join), and its results depend on the cells a remap uncovers only
    // through what those cells push, which the re-sweep after the join
    // recomputes from the refilled values.
    // The force sums that complete a rigid-body step, with the rigid-body
    // step, go with the rebuild or remap (the next sweep does not read
    // particle state), so they leave the critical path too when those are
    // forked.
    const bool psm_work = psm_rb && c->psm_moving, mem_work = mem_rb && c->mem_moving;
    const bool fork = (psm_work || mem_work) && s + 1 < n && !c->in_order && !stream_capturing(c->st) &&
                      ensure_side_stream(c);
    hipStream_t ws = fork ? c->side : c->st;
    if (fork) {
      HIPCHK(c, hipEventRecord(c->fork_ev, c->st));
      HIPCHK(c, hipStreamWaitEvent(c->side, c->fork_ev, 0));
    }
    if (psm_rb)
      HIPCHK(c, psm_sums(c, psum != nullptr, c->inst_d, psm_work ? ws : c->st));
    if (mem_rb)
      HIPCHK(c, launch_finish_sums(mem_list(c), c->n_mem, c->lbeg, c->lend, SUM_THREADS, L.link_blocks, c->red_mem,
                                   L.mem_nsub, (long long)c->n_mem * L.link_blocks * 6, c->parts, c->inst_d, err,
                                   mem_work ? ws : c->st));
    if (psm_work || mem_work) {
      lbmps_status r = psm_work ? rebuild_psm(c, ws) : LBMPS_OK;
      if (!r && mem_work) r = remap_mem(c, ws);
      if (fork) {
        HIPCHK(c, hipEventRecord(c->join_ev, c->side));
        c->join_pending = true;
        c->join_resweep = mem_work;
        c->join_lists = psm_work;
      }
      if (r) return r;
    }
  }
  return LBMPS_OK;
}

lbmps_status lbmps_set_launch(lbmps_ctx* c, int32_t block_threads, int32_t grid_blocks, int32_t sweep_flags) {
  if (!c) return LBMPS_EINVAL;
  if (block_threads < 0 || block_threads > 256 || (block_threads % 64)) return fail(c, LBMPS_EINVAL, "bad block size");
  if (grid_blocks < 0 || (sweep_flags & ~SWEEP_FLAGS_ALL) || __builtin_popcount(sweep_flags & SWEEP_PSM_MODES) > 1 ||
      (sweep_flags & SWEEP_WG_CAP_MASK) == SWEEP_WG_CAP_MASK)
    return fail(c, LBMPS_EINVAL, "bad grid or flags");
  if (sweep_flags & SWEEP_CELL_PAIRS)
    for (const auto& cf : c->cfg)
      if (cf.nx & 1) return fail(c, LBMPS_EINVAL, "cell pairs need an even nx");
  for (const auto& cf : c->cfg)
    if (!quads_ok(sweep_flags, cf.precision, cf.nx))
      return fail(c, LBMPS_EINVAL, "cell quads need FP16/BF16 storage, nx a multiple of 4, and neither bit 3 nor bit 7");
  drop_graph(c);
  c->block = block_threads ? block_threads : 256;
  c->grid = grid_blocks > 0 ? std::min(grid_blocks, c->ntiles) : c->ntiles;
  for (auto& cf : c->cfg) cf.sweep_flags = sweep_flags;
  update_psm_exact(c);
  return LBMPS_OK;
}

static int gcd_int(int a, int b) { return b ? gcd_int(b, a % b) : a; }

lbmps_status lbmps_step_graph(lbmps_ctx* c, int32_t n) {
  if (!c) return LBMPS_EINVAL;
  const Layout& L = c->L;
  int period = 2;
  for (int ns : {L.mem_nsub, L.psm_nsub})
    if (ns > 0) period = period / gcd_int(period, ns) * ns;
  if (n < 0 || n % period) return fail(c, LBMPS_EINVAL, "graph steps must be a multiple of the capture period");
  if (c->sweeps % period) return fail(c, LBMPS_ESTATE, "graph replay must start at a rigid-body step boundary");
  if (!c->st) return fail(c, LBMPS_EINVAL, "graph capture needs a non-default stream");
  if (c->timing) return fail(c, LBMPS_ESTATE, "disable timing before graph replay");
  if (c->graph_exec && (c->graph_period != period || c->graph_cur != c->cur)) drop_graph(c);
  if (!c->graph_exec) {
    HIPCHK(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    const long long sweeps0 = c->sweeps;
    const int cur0 = c->cur;
    lbmps_status r = lbmps_step(c, period);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->st, &g);
    // the captured launches have not run: restore the host-side counters
    c->sweeps = sweeps0;
    c->cur = cur0;
    if (r) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return fail(c, LBMPS_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    c->graph_period = period;
    c->graph_cur = c->cur;
  }
  for (int k = 0; k < n / period; ++k) {
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->st));
    c->sweeps += period;
  }
  return LBMPS_OK;
}

lbmps_status lbmps_sync(lbmps_ctx* c) {
  if (!c) return LBMPS_EINVAL;
  return check_device_errors(c);
}

lbmps_status lbmps_get_particles(lbmps_ctx* c, int32_t inst, int32_t n, lbmps_particle_state* out) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (n != c->n_active[inst]) return fail(c, LBMPS_EINVAL, "n must equal the number of particles set");
  if (n == 0) return check_device_errors(c);
  if (!out) return fail(c, LBMPS_EINVAL, "null output");
  const int b = c->L.part_begin[inst];
  std::vector<double> F(3 * n), T(3 * n), U(3 * n), Om(3 * n), X(3 * n);
  HIPCHK(c, hipMemcpyAsync(F.data(), c->parts.F + 3 * b, 24 * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(T.data(), c->parts.T + 3 * b, 24 * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(U.data(), c->parts.U + 3 * b, 24 * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(Om.data(), c->parts.Om + 3 * b, 24 * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(X.data(), c->parts.X + 3 * b, 24 * n, hipMemcpyDeviceToHost, c->st));
  s = check_device_errors(c);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      out[i].F[k] = F[3 * i + k];
      out[i].T[k] = T[3 * i + k];
      out[i].U[k] = U[3 * i + k];
      out[i].Omega[k] = Om[3 * i + k];
      out[i].X[k] = X[3 * i + k];
    }
  return s;
}

lbmps_status lbmps_get_fields(lbmps_ctx* c, int32_t inst, double* rho, double* u) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!rho || !u) return fail(c, LBMPS_EINVAL, "null output");
  const Layout& L = c->L;
  const long long N = L.ncell[inst];
  const void* buf = (char*)c->buf[c->cur] + L.pdf_off[inst] * L.ssz;
  const int* own = c->owner + L.owner_off[inst];
  std::vector<double> h(4 * L.chunk);
  for (long long c0 = 0; c0 < N; c0 += L.chunk) {
    const long long n = std::min(L.chunk, N - c0);
    HIPCHK(c, launch_fields(L.prec, buf, N, c0, n, own, c->inst_h[inst].fext, c->scratch, c->st));
    if (c->cfg[inst].coupling == LBMPS_PSM && c->n_psm)
      HIPCHK(c, launch_psm_fields(L.prec, c->counts + 1, L.pair_cap, c->inst_d, c->parts, c->pairs, c->cellmap,
                                  c->buf[c->cur], inst, c0, n, c->scratch, c->st));
    HIPCHK(c, hipMemcpyAsync(h.data(), c->scratch, 4 * n * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::memcpy(rho + c0, h.data(), n * 8);
    for (int a = 0; a < 3; ++a) std::memcpy(u + a * N + c0, h.data() + (a + 1) * n, n * 8);
  }
  return check_device_errors(c);
}

lbmps_status lbmps_get_pdfs(lbmps_ctx* c, int32_t inst, double* g) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!g) return fail(c, LBMPS_EINVAL, "null output");
  const Layout& L = c->L;
  const long long N = L.ncell[inst];
  const char* buf = (char*)c->buf[c->cur] + L.pdf_off[inst] * L.ssz;
  const long long ch = 4 * L.chunk;
  for (int q = 0; q < 19; ++q)
    for (long long c0 = 0; c0 < N; c0 += ch) {
      const long long n = std::min(ch, N - c0);
      HIPCHK(c, launch_to_f64(L.prec, buf, q, c0, c->scratch, n, c->st));
      HIPCHK(c, hipMemcpyAsync(g + (long long)q * N + c0, c->scratch, n * 8, hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
    }
  std::vector<int> own(N);
  HIPCHK(c, hipMemcpy(own.data(), c->owner + L.owner_off[inst], N * 4, hipMemcpyDeviceToHost));
  for (long long i = 0; i < N; ++i)
    if (!own_is_fluid(own[i]))
      for (int q = 0; q < 19; ++q) g[(long long)q * N + i] = 0.0;
  return check_device_errors(c);
}

lbmps_status lbmps_set_pdfs(lbmps_ctx* c, int32_t inst, const double* g) {
  lbmps_status s = check_inst(c, inst);
  if (s) return s;
  if (!g) return fail(c, LBMPS_EINVAL, "null input");
  const Layout& L = c->L;
  const long long N = L.ncell[inst];
  char* buf = (char*)c->buf[c->cur] + L.pdf_off[inst] * L.ssz;
  const long long ch = 4 * L.chunk;
  for (int q = 0; q < 19; ++q)
    for (long long c0 = 0; c0 < N; c0 += ch) {
      const long long n = std::min(ch, N - c0);
      HIPCHK(c, hipMemcpyAsync(c->scratch, g + (long long)q * N + c0, n * 8, hipMemcpyHostToDevice, c->st));
      HIPCHK(c, launch_from_f64(L.prec, c->scratch, buf, q, c0, n, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
    }
  return LBMPS_OK;
}

lbmps_status lbmps_get_links(lbmps_ctx* c, int64_t cap, int32_t* cell, int32_t* q, int32_t* particle, double* delta,
                             int64_t* n_out) {
  if (!c || !n_out) return LBMPS_EINVAL;
  int cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->counts + 0, 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (c->n_mem == 0) cnt = 0;
  cnt = std::min(cnt, c->L.link_cap);
  *n_out = cnt;
  const long long n = std::min<long long>(cap, cnt);
  const int b = c->n_wall;
  if (n > 0) {
    HIPCHK(c, hipMemcpy(cell, c->links.cell + b, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(q, c->links.q + b, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(particle, c->links.p + b, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(delta, c->links.delta + b, n * 8, hipMemcpyDeviceToHost));
  }
  return check_device_errors(c);
}

lbmps_status lbmps_get_overlaps(lbmps_ctx* c, int64_t cap, int32_t* cell, int32_t* particle, double* eps,
                                int64_t* n_out) {
  if (!c || !n_out) return LBMPS_EINVAL;
  int cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->counts + 1, 4, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (c->n_psm == 0) cnt = 0;
  cnt = std::min(cnt, c->L.pair_cap);
  *n_out = cnt;
  const long long n = std::min<long long>(cap, cnt);
  if (n > 0) {
    HIPCHK(c, hipMemcpy(cell, c->pairs.cell, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(particle, c->pairs.p, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(eps, c->pairs.eps, n * 8, hipMemcpyDeviceToHost));
  }
  return check_device_errors(c);
}

lbmps_status lbmps_set_timing(lbmps_ctx* c, int32_t enable) {
  if (!c) return LBMPS_EINVAL;
  lbmps_status s = harvest_timing(c);
  if (s) return s;
  if (enable < 0) return fail(c, LBMPS_EINVAL, "timing stride must be >= 0");
  // the event pool is created here, not at the first timed launch, so that a
  // timed region pays only for recording the events
  while (enable > 0 && c->ev.size() < TIMING_EVENTS) {
    hipEvent_t e;
    // timestamps only (read after a stream synchronisation): no system-scope fence
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c->ev.push_back(e);
  }
  c->timing = enable != 0;
  c->timing_stride = enable > 0 ? enable : 1;
  c->timing_seq = 0;
  c->sweep_ms = 0.0;
  c->sweep_launches = 0;
  return LBMPS_OK;
}

lbmps_status lbmps_get_timing(lbmps_ctx* c, double* sweep_ms, int64_t* launches) {
  if (!c || !sweep_ms || !launches) return LBMPS_EINVAL;
  lbmps_status s = harvest_timing(c);
  if (s) return s;
  *sweep_ms = c->sweep_ms;
  *launches = c->sweep_launches;
  return LBMPS_OK;
}

lbmps_status lbmps_set_eps_model(lbmps_ctx* c, const float* hp, double r_min, double r_max) {
  if (!c) return LBMPS_EINVAL;
  if (!hp) return fail(c, LBMPS_EINVAL, "null parameters");
  if (!std::isfinite(r_min) || !std::isfinite(r_max) || r_min > r_max) return fail(c, LBMPS_EINVAL, "bad radius range");
  const int np = mlp_nparam();
  for (int k = 0; k < np; ++k)
    if (!std::isfinite(hp[k])) return fail(c, LBMPS_EINVAL, "non-finite parameter");
  drop_graph(c);
  HIPCHK(c, hipMemcpyAsync(c->mlp_p, hp, (size_t)np * 4, hipMemcpyHostToDevice, c->st));
  c->mlp_set = true;
  c->mlp_rmin = r_min;
  c->mlp_rmax = r_max;
  update_psm_exact(c);
  lbmps_status s = rebuild_psm(c, c->st);
  if (s) return s;
  return check_device_errors(c);
}

lbmps_status lbmps_rebuild_overlaps(lbmps_ctx* c) {
  if (!c) return LBMPS_EINVAL;
  return rebuild_psm(c, c->st);
}

lbmps_status lbmps_eps_judge(lbmps_ctx* c, int32_t stride, double out[3]) {
  if (!c || !out) return LBMPS_EINVAL;
  if (stride < 1) return fail(c, LBMPS_EINVAL, "stride must be >= 1");
  out[0] = out[1] = out[2] = 0.0;
  if (!c->L.learned || c->n_psm == 0) return check_device_errors(c);
  HIPCHK(c, hipMemsetAsync(c->judge, 0, 3 * 8, c->st));
  HIPCHK(c, launch_psm_judge(c->inst_d, c->parts, c->slots, c->cuts, c->L.cut_cap, stride, c->judge, c->st));
  double h[3];
  HIPCHK(c, hipMemcpyAsync(h, c->judge, 3 * 8, hipMemcpyDeviceToHost, c->st));
  lbmps_status s = check_device_errors(c);
  if (s) return s;
  out[0] = h[2] > 0 ? h[0] / h[2] : 0.0;
  out[1] = h[1];
  out[2] = h[2];
  return LBMPS_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------- trainer
struct lbmps_mlp {
  hipStream_t st = nullptr;
  long long cap = 0, n = 0;
  float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *X = nullptr, *T = nullptr, *y = nullptr,
        *partial = nullptr;
  double* rd = nullptr;
  int step = 0;
  int n_inputs = 5;  // features in use (the rest are zero)
  bool labelled = false;
  std::string last;
};

namespace {

constexpr long long MLP_MAX_BATCH = LBMPS_MLP_MAX_BATCH;

struct MlpLayout {
  size_t P, m, v, grad, partial, rd, X, T, y, total;
};

MlpLayout mlp_layout(long long cap) {
  MlpLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  const size_t np = (size_t)mlp_nparam();
  L.P = take(np * 4);
  L.m = take(np * 4);
  L.v = take(np * 4);
  L.grad = take(np * 4);
  L.partial = take((size_t)(MLP_MAX_BATCH / 32) * np * 4);
  L.rd = take((size_t)cap * 4 * 8);
  L.X = take((size_t)cap * 8 * 4);
  L.T = take((size_t)cap * 4);
  L.y = take((size_t)cap * 4);
  L.total = o;
  return L;
}

lbmps_status mfail(lbmps_mlp* m, lbmps_status s, const std::string& msg) {
  if (m) m->last = msg;
  return s;
}

#define MHIPCHK(m, expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return mfail(m, LBMPS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

long long gcd_ll(long long a, long long b) { return b ? gcd_ll(b, a % b) : a; }

lbmps_status check_order(lbmps_mlp* m, long long mult, long long add) {
  if (mult < 1 || mult >= std::max(m->n, 2LL) || gcd_ll(mult, m->n) != 1 || add < 0 || add >= m->n)
    return mfail(m, LBMPS_EINVAL, "sample order needs 1 <= mult < n coprime to n and 0 <= add < n");
  return LBMPS_OK;
}

}  // namespace

extern "C" {

size_t lbmps_mlp_workspace_bytes(int64_t max_samples) {
  if (max_samples < 1 || max_samples >= (1LL << 31)) return 0;
  return mlp_layout(max_samples).total;
}

lbmps_status lbmps_mlp_create(int64_t cap, void* ws, size_t bytes, void* stream, lbmps_mlp** out) {
  if (!out) return LBMPS_EINVAL;
  *out = nullptr;
  if (cap < 1 || cap >= (1LL << 31)) return LBMPS_EINVAL;
  const MlpLayout L = mlp_layout(cap);
  if (!ws || bytes < L.total) return LBMPS_ENOMEM;
  lbmps_mlp* m = new lbmps_mlp();
  char* w = (char*)ws;
  m->st = (hipStream_t)stream;
  m->cap = cap;
  m->P = (float*)(w + L.P);
  m->m = (float*)(w + L.m);
  m->v = (float*)(w + L.v);
  m->grad = (float*)(w + L.grad);
  m->partial = (float*)(w + L.partial);
  m->rd = (double*)(w + L.rd);
  m->X = (float*)(w + L.X);
  m->T = (float*)(w + L.T);
  m->y = (float*)(w + L.y);
  *out = m;
  MHIPCHK(m, hipMemsetAsync(w, 0, L.partial, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  return LBMPS_OK;
}

void lbmps_mlp_destroy(lbmps_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  delete m;
}

lbmps_status lbmps_mlp_set_params(lbmps_mlp* m, const float* hp) {
  if (!m) return LBMPS_EINVAL;
  if (!hp) return mfail(m, LBMPS_EINVAL, "null parameters");
  const size_t np = (size_t)mlp_nparam();
  MHIPCHK(m, hipMemcpyAsync(m->P, hp, np * 4, hipMemcpyHostToDevice, m->st));
  MHIPCHK(m, hipMemsetAsync(m->m, 0, np * 4, m->st));
  MHIPCHK(m, hipMemsetAsync(m->v, 0, np * 4, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  m->step = 0;
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_get_params(lbmps_mlp* m, float* hp) {
  if (!m) return LBMPS_EINVAL;
  if (!hp) return mfail(m, LBMPS_EINVAL, "null output");
  MHIPCHK(m, hipMemcpyAsync(hp, m->P, (size_t)mlp_nparam() * 4, hipMemcpyDeviceToHost, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_set_samples(lbmps_mlp* m, int64_t n, const double* rd) {
  if (!m) return LBMPS_EINVAL;
  if (n < 1 || n > m->cap) return mfail(m, LBMPS_EINVAL, "sample count out of range");
  if (!rd) return mfail(m, LBMPS_EINVAL, "null samples");
  for (long long s = 0; s < n; ++s) {
    bool ok = rd[4 * s] > 0;
    for (int k = 0; k < 4; ++k) ok = ok && std::isfinite(rd[4 * s + k]);
    if (!ok) return mfail(m, LBMPS_EINVAL, "samples need finite values and R > 0");
  }
  MHIPCHK(m, hipMemcpyAsync(m->rd, rd, (size_t)n * 32, hipMemcpyHostToDevice, m->st));
  MHIPCHK(m, launch_mlp_features(m->rd, n, m->n_inputs, m->X, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  m->n = n;
  m->labelled = false;
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_set_inputs(lbmps_mlp* m, int32_t n_inputs) {
  if (!m) return LBMPS_EINVAL;
  if (n_inputs != 3 && n_inputs != 5) return mfail(m, LBMPS_EINVAL, "n_inputs must be 3 or 5");
  m->n_inputs = n_inputs;
  if (m->n > 0) {  // the features of the current samples again (the targets stay)
    MHIPCHK(m, launch_mlp_features(m->rd, m->n, m->n_inputs, m->X, m->st));
    MHIPCHK(m, hipStreamSynchronize(m->st));
  }
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_label(lbmps_mlp* m, int32_t eps_n) {
  if (!m) return LBMPS_EINVAL;
  if (m->n < 1) return mfail(m, LBMPS_ESTATE, "set samples first");
  if (eps_n < 1 || eps_n > 64) return mfail(m, LBMPS_EINVAL, "eps_n must be 1..64");
  MHIPCHK(m, launch_psm_label(m->rd, m->n, eps_n, m->T, m->st));
  m->labelled = true;
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_set_targets(lbmps_mlp* m, const float* h) {
  if (!m) return LBMPS_EINVAL;
  if (m->n < 1) return mfail(m, LBMPS_ESTATE, "set samples first");
  if (!h) return mfail(m, LBMPS_EINVAL, "null targets");
  MHIPCHK(m, hipMemcpyAsync(m->T, h, (size_t)m->n * 4, hipMemcpyHostToDevice, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  m->labelled = true;
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_get_targets(lbmps_mlp* m, float* h) {
  if (!m) return LBMPS_EINVAL;
  if (!m->labelled) return mfail(m, LBMPS_ESTATE, "no targets");
  if (!h) return mfail(m, LBMPS_EINVAL, "null output");
  MHIPCHK(m, hipMemcpyAsync(h, m->T, (size_t)m->n * 4, hipMemcpyDeviceToHost, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_predict(lbmps_mlp* m, float* h) {
  if (!m) return LBMPS_EINVAL;
  if (m->n < 1) return mfail(m, LBMPS_ESTATE, "set samples first");
  if (!h) return mfail(m, LBMPS_EINVAL, "null output");
  MHIPCHK(m, launch_mlp_infer(m->P, m->X, m->n, m->y, m->st));
  MHIPCHK(m, hipMemcpyAsync(h, m->y, (size_t)m->n * 4, hipMemcpyDeviceToHost, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_gradient(lbmps_mlp* m, int64_t b0, int32_t batch, int64_t mult, int64_t add, float* h) {
  if (!m) return LBMPS_EINVAL;
  if (!m->labelled) return mfail(m, LBMPS_ESTATE, "set samples and targets first");
  if (!h) return mfail(m, LBMPS_EINVAL, "null output");
  if (batch < 1 || batch > MLP_MAX_BATCH || b0 < 0) return mfail(m, LBMPS_EINVAL, "batch out of range");
  lbmps_status s = check_order(m, mult, add);
  if (s) return s;
  const int ntiles = (batch + 31) / 32;
  MHIPCHK(m, launch_mlp_grad(m->P, m->X, m->T, m->n, b0 % m->n, mult, add, batch, m->partial, m->st));
  MHIPCHK(m, launch_mlp_reduce_adam(m->P, m->partial, ntiles, m->grad, m->m, m->v, 0, 0.f, 0.f, 0.f, 0.f, 0, m->st));
  MHIPCHK(m, hipMemcpyAsync(h, m->grad, (size_t)mlp_nparam() * 4, hipMemcpyDeviceToHost, m->st));
  MHIPCHK(m, hipStreamSynchronize(m->st));
  return LBMPS_OK;
}

lbmps_status lbmps_mlp_train(lbmps_mlp* m, const lbmps_mlp_train_cfg* cfg) {
  if (!m) return LBMPS_EINVAL;
  if (!cfg || !cfg->mult || !cfg->add) return mfail(m, LBMPS_EINVAL, "null configuration");
  if (!m->labelled) return mfail(m, LBMPS_ESTATE, "set samples and targets first");
  if (cfg->epochs < 0 || cfg->batch < 1 || cfg->batch > MLP_MAX_BATCH) return mfail(m, LBMPS_EINVAL, "bad epochs or batch");
  if (!(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) ||
      !(cfg->adam_eps > 0))
    return mfail(m, LBMPS_EINVAL, "bad optimiser constants");
  for (int e = 0; e < cfg->epochs; ++e) {
    lbmps_status s = check_order(m, cfg->mult[e], cfg->add[e]);
    if (s) return s;
  }
  for (int e = 0; e < cfg->epochs; ++e)
    for (long long b0 = 0; b0 < m->n; b0 += cfg->batch) {
      const int B = (int)std::min<long long>(cfg->batch, m->n - b0);
      m->step++;
      MHIPCHK(m, launch_mlp_grad(m->P, m->X, m->T, m->n, b0, cfg->mult[e], cfg->add[e], B, m->partial, m->st));
      MHIPCHK(m, launch_mlp_reduce_adam(m->P, m->partial, (B + 31) / 32, m->grad, m->m, m->v, 1, cfg->lr, cfg->beta1,
                                        cfg->beta2, cfg->adam_eps, m->step, m->st));
    }
  return LBMPS_OK;
}

const char* lbmps_mlp_last_error(const lbmps_mlp* m) { return m ? m->last.c_str() : "null trainer"; }

const char* lbmps_status_string(lbmps_status s) {
  switch (s) {
    case LBMPS_OK: return "ok";
    case LBMPS_EINVAL: return "invalid argument";
    case LBMPS_ENOMEM: return "workspace or capacity too small";
    case LBMPS_EDEVICE: return "HIP runtime error";
    case LBMPS_EUNSTABLE: return "numerical instability";
    case LBMPS_ESTATE: return "call out of order";
    case LBMPS_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* lbmps_last_error(const lbmps_ctx* c) { return c ? c->last.c_str() : "null context"; }

}  // extern "C"
