// Shared device definitions of the lbmps HIP library (gfx950).
//
// Lattice: D3Q19 (Sec. 2.1), lattice units dx = dt = rho0 = 1, c_s^2 = 1/3.
// Velocity order used by this library (and by every host array it exchanges):
//   q = 0 rest; q = 1..18 in opposite pairs (q odd, q + 1):
//   (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
//   (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
//   (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
// Weights 1/3, 1/18 (axis), 1/36 (diagonal).
//
// PDFs are stored as deviations g_q = f_q - w_q in blocks of PDF_BLOCK = 256
// consecutive cells (linear cell index (z*ny + y)*nx + x): block b holds its 19
// planes one after the other, so (q, cell) lives at
//   ((cell / 256) * 19 + q) * 256 + cell % 256.
// Inside a block this is a structure of arrays; the blocks keep the 19 streams
// of a workgroup within one contiguous region of memory.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int PDF_BLOCK = 256;
__host__ __device__ inline long long pdf_at(long long cell, int q) {
  return ((cell >> 8) * Q + q) * PDF_BLOCK + (cell & (PDF_BLOCK - 1));
}
// elements of one instance's PDF array (cells padded to whole blocks)
__host__ __device__ inline long long pdf_elems(long long ncell) {
  return (ncell + PDF_BLOCK - 1) / PDF_BLOCK * PDF_BLOCK * Q;
}

__host__ __device__ constexpr int cx(int q) {
  return (q == 1 || q == 7 || q == 9 || q == 11 || q == 13) ? 1
       : (q == 2 || q == 8 || q == 10 || q == 12 || q == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int q) {
  return (q == 3 || q == 7 || q == 10 || q == 15 || q == 17) ? 1
       : (q == 4 || q == 8 || q == 9 || q == 16 || q == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int q) {
  return (q == 5 || q == 11 || q == 14 || q == 15 || q == 18) ? 1
       : (q == 6 || q == 12 || q == 13 || q == 16 || q == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
__host__ __device__ constexpr int speed2(int q) { return cx(q) * cx(q) + cy(q) * cy(q) + cz(q) * cz(q); }
__host__ __device__ constexpr double wq(int q) {
  return q == 0 ? 1.0 / 3.0 : (speed2(q) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Coupling / collision / precision codes, identical to the public header.
enum { COUP_NONE = 0, COUP_MEM_BB = 1, COUP_MEM_CLI = 2, COUP_PSM = 3 };
enum { COLL_BGK = 0, COLL_TRT = 1 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16 = 2, PREC_BF16 = 3 };
enum { EPS_FLAT = 0, EPS_RECURSIVE = 1, EPS_LEARNED = 2, EPS_EDGE = 3, EPS_DISTANCE = 4 };

// Owner field values (MEM): -1 fluid, <= -2 static wall group (-2 - k),
// 0 <= p < WAS_BIT solid cell of particle p, WAS_BIT | p: uncovered by p's last
// remap, fluid now (the mark tells the refill which cells are new; p's next
// unmap clears it).
constexpr int OWN_FLUID = -1;
constexpr int WAS_BIT = 1 << 30;
__host__ __device__ inline bool own_is_fluid(int o) { return o == OWN_FLUID || (o >= WAS_BIT); }

// Error flags (bit mask in the device status word).
enum { ERR_LINK_CAP = 1, ERR_PAIR_CAP = 2, ERR_REFILL_CAP = 4, ERR_UNSTABLE = 8, ERR_CONTACT = 16, ERR_CUT_CAP = 32 };

// Per-instance parameters, read by every kernel.
struct InstDev {
  int nx, ny, nz, coupling;
  int collision, psm_m, psm_b, n_sub;
  long long ncell;
  long long pdf_off;      // element offset of this instance's 19*ncell block in each PDF buffer
  long long owner_off;    // int offset of the owner field (-1: none)
  long long cellmap_off;  // int offset of the PSM cell map (-1: none)
  double tau, lam_p, lam_m, mag;
  double fext[3];
  double grav[3];
  int part_begin, part_count, eps_n, eps_mode;
  int refill, pad_;  // MEM reconstruction: 0 extrapolation (Sec. 2.2.3), 1 equilibrium for every uncovered cell
};

// Particle state, structure of arrays of doubles, global over all instances.
struct PartDev {
  double *X, *U, *Om, *D, *rho;   // X,U,Om: 3 per particle
  int *fixed, *inst;
  double *F, *T;                   // subcycle-averaged force/torque of the last rigid-body step
  double *Facc, *Tacc;             // running sums over the current subcycles
  double *Xold;                    // position before the last rigid-body step
};

// Boundary links (x fluid, x + c_q solid), structure of arrays.
struct LinkDev {
  int *cell, *q, *p, *inst, *cli_ok;  // p >= 0 particle, p <= -2 wall group
  double *delta;
};

// PSM (cell, particle) overlap pairs.
struct PairDev {
  int *cell, *p, *next;
  double *eps, *B;
  double *out;  // 6 components per pair, component k at out[k * ostride + pair]
  long long ostride;
};

// Inputs of the solid-fraction network for a cell whose centre lies at d from
// the centre of a sphere of radius R: the signed distance |d| - R of the cell
// centre from the surface, the direction cosines |d_k| / |d| sorted
// descending (the cube symmetry of a cell folds every surface orientation
// into one 48th of the sphere), 8 / R (curvature relative to the cell size),
// then zeros.
__device__ __forceinline__ void eps_features(const double (&d)[3], double R, float (&x)[8]) {
#pragma clang fp contract(off)
  double a = fabs(d[0]), b = fabs(d[1]), c = fabs(d[2]), t;
  if (a < b) { t = a; a = b; b = t; }
  if (b < c) { t = b; b = c; c = t; }
  if (a < b) { t = a; a = b; b = t; }
  const double r = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)), __dmul_rn(c, c)));
  const double inv = r > 0.0 ? 1.0 / r : 0.0;
  x[0] = (float)(r - R);
  x[1] = (float)(a * inv);
  x[2] = (float)(b * inv);
  x[3] = (float)(c * inv);
  x[4] = (float)(8.0 / R);
  x[5] = x[6] = x[7] = 0.f;
}

// Cells cut by a sphere surface, collected while classifying bounding boxes.
struct CutDev {
  int* count;       // number of entries (may exceed the capacity: then truncated)
  long long* slot;  // slot index of the cell
  int *p, *use;     // particle; 1 when the learned estimator evaluates it
  double* d;        // 3 per entry: centre displacement from the sphere centre
  unsigned* err;    // error word (ERR_CUT_CAP on overflow)
};

// -------------------------------------------------------------------------- storage codecs
template <typename S> struct Codec;
template <> struct Codec<double> {
  __device__ static inline double ld(double v) { return v; }
  __device__ static inline double st(double v) { return v; }
};
template <> struct Codec<float> {
  __device__ static inline float ld(float v) { return v; }
  __device__ static inline float st(float v) { return v; }
};
template <> struct Codec<_Float16> {
  __device__ static inline float ld(_Float16 v) { return (float)v; }
  // Round to nearest even from the FP32 value as computed.  The library is
  // built without gfx950's mixed-precision FMAs: one with an FP16 result would
  // fuse this conversion into the FMA that produced v (one rounding instead of
  // two), and whether the compiler forms it depends on the surrounding kernel,
  // so the stored bits would differ between kernels.
  __device__ static inline _Float16 st(float v) { return (_Float16)v; }
};
template <> struct Codec<__bf16> {
  __device__ static inline float ld(__bf16 v) { return (float)v; }
  __device__ static inline __bf16 st(float v) { return (__bf16)v; }  // round to nearest even
};

// Stochastic rounding for the 16-bit storage types: x is stored as the
// representable neighbour below or above it in magnitude, the upper one with
// probability (|x| - lo) / (hi - lo), so that the stored value equals x in
// expectation.  The uniform draw is a hash of x's bits and a key (the cell and
// direction written), by the 32-bit finaliser of MurmurHash3 (Appleby): the
// rounding is a deterministic function of what is stored where.  Used for the
// post-collision values of PSM-overlapped cells, whose solid operator makes
// many cells hold nearly equal values: there round-to-nearest errs the same way
// in every cell, and the PSM force and torque (sums over those cells) collect
// the error coherently.
__device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
__device__ inline uint32_t sr_bits(float x, uint32_t key) { return fmix32(__float_as_uint(x) ^ fmix32(key)); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <typename S> struct StochasticRound {  // 4- and 8-byte storage: the value is stored as computed
  template <typename R> __device__ static inline R apply(R x, uint32_t) { return x; }
};
template <> struct StochasticRound<__bf16> {
  // bfloat16 is the upper half of the FP32 pattern: adding 16 random bits to
  // the magnitude and truncating rounds up with probability (low half) / 2^16;
  // gfx950's v_cvt_sr_bf16_f32 does that with the upper 16 bits of its random
  // word (the result is put in the upper half of a zero word: the FP32 value
  // of the stored BF16)
  __device__ static inline float apply(float x, uint32_t key) {
    const bf16x2 v = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2{}, x, sr_bits(x, key) << 16, true);
    return __uint_as_float(__builtin_bit_cast(uint32_t, v));
  }
};
template <> struct StochasticRound<_Float16> {
  __device__ static inline float apply(float x, uint32_t key) {
    const float a = fabsf(x);
    const _Float16 n = (_Float16)a;  // nearest
    const unsigned short nb = __builtin_bit_cast(unsigned short, n);
    // the two half-precision magnitudes around a (bit patterns of positive
    // halves are ordered like their values)
    unsigned short lo, hi;
    if ((float)n <= a) {
      lo = nb;
      hi = (unsigned short)(nb + 1);
    } else {
      hi = nb;
      lo = (unsigned short)(nb - 1);
    }
    const float flo = (float)__builtin_bit_cast(_Float16, lo), fhi = (float)__builtin_bit_cast(_Float16, hi);
    if (flo == a) return x;  // representable
    const float frac = (a - flo) / (fhi - flo);                        // in (0, 1)
    const float u = (float)(sr_bits(x, key) >> 8) * (1.0f / 16777216.0f);  // uniform in [0, 1)
    return copysignf(u < frac ? fhi : flo, x);
  }
};

// Staging array of the overlapped cells' post-collision values: the 19
// values of the cell led by pair L side by side, so that the cells of one
// sphere row (consecutive pairs) occupy one contiguous span.
__device__ inline long long stage_at(int L, int q) { return (long long)L * Q + q; }

// Stochastic rounding of all 19 post-collision values of a cell when they
// are stored as bfloat16 (other storage types: stored as computed).  BF16
// keeps 8 bits: round-to-nearest of the nearly uniform deviations of a slow
// flow errs the same way in many cells and steps, and that bias, not the
// size of the rounding, drove the BF16 runs' drift.  The random bits: one
// hash of the cell index and of the bits of the cell's post-collision rest
// value (so they change from step to step), spread over the directions by a
// Weyl sequence (additions only), one 32-bit word per value in the order
// q = 0..18.  The rounding itself is gfx950's conversion with stochastic
// rounding (v_cvt_sr_bf16_f32), one instruction per value: it adds the upper
// 16 bits of the random word to the FP32 pattern (the magnitude: sign and
// magnitude are separate) and keeps the upper half, so the value rounds away
// from zero with probability (lower half) / 2^16 and a value already
// representable in BF16 is stored as it is.
template <typename S> struct CellBits {  // no random bits for the other storage types
  __device__ CellBits(float, long long) {}
  __device__ uint32_t next() { return 0u; }
};
template <> struct CellBits<__bf16> {
  uint32_t x, step;
  __device__ CellBits(float o0, long long cell) : x(fmix32((uint32_t)cell * 0x9E3779B9u ^ __float_as_uint(o0))) {
    step = 2u * x + 0x632BE5ABu;
  }
  __device__ uint32_t next() {
    const uint32_t r = x;
    x += step;
    return r;
  }
};
// v rounded stochastically with the random bits r into the low (hi false) or
// high half of the word w; the other half is kept
__device__ inline uint32_t bf16_sr_put(uint32_t w, float v, uint32_t r, bool hi) {
  const bf16x2 o = __builtin_bit_cast(bf16x2, w);
  return __builtin_bit_cast(uint32_t, hi ? __builtin_amdgcn_cvt_sr_bf16_f32(o, v, r, true)
                                         : __builtin_amdgcn_cvt_sr_bf16_f32(o, v, r, false));
}

// One post-collision value converted for storage with the cell's random bits
// r: BF16 rounded stochastically, the other types as Codec<S>::st.
template <typename S> struct CellStore {
  template <typename R> __device__ static inline S st(R v, uint32_t) { return Codec<S>::st(v); }
};
template <> struct CellStore<__bf16> {
  __device__ static inline __bf16 st(float v, uint32_t r) {
    return __builtin_bit_cast(__bf16, (unsigned short)bf16_sr_put(0u, v, r, false));
  }
};

// A 2-byte stored value put into the low or high half of a 32-bit word whose
// other half is kept: FP16 rounded to nearest even, BF16 stochastically with
// the cell's random bits r (the same result as CellStore).
template <typename S> struct Half16;
template <> struct Half16<_Float16> {
  __device__ static inline uint32_t put(uint32_t w, float v, uint32_t, bool hi) {
    const uint32_t b = __builtin_bit_cast(unsigned short, Codec<_Float16>::st(v));
    return w | (hi ? b << 16 : b);
  }
};
template <> struct Half16<__bf16> {
  __device__ static inline uint32_t put(uint32_t w, float v, uint32_t r, bool hi) { return bf16_sr_put(w, v, r, hi); }
};

// compute precision paired with each storage type
template <typename S> struct CompOf { using type = float; };
template <> struct CompOf<double> { using type = double; };

// -------------------------------------------------------------------------- geometry helpers
// Minimum-image displacement of coordinate a from b on a periodic axis of length L.
__device__ inline double min_image(double d, double L) {
  if (d >= 0.5 * L) d -= L;
  if (d < -0.5 * L) d += L;
  return d;
}
__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Work units over the bounding boxes of listed particles: box side `side`,
// slab z split into `nsplit` row ranges.  Unit u of a box covers slab
// z = u / nsplit, rows [y0, y1).  Record lists are compacted unit by unit,
// so their order is fixed by the geometry alone.
struct Unit {
  int z, y0, y1;
};
__device__ inline Unit unit_of(int u, int side, int nsplit) {
  Unit r;
  r.z = u / nsplit;
  const int s = u - r.z * nsplit;
  r.y0 = s * side / nsplit;
  r.y1 = (s + 1) * side / nsplit;
  return r;
}
// Index of bbox cell (z, y, x) of list entry j in the per-cell slot array.
__device__ inline long long slot_index(int j, int side, int z, int y, int x) {
  return (((long long)j * side + z) * side + y) * side + x;
}

// Block-wide exclusive scan of one int per thread (blockDim.x == 256): an
// inclusive scan within each wave by shuffles, then the four wave totals
// through LDS (sh: at least 4 ints).  *total gets the block's sum.
__device__ inline int block_excl_scan256(int v, int* sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int s = sh[k];
    before += k < w ? s : 0;
    all += s;
  }
  *total = all;
  __syncthreads();  // sh may be reused by the caller
  return before + x - v;
}

}  // namespace lbm
