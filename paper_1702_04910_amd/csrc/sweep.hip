// Fused D3Q19 collide-and-push sweep (Sec. 2.1, Eqs. LBM_Collide, LBM_Stream,
// LBM_EQ, LBM_SRT, MEM_TRT, Forcing) and the field/PDF conversion kernels.
//
// One sweep reads the canonical PDFs f(x, t) of every cell from buffer `src`
// (aligned, coalesced along x), collides them with BGK or TRT plus the body
// force, and pushes f~_q(x, t) to x + c_q in buffer `dst` (periodic wrap).
// MEM coupling is applied afterwards by the link kernel, which overwrites the
// few affected values.  PSM cells are handled in one of three ways, with
// identical results: collided here (the sweep reads the cell map and applies
// the partially saturated collision to cells of a single particle inline;
// cells shared by several particles are re-collided afterwards), re-collided
// afterwards by the overlap kernel, or collided beforehand by the overlap
// kernel into a staging array indexed by the cell's leader pair, from which
// the sweep takes their post-collision values (so every store of the
// overlapped cells is part of the sweep's aligned row writes).  Each workgroup
// owns whole x-rows and realigns the +-x shifted values through LDS, so all
// stores are aligned row segments.
#include <climits>

#include "common.h"
#include "kernels.h"
#include "psm_cell.h"

namespace lbm {

// c.v for a lattice velocity with components (a, b, c) in {-1, 0, 1}, without
// multiplications or additions of zero terms.
template <typename R, int k>
__device__ __forceinline__ R term(R v) {
  return k == 1 ? v : -v;
}
template <typename R, int a, int b, int c>
__device__ __forceinline__ R dot3(R x, R y, R z) {
  if constexpr (a != 0 && b != 0) return term<R, a>(x) + term<R, b>(y);
  else if constexpr (a != 0 && c != 0) return term<R, a>(x) + term<R, c>(z);
  else if constexpr (b != 0 && c != 0) return term<R, b>(y) + term<R, c>(z);
  else if constexpr (a != 0) return term<R, a>(x);
  else if constexpr (b != 0) return term<R, b>(y);
  else if constexpr (c != 0) return term<R, c>(z);
  else return (R)0;
}

// Pair p = 0..8 holds the opposite directions (2p + 1, 2p + 2); PAIR_C[k][p]
// is component k of c_{2p+1}.  The moment sums below are written out from this
// table, which is checked against the velocity set at compile time.
constexpr int PAIR_C[3][9] = {{1, 0, 0, 1, 1, 1, 1, 0, 0}, {0, 1, 0, 1, -1, 0, 0, 1, 1}, {0, 0, 1, 0, 0, 1, -1, 1, -1}};
constexpr bool pair_table_ok() {
  for (int p = 0; p < 9; ++p)
    if (PAIR_C[0][p] != cx(2 * p + 1) || PAIR_C[1][p] != cy(2 * p + 1) || PAIR_C[2][p] != cz(2 * p + 1) ||
        opp(2 * p + 1) != 2 * p + 2)
      return false;
  return true;
}
static_assert(pair_table_ok(), "pair table does not match the velocity set");

// TRT collision of the pair (QA, QA + 1) in deviation variables: Eq. MEM_TRT
// with f^+- = (f_q +- f_qbar)/2, f^eq+ = w (base + 4.5 (c.u)^2), f^eq- = 3 w c.u,
// and the forcing of Eq. Forcing split into its symmetric part w (9 (c.u)(c.F)
// - 3 u.F) and antisymmetric part 3 w c.F.  With s = g_q + g_qbar and
// d = g_q - g_qbar the two changes are
//   c+ = lp (s/2 - f^eq+) + w (9 cu cf - 3 fu) = (lp/2) s + w (A + cu (9 cf - 4.5 lp cu)),
//   c- = lm (d/2 - f^eq-) + 3 w cf             = (lm/2) d + 3 w (cf - lm cu),
// with the per-cell A = -lp base - 3 fu; g_q gains c+ + c-, g_qbar c+ - c-.
// The quadratic term is formed as lp (-4.5 cu), not with a rounded constant
// -4.5 lp: that constant's fixed rounding error, multiplied by cu^2 >= 0 in
// every cell, would bias the mass by a few 1e-12 per cell and sweep in FP32.
// Contraction is off and the fused multiply-adds are explicit (fmac), so every
// sweep variant, whatever code surrounds this, produces the same bits.
template <typename R, int P>
__device__ __forceinline__ void trt_pair(const R (&g)[Q], const R (&s)[9], const R (&d)[9], R (&o)[Q], R A, R ux,
                                         R uy, R uz, R fx, R fy, R fz, R hp, R hm, R lp, R lm) {
#pragma clang fp contract(off)
  constexpr int QA = 2 * P + 1, QB = QA + 1;
  const R w = (R)wq(QA);
  const R cu = dot3<R, cx(QA), cy(QA), cz(QA)>(ux, uy, uz);
  const R cf = dot3<R, cx(QA), cy(QA), cz(QA)>(fx, fy, fz);
  const R cp = fmac<R>(w, fmac<R>(cu, fmac<R>((R)9, cf, lp * ((R)-4.5 * cu)), A), hp * s[P]);
  const R cm = fmac<R>((R)(3.0 * wq(QA)), fmac<R>(-lm, cu, cf), hm * d[P]);
  o[QA] = (g[QA] + cp) + cm;
  o[QB] = (g[QB] + cp) - cm;
}

// One cell's TRT collision with body force (lp, lm: the relaxation factors of
// the symmetric and antisymmetric parts, negative).  The moments are taken from
// the pair sums and differences that the collision needs anyway: drho = g_0 +
// sum s_p, j = sum_p c_{2p+1} d_p.
template <typename R>
__device__ __forceinline__ void collide_cell(const R (&g)[Q], R (&o)[Q], R lp, R lm, R fx, R fy, R fz) {
#pragma clang fp contract(off)
  R s[9], d[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    s[p] = g[2 * p + 1] + g[2 * p + 2];
    d[p] = g[2 * p + 1] - g[2 * p + 2];
  }
  const R drho = (((g[0] + s[0]) + (s[1] + s[2])) + ((s[3] + s[4]) + (s[5] + s[6]))) + (s[7] + s[8]);
  const R ux = ((d[0] + d[3]) + d[4]) + (d[5] + d[6]);
  const R uy = ((d[1] + d[3]) - d[4]) + (d[7] + d[8]);
  const R uz = ((d[2] + d[5]) - d[6]) + (d[7] - d[8]);
  const R uu = fmac<R>(uz, uz, fmac<R>(uy, uy, ux * ux));
  const R fu = fmac<R>(uz, fz, fmac<R>(uy, fy, ux * fx));
  const R base = fmac<R>((R)-1.5, uu, drho);
  const R A = fmac<R>(-lp, base, (R)-3 * fu);
  const R hp = (R)0.5 * lp, hm = (R)0.5 * lm;
  // rest direction: g_0 + lp (g_0 - w_0 base) - 3 w_0 fu = g_0 + lp g_0 + w_0 A
  o[0] = fmac<R>(lp, g[0], fmac<R>((R)wq(0), A, g[0]));
  trt_pair<R, 0>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 1>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 2>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 3>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 4>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 5>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 6>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 7>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
  trt_pair<R, 8>(g, s, d, o, A, ux, uy, uz, fx, fy, fz, hp, hm, lp, lm);
}

template <int q>
__device__ __forceinline__ int pick(int m, int c, int p) {
  return q < 0 ? m : (q > 0 ? p : c);
}

// Streaming stores that bypass the cache hierarchy's write-allocate path.
template <typename S>
__device__ __forceinline__ void st_nt(S* p, S v) {
  __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void st_nt<__bf16>(__bf16* p, __bf16 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short*)p);
}

// Directions with c_x != 0 and their slot in the LDS staging area.
__host__ __device__ constexpr int xslot(int q) {
  return q == 1 ? 0 : q == 2 ? 1 : q == 7 ? 2 : q == 8 ? 3 : q == 9 ? 4 : q == 10 ? 5 : q == 11 ? 6
       : q == 12 ? 7 : q == 13 ? 8 : q == 14 ? 9 : -1;
}
constexpr int NXSHIFT = 10;

// One tile = `tl.z` whole x-rows of one instance.  Phase 1: every cell is
// loaded (19 coalesced loads), collided, and its 9 post-collision values with
// c_x = 0 are pushed straight to the neighbouring rows (aligned).  The 10
// values with c_x = +-1 land in the same local row shifted by one cell, so they
// are staged in LDS at their shifted position.  Phase 2: the staged rows are
// written out aligned.  Every global store therefore covers whole, aligned row
// segments.
template <typename S>
__device__ __forceinline__ S ld_nt(const S* p) {
  return __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ __bf16 ld_nt<__bf16>(const __bf16* p) {
  return __builtin_bit_cast(__bf16, __builtin_nontemporal_load((const unsigned short*)p));
}

// Two x-adjacent values of storage type S moved as one word (the cell-pair
// variant of the sweep): W is the word, U the bit pattern of one value.
template <typename S> struct Twin;
template <> struct Twin<double> {
  typedef unsigned long long W __attribute__((ext_vector_type(2)));
  using U = unsigned long long;
};
template <> struct Twin<float> { using W = unsigned long long; using U = unsigned int; };
template <> struct Twin<_Float16> { using W = unsigned int; using U = unsigned short; };
template <> struct Twin<__bf16> { using W = unsigned int; using U = unsigned short; };

template <typename S>
__device__ __forceinline__ typename Twin<S>::W twin_pack(S a, S b) {
  using U = typename Twin<S>::U;
  using W = typename Twin<S>::W;
  const U ua = __builtin_bit_cast(U, a), ub = __builtin_bit_cast(U, b);
  if constexpr (sizeof(S) == 8) {
    W w;
    w.x = ua;
    w.y = ub;
    return w;
  } else {
    return (W)ua | ((W)ub << (8 * sizeof(S)));  // the lower address holds the low bits
  }
}
// The stored word of a cell pair from the two post-collision values and the
// cells' random bits (2-byte storage: each value converted into its half).
template <typename S, typename R>
__device__ __forceinline__ typename Twin<S>::W twin_word(R a, R b, uint32_t ra, uint32_t rb) {
  if constexpr (sizeof(S) == 2)
    return Half16<S>::put(Half16<S>::put(0u, a, ra, false), b, rb, true);
  else
    return twin_pack<S>(CellStore<S>::st(a, ra), CellStore<S>::st(b, rb));
}
template <typename S>
__device__ __forceinline__ void twin_unpack(typename Twin<S>::W w, S& a, S& b) {
  using U = typename Twin<S>::U;
  if constexpr (sizeof(S) == 8) {
    a = __builtin_bit_cast(S, (U)w.x);
    b = __builtin_bit_cast(S, (U)w.y);
  } else {
    a = __builtin_bit_cast(S, (U)w);
    b = __builtin_bit_cast(S, (U)(w >> (8 * sizeof(S))));
  }
}
template <typename S, bool NT>
__device__ __forceinline__ typename Twin<S>::W twin_ld(const S* p) {
  const typename Twin<S>::W* q = reinterpret_cast<const typename Twin<S>::W*>(p);
  if constexpr (NT)
    return __builtin_nontemporal_load(q);
  else
    return *q;
}
template <typename S>
__device__ __forceinline__ void twin_st_nt(S* p, typename Twin<S>::W w) {
  __builtin_nontemporal_store(w, reinterpret_cast<typename Twin<S>::W*>(p));
}

// The sweep with every thread handling the two adjacent cells (x, x + 1), x
// even (nx even, so a pair never straddles rows; every pair address is aligned
// to two values): one word per q and cell pair for loads, c_x = 0 pushes and
// the aligned row writes of the LDS-staged c_x = +-1 pushes.  More bytes in
// flight per wave.  No overlapped-cell handling (PSM collided after the sweep).
template <typename S, bool NTLD>
__device__ __forceinline__ void sweep_body_twin(const InstDev* __restrict__ insts, const int4* __restrict__ tiles,
                                                int ntiles, const S* __restrict__ src, S* __restrict__ dst) {
  using R = typename CompOf<S>::type;
  using W = typename Twin<S>::W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  S* sh = reinterpret_cast<S*>(smem_raw);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    const InstDev& I = insts[tl.x];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const S* __restrict__ s = src + I.pdf_off;
    S* __restrict__ d = dst + I.pdf_off;
    const R lp = (R)I.lam_p, lm = (R)I.lam_m;
    const R fx = (R)I.fext[0], fy = (R)I.fext[1], fz = (R)I.fext[2];
    const int ncells = tl.z * nx;
    for (int ip = threadIdx.x; 2 * ip < ncells; ip += blockDim.x) {
      const int i = 2 * ip;
      const int r = i / nx;
      const int x = i - r * nx;  // even; x + 1 < nx
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int idx = row * nx + x;
      R g0[Q], g1[Q], o0[Q], o1[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        S a, b;
        twin_unpack<S>(twin_ld<S, NTLD>(&s[pdf_at(idx, q)]), a, b);
        g0[q] = Codec<S>::ld(a);
        g1[q] = Codec<S>::ld(b);
      }
      collide_cell<R>(g0, o0, lp, lm, fx, fy, fz);
      collide_cell<R>(g1, o1, lp, lm, fx, fy, fz);
      CellBits<S> rb0(o0[0], idx), rb1(o1[0], idx + 1);
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
      const int xm = x == 0 ? nx - 1 : x - 1, xpp = x + 2 == nx ? 0 : x + 2;
      const int lrow = r * nx;
#define LBM_PUSH2(qq)                                                                       \
  {                                                                                         \
    const uint32_t r0 = rb0.next(), r1 = rb1.next();                                        \
    if constexpr (cx(qq) == 0) {                                                            \
      const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                 \
      twin_st_nt<S>(&d[pdf_at((za * ny + ya) * nx + x, qq)], twin_word<S>(o0[qq], o1[qq], r0, r1)); \
    } else {                                                                                \
      sh[xslot(qq) * ncells + lrow + (cx(qq) > 0 ? x + 1 : xm)] = CellStore<S>::st(o0[qq], r0); \
      sh[xslot(qq) * ncells + lrow + (cx(qq) > 0 ? xpp : x)] = CellStore<S>::st(o1[qq], r1);    \
    }                                                                                       \
  }
      LBM_PUSH2(0) LBM_PUSH2(1) LBM_PUSH2(2) LBM_PUSH2(3) LBM_PUSH2(4) LBM_PUSH2(5) LBM_PUSH2(6)
      LBM_PUSH2(7) LBM_PUSH2(8) LBM_PUSH2(9) LBM_PUSH2(10) LBM_PUSH2(11) LBM_PUSH2(12) LBM_PUSH2(13)
      LBM_PUSH2(14) LBM_PUSH2(15) LBM_PUSH2(16) LBM_PUSH2(17) LBM_PUSH2(18)
#undef LBM_PUSH2
    }
    __syncthreads();
    for (int ip = threadIdx.x; 2 * ip < ncells; ip += blockDim.x) {
      const int i = 2 * ip;
      const int r = i / nx;
      const int x = i - r * nx;
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
#define LBM_FLUSH2(qq)                                                                      \
  {                                                                                         \
    const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                   \
    twin_st_nt<S>(&d[pdf_at((za * ny + ya) * nx + x, qq)],                                  \
                  *reinterpret_cast<const W*>(&sh[xslot(qq) * ncells + i]));                \
  }
      LBM_FLUSH2(1) LBM_FLUSH2(2) LBM_FLUSH2(7) LBM_FLUSH2(8) LBM_FLUSH2(9) LBM_FLUSH2(10) LBM_FLUSH2(11)
      LBM_FLUSH2(12) LBM_FLUSH2(13) LBM_FLUSH2(14)
#undef LBM_FLUSH2
    }
    __syncthreads();
  }
}

// The sweep with every thread handling four x-adjacent cells x .. x + 3, x a
// multiple of 4 (nx a multiple of 4), for 2-byte storage: each load and store
// moves one 8-byte word of four values, and the address arithmetic is shared by
// four cells.  The c_x = +-1 values are staged in LDS as whole words at the
// position of the cell that produced them; the write-out assembles each
// destination word from the staged word at the same position and the last
// (c_x = +1) or first (c_x = -1) value of its neighbour word in the row
// (periodic).  No overlapped-cell handling (PSM collided after the sweep).
template <typename S, bool NTLD>
__device__ __forceinline__ void sweep_body_quad(const InstDev* __restrict__ insts, const int4* __restrict__ tiles,
                                                int ntiles, const S* __restrict__ src, S* __restrict__ dst) {
  static_assert(sizeof(S) == 2, "four cells per word: 2-byte storage only");
  using R = typename CompOf<S>::type;
  using W = unsigned long long;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  W* sh = reinterpret_cast<W*>(smem_raw);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    const InstDev& I = insts[tl.x];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const S* __restrict__ s = src + I.pdf_off;
    S* __restrict__ d = dst + I.pdf_off;
    const R lp = (R)I.lam_p, lm = (R)I.lam_m;
    const R fx = (R)I.fext[0], fy = (R)I.fext[1], fz = (R)I.fext[2];
    const int nxq = nx >> 2;
    const int nq = tl.z * nxq;  // words per staged direction in this tile
    for (int iq = threadIdx.x; iq < nq; iq += blockDim.x) {
      const int r = iq / nxq;
      const int x = (iq - r * nxq) << 2;
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int idx = row * nx + x;
      W win[Q], wout[Q];
      uint32_t wlo[Q], whi[Q];  // cells 0, 1 and cells 2, 3 of the word
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const W* a = reinterpret_cast<const W*>(&s[pdf_at(idx, q)]);
        win[q] = NTLD ? __builtin_nontemporal_load(a) : *a;
        wlo[q] = whi[q] = 0u;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        R g[Q], o[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) g[q] = Codec<S>::ld(__builtin_bit_cast(S, (unsigned short)(win[q] >> (16 * k))));
        collide_cell<R>(g, o, lp, lm, fx, fy, fz);
        CellBits<S> rb(o[0], idx + k);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          uint32_t& w = k < 2 ? wlo[q] : whi[q];
          w = Half16<S>::put(w, o[q], rb.next(), (k & 1) != 0);
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) wout[q] = (W)whi[q] << 32 | wlo[q];
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
#define LBM_PUSH4(qq)                                                                       \
  if constexpr (cx(qq) == 0) {                                                              \
    const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                   \
    __builtin_nontemporal_store(wout[qq], reinterpret_cast<W*>(&d[pdf_at((za * ny + ya) * nx + x, qq)])); \
  } else {                                                                                  \
    sh[xslot(qq) * nq + iq] = wout[qq];                                                     \
  }
      LBM_PUSH4(0) LBM_PUSH4(1) LBM_PUSH4(2) LBM_PUSH4(3) LBM_PUSH4(4) LBM_PUSH4(5) LBM_PUSH4(6)
      LBM_PUSH4(7) LBM_PUSH4(8) LBM_PUSH4(9) LBM_PUSH4(10) LBM_PUSH4(11) LBM_PUSH4(12) LBM_PUSH4(13)
      LBM_PUSH4(14) LBM_PUSH4(15) LBM_PUSH4(16) LBM_PUSH4(17) LBM_PUSH4(18)
#undef LBM_PUSH4
    }
    __syncthreads();
    for (int iq = threadIdx.x; iq < nq; iq += blockDim.x) {
      const int r = iq / nxq;
      const int xq = iq - r * nxq;
      const int x = xq << 2;
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
      // neighbour words in the same row, periodic in x
      const int iprev = xq == 0 ? iq + nxq - 1 : iq - 1;
      const int inext = xq == nxq - 1 ? iq - nxq + 1 : iq + 1;
#define LBM_FLUSH4(qq)                                                                      \
  {                                                                                         \
    const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                   \
    const W cur = sh[xslot(qq) * nq + iq];                                                  \
    const W v = cx(qq) > 0 ? (cur << 16) | (sh[xslot(qq) * nq + iprev] >> 48)               \
                           : (cur >> 16) | (sh[xslot(qq) * nq + inext] << 48);              \
    __builtin_nontemporal_store(v, reinterpret_cast<W*>(&d[pdf_at((za * ny + ya) * nx + x, qq)])); \
  }
      LBM_FLUSH4(1) LBM_FLUSH4(2) LBM_FLUSH4(7) LBM_FLUSH4(8) LBM_FLUSH4(9) LBM_FLUSH4(10) LBM_FLUSH4(11)
      LBM_FLUSH4(12) LBM_FLUSH4(13) LBM_FLUSH4(14)
#undef LBM_FLUSH4
    }
    __syncthreads();
  }
}

// PSM: 0 no overlapped cells, 1 collide single-pair cells inline, 2 take the
// staged post-collision values of overlapped cells (stage[stage_at(leader
// pair, q)]).
template <typename S, bool NTLD, int PSM>
__device__ __forceinline__ void sweep_body(const InstDev* __restrict__ insts, const int4* __restrict__ tiles,
                                           int ntiles, const S* __restrict__ src, S* __restrict__ dst,
                                           const int* __restrict__ cellmap, const PairDev& pairs, const PartDev& P,
                                           const S* __restrict__ stage, long long sstride) {
  using R = typename CompOf<S>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  S* sh = reinterpret_cast<S*>(smem_raw);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    const InstDev& I = insts[tl.x];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const long long N = I.ncell;
    const S* __restrict__ s = src + I.pdf_off;
    S* __restrict__ d = dst + I.pdf_off;
    const R lp = (R)I.lam_p, lm = (R)I.lam_m;
    const R fx = (R)I.fext[0], fy = (R)I.fext[1], fz = (R)I.fext[2];
    const int ncells = tl.z * nx;
    for (int i = threadIdx.x; i < ncells; i += blockDim.x) {
      const int r = i / nx;
      const int x = i - r * nx;
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int idx = row * nx + x;
      // staged mode: the cell map is read before the PDFs and every cell is
      // collided (the result replaced for overlapped cells), so that the PDF
      // loads stay ahead of the test of the map and the staged values are
      // requested while they are still in flight
      int Lst = INT_MAX;
      if constexpr (PSM == 2) Lst = I.cellmap_off >= 0 ? cellmap[I.cellmap_off + idx] : INT_MAX;
      R g[Q], o[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const S* a = &s[pdf_at(idx, q)];
        g[q] = Codec<S>::ld(NTLD ? ld_nt(a) : *a);
      }
      // keep the test of the map (and its wait) behind the PDF loads
      if constexpr (PSM == 2) __builtin_amdgcn_sched_barrier(0);
      if constexpr (PSM == 1) {
        // cells of a single pair are collided here, with the solid operator
        // fixed per branch; cells shared by several particles get the fluid
        // collision, which the overlap kernel overwrites after the sweep
        const int L = I.cellmap_off >= 0 ? cellmap[I.cellmap_off + idx] : INT_MAX;
        if (L != INT_MAX && pairs.next[L] < 0) {
          if (I.psm_m == 1) psm_cell_collide<1, true, R>(g, o, I, P, pairs, L, idx);
          else if (I.psm_m == 2) psm_cell_collide<2, true, R>(g, o, I, P, pairs, L, idx);
          else psm_cell_collide<3, true, R>(g, o, I, P, pairs, L, idx);
#pragma unroll
          for (int q = 0; q < Q; ++q) o[q] = StochasticRound<S>::apply(o[q], (uint32_t)idx * Q + q);
        } else {
          collide_cell<R>(g, o, lp, lm, fx, fy, fz);
        }
      } else if constexpr (PSM == 2) {
        R st[Q];
        if (Lst != INT_MAX) {
#pragma unroll
          for (int q = 0; q < Q; ++q) st[q] = Codec<S>::ld(stage[stage_at(Lst, q)]);
        }
        collide_cell<R>(g, o, lp, lm, fx, fy, fz);
        if (Lst != INT_MAX) {
#pragma unroll
          for (int q = 0; q < Q; ++q) o[q] = st[q];
        }
      } else {
        collide_cell<R>(g, o, lp, lm, fx, fy, fz);
      }
      CellBits<S> rb(o[0], idx);
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
      const int lrow = r * nx;
#define LBM_PUSH(qq)                                                                        \
  {                                                                                         \
    const S v = CellStore<S>::st(o[qq], rb.next());                                         \
    if constexpr (cx(qq) == 0) {                                                            \
      const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                 \
      st_nt(&d[pdf_at((za * ny + ya) * nx + x, qq)], v);                                    \
    } else {                                                                                \
      sh[xslot(qq) * ncells + lrow + pick<cx(qq)>(xm, x, xp)] = v;                          \
    }                                                                                       \
  }
      LBM_PUSH(0) LBM_PUSH(1) LBM_PUSH(2) LBM_PUSH(3) LBM_PUSH(4) LBM_PUSH(5) LBM_PUSH(6)
      LBM_PUSH(7) LBM_PUSH(8) LBM_PUSH(9) LBM_PUSH(10) LBM_PUSH(11) LBM_PUSH(12) LBM_PUSH(13)
      LBM_PUSH(14) LBM_PUSH(15) LBM_PUSH(16) LBM_PUSH(17) LBM_PUSH(18)
#undef LBM_PUSH
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ncells; i += blockDim.x) {
      const int r = i / nx;
      const int x = i - r * nx;
      const int row = tl.y + r;
      const int z = row / ny;
      const int y = row - z * ny;
      const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
#define LBM_FLUSH(qq)                                                                       \
  {                                                                                         \
    const int ya = pick<cy(qq)>(ym, y, yp), za = pick<cz(qq)>(zm, z, zp);                   \
    st_nt(&d[pdf_at((za * ny + ya) * nx + x, qq)], sh[xslot(qq) * ncells + i]);             \
  }
      LBM_FLUSH(1) LBM_FLUSH(2) LBM_FLUSH(7) LBM_FLUSH(8) LBM_FLUSH(9) LBM_FLUSH(10) LBM_FLUSH(11)
      LBM_FLUSH(12) LBM_FLUSH(13) LBM_FLUSH(14)
#undef LBM_FLUSH
    }
    __syncthreads();
  }
}

template <typename S, bool NTLD, int PSM>
__global__ __launch_bounds__(256) void sweep_kernel(const InstDev* __restrict__ insts, const int4* __restrict__ tiles,
                                                    int ntiles, const S* __restrict__ src, S* __restrict__ dst,
                                                    const int* __restrict__ cellmap, PairDev pairs, PartDev P,
                                                    const S* __restrict__ stage, long long sstride) {
  sweep_body<S, NTLD, PSM>(insts, tiles, ntiles, src, dst, cellmap, pairs, P, stage, sstride);
}

template <typename S, bool NTLD>
__global__ __launch_bounds__(256) void sweep_kernel_twin(const InstDev* __restrict__ insts,
                                                         const int4* __restrict__ tiles, int ntiles,
                                                         const S* __restrict__ src, S* __restrict__ dst) {
  sweep_body_twin<S, NTLD>(insts, tiles, ntiles, src, dst);
}

template <typename S, bool NTLD>
__global__ __launch_bounds__(256) void sweep_kernel_quad(const InstDev* __restrict__ insts,
                                                         const int4* __restrict__ tiles, int ntiles,
                                                         const S* __restrict__ src, S* __restrict__ dst) {
  sweep_body_quad<S, NTLD>(insts, tiles, ntiles, src, dst);
}

// The same sweep compiled for six waves per SIMD (at most 80 registers per
// lane instead of ~105): more loads in flight per CU.  Chosen by the launch
// tuner; without spills for 4- and 2-byte storage only.
template <typename S, bool NTLD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void sweep_kernel_occ6(
    const InstDev* __restrict__ insts, const int4* __restrict__ tiles, int ntiles, const S* __restrict__ src,
    S* __restrict__ dst) {
  sweep_body<S, NTLD, 0>(insts, tiles, ntiles, src, dst, nullptr, PairDev{}, PartDev{}, nullptr, 0);
}

// Uniform equilibrium initial state, Eq. LBM_EQ: g_q = w_q (rho - 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u).
template <typename S>
__global__ void init_eq_kernel(S* __restrict__ buf, long long N, double rho, double ux, double uy, double uz) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cu = cx(q) * ux + cy(q) * uy + cz(q) * uz;
    const double v = wq(q) * ((rho - 1.0) + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    buf[pdf_at(i, q)] = Codec<S>::st((typename CompOf<S>::type)v);
  }
}

// Plane q, cells [c0, c0 + n) of one instance <-> a dense FP64 array.
template <typename S>
__global__ void to_f64_kernel(const S* __restrict__ a, int q, long long c0, double* __restrict__ b, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)Codec<S>::ld(a[pdf_at(c0 + i, q)]);
}

template <typename S>
__global__ void from_f64_kernel(const double* __restrict__ a, S* __restrict__ b, int q, long long c0, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[pdf_at(c0 + i, q)] = Codec<S>::st((typename CompOf<S>::type)a[i]);
}

// Density and macroscopic velocity (Eq. MacVel) of cells [c0, c0 + n); solid
// cells of the owner field report rho = 1, u = 0.  Output: out[0..n) rho,
// out[n..4n) u_x, u_y, u_z.
template <typename S>
__global__ void fields_kernel(const S* __restrict__ buf, long long N, long long c0, long long n,
                              const int* __restrict__ owner, double fx, double fy, double fz,
                              double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long c = c0 + i;
  double rho = 1.0, ux = 0.0, uy = 0.0, uz = 0.0;
  const bool solid = owner != nullptr && !own_is_fluid(owner[c]);
  if (!solid) {
    double g[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = (double)Codec<S>::ld(buf[pdf_at(c, q)]);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += g[q];
    rho = 1.0 + s;
    double jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      jx += cx(q) * g[q];
      jy += cy(q) * g[q];
      jz += cz(q) * g[q];
    }
    ux = jx + 0.5 * fx;
    uy = jy + 0.5 * fy;
    uz = jz + 0.5 * fz;
  }
  out[i] = rho;
  out[n + i] = ux;
  out[2 * n + i] = uy;
  out[3 * n + i] = uz;
}

// Collide-and-push of listed cells only: the cells that a MEM remap uncovered
// (count, rcell, rpart as written by the link-list fill), when the sweep ran
// while their refill was still in progress.  Each listed cell is collided
// from its refilled values in `src` and its 19 values are pushed to `dst`
// exactly as the sweep pushes them (same collision, same rounding), replacing
// what the sweep pushed from its earlier values; no other cell's sweep result
// depends on a listed cell, and the remap writes no other PDFs.
template <typename S>
__global__ __launch_bounds__(256) void resweep_cells_kernel(const int* __restrict__ count, int cap,
                                                            const int* __restrict__ rcell,
                                                            const int* __restrict__ rpart,
                                                            const InstDev* __restrict__ insts, PartDev P,
                                                            const S* __restrict__ src, S* __restrict__ dst) {
  using R = typename CompOf<S>::type;
  const int n = min(*count, cap);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const int cell = rcell[r];
    const InstDev& I = insts[P.inst[rpart[r]]];
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const S* __restrict__ s = src + I.pdf_off;
    S* __restrict__ d = dst + I.pdf_off;
    R g[Q], o[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = Codec<S>::ld(s[pdf_at(cell, q)]);
    collide_cell<R>(g, o, (R)I.lam_p, (R)I.lam_m, (R)I.fext[0], (R)I.fext[1], (R)I.fext[2]);
    CellBits<S> rb(o[0], cell);
    const int x = cell % nx, yz = cell / nx, y = yz % ny, z = yz / ny;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int xa = wrapi(x + cx(q), nx), ya = wrapi(y + cy(q), ny), za = wrapi(z + cz(q), nz);
      d[pdf_at(((long long)za * ny + ya) * nx + xa, q)] = CellStore<S>::st(o[q], rb.next());
    }
  }
}

// ------------------------------------------------------------------------ launchers
template <typename S, bool NTLD>
hipError_t launch_sweep_n(const InstDev* insts, const int4* tiles, int ntiles, int grid, int block, size_t lds,
                          int psm_mode, const void* src, void* dst, const int* cellmap, PairDev pairs, PartDev parts,
                          const void* stage, long long sstride, bool occ6, bool twin, bool quad, hipStream_t st) {
  if constexpr (sizeof(S) < 8) {
    if (occ6 && psm_mode == 0) {  // single cells only: the pair variant would spill within 80 registers
      hipLaunchKernelGGL((sweep_kernel_occ6<S, NTLD>), dim3(grid), dim3(block), lds, st, insts, tiles, ntiles,
                         (const S*)src, (S*)dst);
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(S) == 2) {
    if (quad && psm_mode == 0) {
      hipLaunchKernelGGL((sweep_kernel_quad<S, NTLD>), dim3(grid), dim3(block), lds, st, insts, tiles, ntiles,
                         (const S*)src, (S*)dst);
      return hipGetLastError();
    }
  }
  if (twin && psm_mode == 0) {
    hipLaunchKernelGGL((sweep_kernel_twin<S, NTLD>), dim3(grid), dim3(block), lds, st, insts, tiles, ntiles,
                       (const S*)src, (S*)dst);
    return hipGetLastError();
  }
#define LBM_SWEEP(MODE)                                                                                          \
  hipLaunchKernelGGL((sweep_kernel<S, NTLD, MODE>), dim3(grid), dim3(block), lds, st, insts, tiles, ntiles,       \
                     (const S*)src, (S*)dst, cellmap, pairs, parts, (const S*)stage, sstride)
  if (psm_mode == 1) LBM_SWEEP(1);
  else if (psm_mode == 2) LBM_SWEEP(2);
  else LBM_SWEEP(0);
#undef LBM_SWEEP
  return hipGetLastError();
}
template <typename S>
hipError_t launch_sweep_t(const InstDev* insts, const int4* tiles, int ntiles, int grid, int block, int max_tile_cells,
                          int flags, int psm_mode, const void* src, void* dst, const int* cellmap, PairDev pairs,
                          PartDev parts, const void* stage, long long sstride, hipStream_t st) {
  const size_t lds = sweep_lds_bytes((size_t)NXSHIFT * max_tile_cells * sizeof(S), flags);
  const bool occ6 = (flags & SWEEP_OCC6) != 0, twin = (flags & SWEEP_CELL_PAIRS) != 0,
             quad = (flags & SWEEP_CELL_QUADS) != 0;
  if (flags & SWEEP_NT_LOADS)
    return launch_sweep_n<S, true>(insts, tiles, ntiles, grid, block, lds, psm_mode, src, dst, cellmap, pairs, parts,
                                   stage, sstride, occ6, twin, quad, st);
  return launch_sweep_n<S, false>(insts, tiles, ntiles, grid, block, lds, psm_mode, src, dst, cellmap, pairs, parts,
                                  stage, sstride, occ6, twin, quad, st);
}
hipError_t launch_sweep(int prec, const InstDev* insts, const int4* tiles, int ntiles, int grid, int block,
                        int max_tile_cells, int flags, int psm_mode, const void* src, void* dst, const int* cellmap,
                        PairDev pairs, PartDev parts, const void* stage, long long sstride, hipStream_t st) {
  switch (prec) {
    case PREC_FP64:
      return launch_sweep_t<double>(insts, tiles, ntiles, grid, block, max_tile_cells, flags, psm_mode, src, dst,
                                    cellmap, pairs, parts, stage, sstride, st);
    case PREC_FP32:
      return launch_sweep_t<float>(insts, tiles, ntiles, grid, block, max_tile_cells, flags, psm_mode, src, dst,
                                   cellmap, pairs, parts, stage, sstride, st);
    case PREC_FP16:
      return launch_sweep_t<_Float16>(insts, tiles, ntiles, grid, block, max_tile_cells, flags, psm_mode, src, dst,
                                      cellmap, pairs, parts, stage, sstride, st);
    case PREC_BF16:
      return launch_sweep_t<__bf16>(insts, tiles, ntiles, grid, block, max_tile_cells, flags, psm_mode, src, dst,
                                    cellmap, pairs, parts, stage, sstride, st);
  }
  return hipErrorInvalidValue;
}

#define LBM_DISPATCH(prec, CALL)                  \
  switch (prec) {                                 \
    case PREC_FP64: { using S = double; CALL; } break;   \
    case PREC_FP32: { using S = float; CALL; } break;    \
    case PREC_FP16: { using S = _Float16; CALL; } break; \
    case PREC_BF16: { using S = __bf16; CALL; } break;   \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_init_eq(int prec, void* buf, long long N, double rho, const double u[3], hipStream_t st) {
  const int b = 256;
  const unsigned g = (unsigned)((N + b - 1) / b);
  LBM_DISPATCH(prec, hipLaunchKernelGGL(init_eq_kernel<S>, dim3(g), dim3(b), 0, st, (S*)buf, N, rho, u[0], u[1], u[2]));
  return hipGetLastError();
}

hipError_t launch_to_f64(int prec, const void* a, int q, long long c0, double* b, long long n, hipStream_t st) {
  const int bl = 256;
  const unsigned g = (unsigned)((n + bl - 1) / bl);
  LBM_DISPATCH(prec, hipLaunchKernelGGL(to_f64_kernel<S>, dim3(g), dim3(bl), 0, st, (const S*)a, q, c0, b, n));
  return hipGetLastError();
}

hipError_t launch_from_f64(int prec, const double* a, void* b, int q, long long c0, long long n, hipStream_t st) {
  const int bl = 256;
  const unsigned g = (unsigned)((n + bl - 1) / bl);
  LBM_DISPATCH(prec, hipLaunchKernelGGL(from_f64_kernel<S>, dim3(g), dim3(bl), 0, st, a, (S*)b, q, c0, n));
  return hipGetLastError();
}

hipError_t launch_resweep_cells(int prec, const int* count, int cap, const int* rcell, const int* rpart,
                                const InstDev* insts, PartDev parts, const void* src, void* dst, hipStream_t st) {
  // the list is a few cells per rigid-body step and particle; a grid-stride
  // loop covers longer ones
  LBM_DISPATCH(prec, hipLaunchKernelGGL(resweep_cells_kernel<S>, dim3(16), dim3(256), 0, st, count, cap, rcell, rpart,
                                        insts, parts, (const S*)src, (S*)dst));
  return hipGetLastError();
}

hipError_t launch_fields(int prec, const void* buf, long long N, long long c0, long long n, const int* owner,
                         const double f[3], double* out, hipStream_t st) {
  const int bl = 256;
  const unsigned g = (unsigned)((n + bl - 1) / bl);
  LBM_DISPATCH(prec, hipLaunchKernelGGL(fields_kernel<S>, dim3(g), dim3(bl), 0, st, (const S*)buf, N, c0, n, owner,
                                        f[0], f[1], f[2], out));
  return hipGetLastError();
}

}  // namespace lbm
