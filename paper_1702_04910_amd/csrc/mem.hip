// Momentum exchange coupling (Sec. 2.2): binary particle mapping, boundary
// links with their wall distance delta_q, the bounce-back (Eq. MEM_BB) and
// central linear interpolation (Eq. MEM_CLI) link rules with the link force
// of Eq. MEM_Force, and the refill of uncovered cells (Eq. MEM_Reconstruction
// followed by the moment-space velocity constraint).
//
// The PDFs in the working buffer are canonical f(x, t+1) after the push sweep,
// except at the link slots f_qbar(x, t+1) of fluid cells next to solid cells,
// which the link kernel writes.  It reads, for a link (x, q) with x + c_q solid:
//   f~_q(x, t)        -- pushed by x into the solid cell x + c_q, slot q;
//   f~_q(x - c_q, t)  -- pushed by the fluid cell x - c_q into x, slot q;
//   f~_qbar(x, t)     -- pushed by x into x - c_q, slot qbar.
// None of these slots is written by another link, so links are independent.
#include "bbox.h"
#include "common.h"
#include "kernels.h"
#include "particle_sum.h"

namespace lbm {

// Squared distance ((x^2 + y^2) + z^2) with every product and sum rounded on
// its own: no fused multiply-add may form across them (__dmul_rn / __dadd_rn
// alone do not prevent that once inlined).
__device__ __forceinline__ double sq3m(double x, double y, double z) {
#pragma clang fp contract(off)
  return (x * x + y * y) + z * z;
}

// delta_q: the smallest root in (0, 1] of |d + delta c_q|^2 = R^2, as
// e / (-b + sqrt(b^2 - a e)) with a = c.c, b = d.c, e = |d|^2 - R^2, each
// operation rounded on its own as plain FP64 evaluates it (e cancels, so a
// fused rounding would move delta by a few units of R^2 / |b|).
__device__ __forceinline__ double link_delta(const double (&d)[3], double R, int q) {
#pragma clang fp contract(off)
  const double e = sq3m(d[0], d[1], d[2]) - R * R;
  const double a = (double)speed2(q);
  const double b = (d[0] * cx(q) + d[1] * cy(q)) + d[2] * cz(q);
  return e / (-b + sqrt(b * b - a * e));
}

__device__ __forceinline__ void mem_bbox_lo(const PartDev& P, int p, int (&lo)[3]) {
  const double R = 0.5 * P.D[p];
#pragma unroll
  for (int k = 0; k < 3; ++k) lo[k] = (int)floor(P.X[3 * p + k] - R - 2.0);
}

__device__ __forceinline__ void disp(const InstDev& I, const PartDev& P, int p, int i, int j, int k, double (&d)[3]) {
  d[0] = min_image(((double)i + 0.5) - P.X[3 * p + 0], (double)I.nx);
  d[1] = min_image(((double)j + 0.5) - P.X[3 * p + 1], (double)I.ny);
  d[2] = min_image(((double)k + 0.5) - P.X[3 * p + 2], (double)I.nz);
}

// Workgroup (x, j) handles the work units x, x + gridDim.x, ... (a unit is a
// row range of one slab) of the bounding box of particle list[j], restricted
// to the particle's own extent (rows [U.y0, min(U.y1, ext)) of slab U.z < ext,
// ext cells each), in contiguous per-thread chunks; MEM_BBOX_END closes the
// loop over units.
#define MEM_BBOX_BEGIN                                                                 \
  const int jl = blockIdx.y;                                                           \
  const int p = list[jl];                                                              \
  const InstDev& I = insts[P.inst[p]];                                                 \
  int lo[3];                                                                           \
  mem_bbox_lo(P, p, lo);                                                               \
  int* own = owner + I.owner_off;                                                      \
  (void)own;                                                                           \
  const int ext_ = bbox_extent(P, p, side);                                            \
  for (int ub = blockIdx.x; ub < side * nsplit; ub += gridDim.x) {                     \
    const Unit U_ = unit_of(ub, side, nsplit);                                         \
    const int ncs = unit_cells(U_, ext_);                                              \
    const int chunk = (ncs + 255) / 256;                                               \
    const int ca = min(ncs, (int)threadIdx.x * chunk), cb = min(ncs, ca + chunk);
#define MEM_BBOX_END }

// The unit's cells of this thread's chunk, each with its lattice cell and
// slot index.
#define MEM_FOR_CELLS BBOX_FOR_CELLS(c, ca, cb, U_.y0, ext_, dy_, dx_)
#define MEM_CELL_COORDS                                                              \
  const int ci = wrap_near(lo[0] + dx_, I.nx), cj = wrap_near(lo[1] + dy_, I.ny),  \
            ck = wrap_near(lo[2] + U_.z, I.nz);                                    \
  const int cell = (ck * I.ny + cj) * I.nx + ci;                           \
  const long long sidx = slot_index(jl, side, U_.z, dy_, dx_);             \
  (void)sidx;

__global__ __launch_bounds__(256) void mem_unmap_kernel(const int* __restrict__ list, int side, int nsplit,
                                                        const InstDev* __restrict__ insts, PartDev P,
                                                        int* __restrict__ owner) {
  MEM_BBOX_BEGIN
  MEM_FOR_CELLS {
    MEM_CELL_COORDS
    // solid cells of p become "was solid of p"; the marks of p's previous
    // remap (cells it uncovered then, all within this box) become plain fluid
    const int o = own[cell];
    if (o == p) own[cell] = WAS_BIT | p;
    else if (o == (WAS_BIT | p)) own[cell] = OWN_FLUID;
  }
  MEM_BBOX_END
}

__global__ __launch_bounds__(256) void mem_map_kernel(const int* __restrict__ list, int side, int nsplit,
                                                      const InstDev* __restrict__ insts, PartDev P,
                                                      int* __restrict__ owner) {
  MEM_BBOX_BEGIN
  const double R = 0.5 * P.D[p];
  const double R2 = __dmul_rn(R, R);
  MEM_FOR_CELLS {
    MEM_CELL_COORDS
    double d[3];
    disp(I, P, p, ci, cj, ck, d);
    if (sq3m(d[0], d[1], d[2]) <= R2 && own_is_fluid(own[cell])) own[cell] = p;
  }
  MEM_BBOX_END
}

hipError_t launch_mem_unmap(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                            int* owner, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(mem_unmap_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts, parts,
                     owner);
  return hipGetLastError();
}

hipError_t launch_mem_map(const int* list, int nlist, int side, int nsplit, const InstDev* insts, PartDev parts,
                          int* owner, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(mem_map_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts, parts,
                     owner);
  return hipGetLastError();
}

// Slot word of a bounding-box cell: bits 1..18 = the directions q whose
// neighbour x + c_q is a solid cell of p (one link each); bit 0 = the cell
// was uncovered by p; bit 19 + k for the opposite pair (2k + 1, 2k + 2) =
// the pair has one link and the neighbour on its other side, x - c_q, is a
// fluid cell (the CLI condition of that link).  Both members of a pair cannot
// be links with the other side fluid, so one bit per pair suffices.
constexpr int SLOT_LINKS = ((1 << Q) - 1) & ~1;
__device__ __forceinline__ int slot_cli_bit(int q) { return 1 << (Q + ((q - 1) >> 1)); }

// Per fluid cell the slot word (see above); link counts to totals and, with
// `uncovered`, uncovered-cell counts to totals2.
__global__ __launch_bounds__(256) void mem_count_kernel(bool uncovered, const int* __restrict__ list, int side,
                                                        int nsplit, const InstDev* __restrict__ insts, PartDev P,
                                                        int* __restrict__ owner, int* __restrict__ slots,
                                                        int* __restrict__ totals, int* __restrict__ totals2) {
  MEM_BBOX_BEGIN
  int local = 0, local2 = 0;
  MEM_FOR_CELLS {
    MEM_CELL_COORDS
    int v = 0;
    if (own_is_fluid(own[cell])) {
      int fl = 0;
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        const int ni = wrap_near(ci + cx(q), I.nx), nj = wrap_near(cj + cy(q), I.ny), nk = wrap_near(ck + cz(q), I.nz);
        const int o = own[(nk * I.ny + nj) * I.nx + ni];
        if (o == p) v |= 1 << q;
        if (own_is_fluid(o)) fl |= 1 << q;
      }
#pragma unroll
      for (int q = 1; q < Q; ++q)
        if ((v & (1 << q)) && (fl & (1 << opp(q)))) v |= slot_cli_bit(q);
    }
    local += __popc(v & SLOT_LINKS);
    if (uncovered && own[cell] == (WAS_BIT | p)) {
      v |= 1;
      ++local2;
    }
    slots[sidx] = v;
  }
  __shared__ int sh[256];
  int total;
  block_excl_scan256(local, sh, &total);
  if (threadIdx.x == 0) totals[jl * (side * nsplit) + ub] = total;
  if (uncovered) {
    block_excl_scan256(local2, sh, &total);
    if (threadIdx.x == 0) totals2[jl * (side * nsplit) + ub] = total;
  }
  MEM_BBOX_END
}

hipError_t launch_mem_count(bool uncovered, const int* list, int nlist, int side, int nsplit, const InstDev* insts,
                            PartDev parts, const int* owner, int* slots, int* totals, int* totals2, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(mem_count_kernel, grid, dim3(256), 0, st, uncovered, list, side, nsplit,
                     insts, parts, (int*)owner, slots, totals, totals2);
  return hipGetLastError();
}

// Writes the links of each fluid cell in increasing q (slot bits 1..18) and,
// with refill lists (rcell != nullptr), the uncovered cells (slot bit 0) at
// their own scanned offsets.  Links carry delta_q = the smallest root in
// (0, 1] of |d + delta c|^2 = R^2 computed as e/(-b + sqrt(b^2 - a e))
// (a = c.c, b = d.c, e = |d|^2 - R^2), and whether x - c_q is fluid (needed by
// CLI; taken from the slot word, so the fill reads no owner entries).
__global__ __launch_bounds__(256) void mem_fill_links_kernel(const int* __restrict__ list, int side, int nsplit,
                                                             const InstDev* __restrict__ insts, PartDev P,
                                                             int* __restrict__ owner, const int* __restrict__ slots,
                                                             const int* __restrict__ offsets, int base, int cap,
                                                             LinkDev L, const int* __restrict__ offsets2, int cap2,
                                                             int* __restrict__ rcell, int* __restrict__ rpart) {
  MEM_BBOX_BEGIN
  int local = 0, local2 = 0;
  MEM_FOR_CELLS {
    MEM_CELL_COORDS
    const int m = slots[sidx];
    local += __popc(m & SLOT_LINKS);
    local2 += m & 1;
  }
  __shared__ int sh[256];
  int total;
  int pos = base + offsets[jl * (side * nsplit) + ub] + block_excl_scan256(local, sh, &total);
  int pos2 = 0;
  if (rcell) pos2 = offsets2[jl * (side * nsplit) + ub] + block_excl_scan256(local2, sh, &total);
  const double R = 0.5 * P.D[p];
  MEM_FOR_CELLS {
    MEM_CELL_COORDS
    const int m = slots[sidx];
    if (rcell && (m & 1)) {
      if (pos2 < cap2) {
        rcell[pos2] = cell;
        rpart[pos2] = p;
      }
      ++pos2;
    }
    if ((m & SLOT_LINKS) == 0) continue;
    double d[3];
    disp(I, P, p, ci, cj, ck, d);
    for (int q = 1; q < Q; ++q) {
      if (!(m & (1 << q))) continue;
      if (pos < base + cap) {
        const double delta = link_delta(d, R, q);
        L.cell[pos] = cell;
        L.q[pos] = q;
        L.p[pos] = p;
        L.inst[pos] = P.inst[p];
        L.delta[pos] = delta;
        L.cli_ok[pos] = (m & slot_cli_bit(q)) ? 1 : 0;
      }
      ++pos;
    }
  }
  MEM_BBOX_END
}

hipError_t launch_mem_fill_links(const int* list, int nlist, int side, int nsplit, const InstDev* insts,
                                 PartDev parts, int* owner, const int* slots, const int* offsets, int base, int cap,
                                 LinkDev links, const int* offsets2, int cap2, int* rcell, int* rpart,
                                 hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const dim3 grid(unit_grid(side * nsplit, nlist), nlist);
  hipLaunchKernelGGL(mem_fill_links_kernel, grid, dim3(256), 0, st, list, side, nsplit, insts,
                     parts, owner, slots, offsets, base, cap, links, offsets2, cap2, rcell, rpart);
  return hipGetLastError();
}

// Refill of one uncovered cell x (Sec. 2.2.3), one wave per cell, lane q
// handling direction q:
//  * q_n maximises n.c_q/|c_q| with n along x - X_p (ties: largest (cx, cy, cz)
//    lexicographically);
//  * sources x + k c_qn, k = 1..3, must be fluid cells that were fluid before the
//    remap; quadratic 3 f1 - 3 f2 + f3, else linear 2 f1 - f2, else constant f1,
//    else f^eq(rho0 + drho_bar, v(x)) with drho_bar the mean density fluctuation
//    of the old-fluid neighbours (0 if there are none); the equilibrium
//    reconstruction (I.refill) takes that last rule for every uncovered cell;
//  * velocity constraint: f_q += c_q.(j* - j)/10 with j* = v(x) - f_ext/2.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename S>
__global__ __launch_bounds__(256) void mem_refill_kernel(const int* __restrict__ count, int cap,
                                                         const int* __restrict__ rcell, const int* __restrict__ rpart,
                                                         const InstDev* __restrict__ insts, PartDev P,
                                                         const int* __restrict__ owner, S* __restrict__ buf) {
  const int n = min(*count, cap);
  const int lane = threadIdx.x & 63;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += nw) {
    const int cell = rcell[r], p = rpart[r];
    const InstDev& I = insts[P.inst[p]];
    const int* own = owner + I.owner_off;
    S* b = buf + I.pdf_off;
    const long long N = I.ncell;
    const int x = cell % I.nx, yz = cell / I.nx, y = yz % I.ny, z = yz / I.ny;
    double d[3];
    disp(I, P, p, x, y, z, d);
    int qn = 1;
    double best = -1e300;
    int bx = -2, by = -2, bz = -2;
    for (int q = 1; q < Q; ++q) {
      const double dc = d[0] * cx(q) + d[1] * cy(q) + d[2] * cz(q);
      const double score = speed2(q) == 1 ? dc : dc * 0.7071067811865476;
      const bool better = score > best ||
                          (score == best && (cx(q) > bx || (cx(q) == bx && (cy(q) > by || (cy(q) == by && cz(q) > bz)))));
      if (better) {
        best = score;
        qn = q;
        bx = cx(q);
        by = cy(q);
        bz = cz(q);
      }
    }
    // source cells along c_qn that are old fluid (consecutive from k = 1)
    int src_cell[3];
    int ns = 0;
    for (int k = 1; k <= 3; ++k) {
      const int xi = wrapi(x + k * cx(qn), I.nx), yi = wrapi(y + k * cy(qn), I.ny), zi = wrapi(z + k * cz(qn), I.nz);
      src_cell[k - 1] = (zi * I.ny + yi) * I.nx + xi;
    }
    // all three owner entries and (below) source PDFs are read before any is
    // tested, so their loads are in flight together
    const int os[3] = {own[src_cell[0]], own[src_cell[1]], own[src_cell[2]]};
    for (int k = 0; k < 3 && !I.refill; ++k) {  // no extrapolation sources for the equilibrium reconstruction
      if (os[k] != OWN_FLUID) break;
      ++ns;
    }
    const double* Up = P.U + 3 * p;
    const double* Wp = P.Om + 3 * p;
    const double v[3] = {Up[0] + (Wp[1] * d[2] - Wp[2] * d[1]), Up[1] + (Wp[2] * d[0] - Wp[0] * d[2]),
                         Up[2] + (Wp[0] * d[1] - Wp[1] * d[0])};
    const int q = lane < Q ? lane : 0;
    double o = 0.0;
    double f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = (double)Codec<S>::ld(b[pdf_at(src_cell[k], q)]);
    if (ns > 0) {
      o = ns == 3 ? 3.0 * f[0] - 3.0 * f[1] + f[2] : (ns == 2 ? 2.0 * f[0] - f[1] : f[0]);
    } else {
      // lane q' < 18 inspects neighbour q' + 1; fluctuation sum over its 19 PDFs
      double s = 0.0, cntv = 0.0;
      if (lane < 18) {
        const int qq = lane + 1;
        const int xi = wrapi(x + cx(qq), I.nx), yi = wrapi(y + cy(qq), I.ny), zi = wrapi(z + cz(qq), I.nz);
        const int c2 = (zi * I.ny + yi) * I.nx + xi;
        if (own[c2] == OWN_FLUID) {
          for (int k = 0; k < Q; ++k) s += (double)Codec<S>::ld(b[pdf_at(c2, k)]);
          cntv = 1.0;
        }
      }
      // fixed-order sum over the 18 neighbours (lane order)
      __shared__ double red[4][64];
      const int w = (threadIdx.x >> 6);
      red[w][lane] = s;
      double nr = wave_sum(cntv);
      double rs = 0.0;
      for (int k = 0; k < 18; ++k) rs += red[w][k];
      const double drho = nr > 0.0 ? rs / nr : 0.0;
      const double uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      const double cu = cx(q) * v[0] + cy(q) * v[1] + cz(q) * v[2];
      o = wq(q) * ((drho - 1.5 * uu) + cu * (3.0 + 4.5 * cu));
    }
    const double om = lane < Q ? o : 0.0;
    const double jx = wave_sum(cx(q) * om), jy = wave_sum(cy(q) * om), jz = wave_sum(cz(q) * om);
    const double dj[3] = {(v[0] - 0.5 * I.fext[0]) - jx, (v[1] - 0.5 * I.fext[1]) - jy, (v[2] - 0.5 * I.fext[2]) - jz};
    if (lane < Q) {
      const double val = o + (cx(q) * dj[0] + cy(q) * dj[1] + cz(q) * dj[2]) / 10.0;
      b[pdf_at(cell, q)] = Codec<S>::st((typename CompOf<S>::type)val);
    }
  }
}

#define LBM_DISPATCH(prec, CALL)                          \
  switch (prec) {                                         \
    case PREC_FP64: { using S = double; CALL; } break;    \
    case PREC_FP32: { using S = float; CALL; } break;     \
    case PREC_FP16: { using S = _Float16; CALL; } break;  \
    case PREC_BF16: { using S = __bf16; CALL; } break;    \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t launch_mem_refill(int prec, const int* count, int cap, const int* rcell, const int* rpart,
                             const InstDev* insts, PartDev parts, const int* owner, void* buf, hipStream_t st) {
  LBM_DISPATCH(prec, hipLaunchKernelGGL(mem_refill_kernel<S>, dim3(64), dim3(256), 0, st, count, cap, rcell, rpart,
                                        insts, parts, owner, (S*)buf));
  return hipGetLastError();
}

// Link rule and link force of link i.  Walls (p <= -2) use BB with their wall
// velocity; particle links use BB or CLI (CLI falls back to BB where x - c_q
// is not fluid).  For a particle link ft gets the deviation part
// (c_q - v) g~_q + (c_q + v) g_qbar of Eq. MEM_Force and its torque about X_p.
// ROW: the link belongs to particle p_row of instance inst_row (a particle
// row of the link kernel, where both are the same for the whole workgroup,
// so their fields come through scalar loads); otherwise both are read from
// the link.
template <typename S, bool ROW>
__device__ __forceinline__ void link_rule(int i, const LinkDev& L, const double* __restrict__ wall_v,
                                          const InstDev* __restrict__ insts, const PartDev& P, S* __restrict__ buf,
                                          int p_row, int inst_row, double (&ft)[6]) {
  const int inst = ROW ? inst_row : L.inst[i];
  const int cell = L.cell[i], q = L.q[i], p = ROW ? p_row : L.p[i];
  const int cli_ok = L.cli_ok[i];  // read with the other link fields, used by particle links
  const double delta_l = L.delta[i];
  // body state (particle centre, velocity, angular velocity; wall velocity),
  // requested before the instance fields and PDFs so the loads overlap
  double Xb[3] = {0, 0, 0}, Ub[3], Wb[3] = {0, 0, 0};
  if (p >= 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Xb[k] = P.X[3 * p + k];
      Ub[k] = P.U[3 * p + k];
      Wb[k] = P.Om[3 * p + k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) Ub[k] = wall_v[WALL_REC * (-2 - p) + k];
  }
  const InstDev& I = insts[inst];
  const int qb = opp(q);
  const int x = cell % I.nx, yz = cell / I.nx, y = yz % I.ny, z = yz / I.ny;
  S* b = buf + I.pdf_off;
  const int c[3] = {cx(q), cy(q), cz(q)};
  const int xs = wrap_near(x + c[0], I.nx), ys = wrap_near(y + c[1], I.ny), zs = wrap_near(z + c[2], I.nz);
  // the three PDFs a link may need are requested together, before the CLI
  // test, so one memory latency covers them
  const int xm = wrap_near(x - c[0], I.nx), ym = wrap_near(y - c[1], I.ny), zm = wrap_near(z - c[2], I.nz);
  const double gtq = (double)Codec<S>::ld(b[pdf_at(((long long)zs * I.ny + ys) * I.nx + xs, q)]);
  const double gq_m = (double)Codec<S>::ld(b[pdf_at(cell, q)]);
  const double gqb = (double)Codec<S>::ld(b[pdf_at(((long long)zm * I.ny + ym) * I.nx + xm, qb)]);
  double v[3], arm[3] = {0, 0, 0};
  bool cli = false;
  double delta = 0.5;
  if (p >= 0) {
    cli = I.coupling == COUP_MEM_CLI && cli_ok;
    if (cli) delta = delta_l;
    const double d[3] = {min_image(((double)x + 0.5) - Xb[0], (double)I.nx),
                         min_image(((double)y + 0.5) - Xb[1], (double)I.ny),
                         min_image(((double)z + 0.5) - Xb[2], (double)I.nz)};
    for (int k = 0; k < 3; ++k) arm[k] = d[k] + delta * c[k];
    v[0] = Ub[0] + (Wb[1] * arm[2] - Wb[2] * arm[1]);
    v[1] = Ub[1] + (Wb[2] * arm[0] - Wb[0] * arm[2]);
    v[2] = Ub[2] + (Wb[0] * arm[1] - Wb[1] * arm[0]);
  } else {
    v[0] = Ub[0];
    v[1] = Ub[1];
    v[2] = Ub[2];
  }
  const double vc = v[0] * c[0] + v[1] * c[1] + v[2] * c[2];
  const double w = wq(q);
  double val;
  if (cli) {
    const double k0 = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
    const double alpha = 4.0 / (1.0 + 2.0 * delta);
    val = gtq + k0 * gq_m - k0 * gqb - 3.0 * alpha * w * vc;
  } else {
    val = gtq - 6.0 * w * vc;
  }
  const S sv = Codec<S>::st((typename CompOf<S>::type)val);
  b[pdf_at(cell, qb)] = sv;
  if (p >= 0) {
    const double vs = (double)Codec<S>::ld(sv);
    double F[3];
    for (int k = 0; k < 3; ++k) F[k] = (c[k] - v[k]) * gtq + (c[k] + v[k]) * vs;
    ft[0] = F[0];
    ft[1] = F[1];
    ft[2] = F[2];
    ft[3] = arm[1] * F[2] - arm[2] * F[1];
    ft[4] = arm[2] * F[0] - arm[0] * F[2];
    ft[5] = arm[0] * F[1] - arm[1] * F[0];
  }
}

// Outflow rule of a wall link i whose group is an outflow (Sec. 4.1, after
// Ginzburg): f_qbar(x, t+1) = -f~_q(x, t) + 2 f^eq,+_q(rho_out, u(x, t)), in
// deviations g_qbar = -g~_q + 2 w_q (rho_out - 1 + 9/2 (c_q.u)^2 - 3/2 u.u),
// with u(x, t) = U + f_ext/2 (Eq. MacVel) from the fluid cell's PDFs before its
// collision (src).  wp: the group's record (rho_out at WALL_RHO_OUT).
template <typename S>
__device__ __forceinline__ void outflow_rule(int i, const LinkDev& L, const double* __restrict__ wp,
                                             const InstDev* __restrict__ insts, const S* __restrict__ src,
                                             S* __restrict__ buf) {
  const InstDev& I = insts[L.inst[i]];
  const int cell = L.cell[i], q = L.q[i], qb = opp(q);
  const int x = cell % I.nx, yz = cell / I.nx, y = yz % I.ny, z = yz / I.ny;
  const int xs = wrap_near(x + cx(q), I.nx), ys = wrap_near(y + cy(q), I.ny), zs = wrap_near(z + cz(q), I.nz);
  S* b = buf + I.pdf_off;
  const S* a = src + I.pdf_off;
  const double gtq = (double)Codec<S>::ld(b[pdf_at(((long long)zs * I.ny + ys) * I.nx + xs, q)]);
  double U[3] = {0.0, 0.0, 0.0};
  for (int r = 1; r < Q; ++r) {
    const double g = (double)Codec<S>::ld(a[pdf_at(cell, r)]);
    U[0] += cx(r) * g;
    U[1] += cy(r) * g;
    U[2] += cz(r) * g;
  }
  for (int k = 0; k < 3; ++k) U[k] += 0.5 * I.fext[k];
  const double cu = U[0] * cx(q) + U[1] * cy(q) + U[2] * cz(q);
  const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  const double val = -gtq + 2.0 * wq(q) * ((wp[WALL_RHO_OUT] - 1.0) + 4.5 * cu * cu - 1.5 * uu);
  b[pdf_at(cell, qb)] = Codec<S>::st((typename CompOf<S>::type)val);
}

// Row j < nlist of the grid: the links [n_wall + lbeg[j], n_wall + lend[j]) of
// particle list[j], one link per thread in chunks of SUM_THREADS; workgroup
// k < width takes chunks k, k + width, ... (the rest of the row is idle).
// Each thread keeps the sum of its links' force and torque; the workgroup
// stores their block_sum6 (in the sweep's set of `partial`), and after the
// last sweep of the rigid-body step finish_sums_kernel adds a particle's
// workgroup sums in a fixed order, so the total repeats bit for bit.
// Row nlist: the wall links [0, n_wall), strided over the whole row (velocity
// walls by link_rule, outflow groups by outflow_rule).
template <typename S>
__global__ __launch_bounds__(SUM_THREADS) void links_bc_kernel(int n_wall, const int* __restrict__ list, int nlist,
                                                               const int* __restrict__ lbeg,
                                                               const int* __restrict__ lend, LinkDev L,
                                                               const double* __restrict__ wall_v,
                                                               const InstDev* __restrict__ insts, PartDev P,
                                                               const S* __restrict__ src, S* __restrict__ buf,
                                                               double* __restrict__ partial, int width) {
  const int j = blockIdx.y, kb = blockIdx.x;
  double ft[6];
  if (j == nlist) {
    for (int i = kb * SUM_THREADS + (int)threadIdx.x; i < n_wall; i += gridDim.x * SUM_THREADS) {
      const double* wp = wall_v + WALL_REC * (-2 - L.p[i]);
      if (wp[WALL_KIND] != 0.0)
        outflow_rule<S>(i, L, wp, insts, src, buf);
      else
        link_rule<S, false>(i, L, wall_v, insts, P, buf, 0, 0, ft);
    }
    return;
  }
  const int nb = width;  // workgroups per particle: the rows of `partial` are this wide
  const int b = n_wall + lbeg[j], e = n_wall + lend[j];
  const int p_row = list[j], inst_row = P.inst[p_row];
  const int nch = (e - b + SUM_THREADS - 1) / SUM_THREADS;
  if (kb >= nch || kb >= nb) return;  // no links for this workgroup; it takes no part
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int ch = kb; ch < nch; ch += nb) {
    const int i = b + ch * SUM_THREADS + (int)threadIdx.x;
    if (i < e) {
      link_rule<S, true>(i, L, wall_v, insts, P, buf, p_row, inst_row, ft);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] += ft[k];
    }
  }
  double s[6];
  block_sum6(acc, s);
  store_chunk_sum(j, kb, nb, s, partial);
}

hipError_t launch_links_bc(int prec, int n_wall, const int* list, int nlist, const int* lbeg, const int* lend,
                           int width, LinkDev links, const double* wall_v, const InstDev* insts, PartDev parts,
                           const void* src, void* buf, double* partial, int set, hipStream_t st) {
  if (nlist <= 0 && n_wall <= 0) return hipSuccess;
  if (set < 0) return hipErrorInvalidValue;
  const long long set_stride = (long long)nlist * width * 6;
  // wall links get at least enough workgroups for one link per thread, up to 512
  const int blocks = std::max(width, std::min(512, (n_wall + SUM_THREADS - 1) / SUM_THREADS));
  LBM_DISPATCH(prec, hipLaunchKernelGGL(links_bc_kernel<S>, dim3(blocks, nlist + (n_wall > 0 ? 1 : 0)),
                                        dim3(SUM_THREADS), 0, st, n_wall, list, nlist, lbeg, lend, links, wall_v,
                                        insts, parts, (const S*)src, (S*)buf, partial + set * set_stride, width));
  return hipGetLastError();
}

}  // namespace lbm
