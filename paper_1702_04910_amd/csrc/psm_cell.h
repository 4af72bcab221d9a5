// Collision of one partially saturated cell (Sec. 2.3.1, Eqs. PSM, PSM_B1/B2,
// PSM_M1..M3, LBM_Collide_PSM) with the force and torque terms of every
// particle overlapping it (Eqs. PSM_TotForce/TotTorque).  Shared by the
// overlap kernel and the sweep that handles overlapped cells inline, so both
// produce identical bits.
#pragma once

#include "common.h"

namespace lbm {

constexpr int KMAX = 8;  // particles sharing one cell

// Members of the cell led by pair L, in increasing pair order.
__device__ __forceinline__ int gather_members(const PairDev& pairs, int L, int (&mem)[KMAX]) {
  int k = 0;
  mem[k++] = L;
  int nx = pairs.next[L];
  while (nx >= 0 && k < KMAX) {
    mem[k++] = nx;
    nx = pairs.next[nx];
  }
  for (int a = 1; a < k; ++a) {
    const int v = mem[a];
    int b = a - 1;
    while (b >= 0 && mem[b] > v) {
      mem[b + 1] = mem[b];
      --b;
    }
    mem[b + 1] = v;
  }
  return k;
}

// Every expression below is evaluated exactly as written: contraction into
// fused multiply-adds is switched off in each function and the fused
// operations that are wanted are spelled out (fmac).  The overlap kernel is
// compiled in several specialisations and inside the sweep; this keeps their
// results identical bit for bit, whatever code surrounds them.
template <typename R>
__device__ __forceinline__ R fmac(R a, R b, R c) {
  if constexpr (sizeof(R) == 8)
    return __builtin_fma(a, b, c);
  else
    return __builtin_fmaf(a, b, c);
}

// c_q . (x, y, z) for lattice components in {-1, 0, 1}: signed sum of the
// non-zero terms in x, y, z order (no multiplications).
template <typename R>
__device__ __forceinline__ R dotc(int q, R x, R y, R z) {
#pragma clang fp contract(off)
  R r = 0;
  bool first = true;
  const int c[3] = {cx(q), cy(q), cz(q)};
  const R v[3] = {x, y, z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (c[k] == 0) continue;
    const R t = c[k] > 0 ? v[k] : -v[k];
    r = first ? t : r + t;
    first = false;
  }
  return r;
}

// drho - 1.5 |u|^2
template <typename R>
__device__ __forceinline__ R eq_base(R drho, R ux, R uy, R uz) {
  return fmac<R>((R)-1.5, fmac<R>(uz, uz, fmac<R>(uy, uy, ux * ux)), drho);
}

// Equilibrium deviation of one direction, Eq. LBM_EQ minus w_q: w_q (base +
// cu (3 + 4.5 cu)) with base = drho - 1.5 |u|^2 and cu = c_q . u.  The value
// for the opposite direction is the same expression at -cu.
template <typename R>
__device__ __forceinline__ R geq1(R w, R base, R cu) {
#pragma clang fp contract(off)
  return w * fmac<R>(cu, fmac<R>((R)4.5, cu, (R)3), base);
}

// Solid operator Omega_q of one particle (Eqs. PSM_M1..M3) for every q, added
// to acc with weight B; returns sum_q Omega_q c_q in m.  Equilibria are formed
// per direction as needed (no 19-entry tables: fewer live registers).
template <int M, typename R>
__device__ __forceinline__ void add_solid_operator(const R (&g)[Q], R (&acc)[Q], R B, R baseU, R ux, R uy, R uz,
                                                   R baseV, R vx, R vy, R vz, R one_m_inv_tau, R (&m)[3]) {
#pragma clang fp contract(off)
  m[0] = m[1] = m[2] = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int qb = opp(q);
    const R w = (R)wq(q);
    const R cuV = dotc<R>(q, vx, vy, vz);
    const R eVq = geq1<R>(w, baseV, cuV);
    R om;
    if (M == 1) {
      om = (g[qb] - geq1<R>(w, baseU, -dotc<R>(q, ux, uy, uz))) - (g[q] - eVq);
    } else if (M == 2) {
      om = fmac<R>(one_m_inv_tau, g[q] - geq1<R>(w, baseU, dotc<R>(q, ux, uy, uz)), eVq - g[q]);
    } else {
      om = (g[qb] - geq1<R>(w, baseV, -cuV)) - (g[q] - eVq);
    }
    acc[q] = fmac<R>(B, om, acc[q]);
    // m -= c_q om, component by component
    if (cx(q) > 0) m[0] -= om;
    if (cx(q) < 0) m[0] += om;
    if (cy(q) > 0) m[1] -= om;
    if (cy(q) < 0) m[1] += om;
    if (cz(q) > 0) m[2] -= om;
    if (cz(q) < 0) m[2] += om;
  }
}

// g: pre-collision deviations of cell c (instance I), L: the cell's leader
// pair.  Writes the post-collision deviations to out and the six force/torque
// components of every member pair to pairs.out (with FT_REGS, for a SINGLE
// cell, to ft instead).  M in {1, 2, 3} fixes the solid operator at compile
// time (0: I.psm_m decides); SINGLE declares that L is the cell's only pair.
// These only narrow what is compiled: every specialisation evaluates the same
// expressions in the same order.
template <int M, bool SINGLE, typename R, bool FT_REGS = false>
__device__ __forceinline__ void psm_cell_collide(const R (&g)[Q], R (&out)[Q], const InstDev& I, const PartDev& P,
                                                 const PairDev& pairs, int L, int c, double* ft = nullptr) {
#pragma clang fp contract(off)
  static_assert(SINGLE || !FT_REGS, "force terms in registers only for cells of a single pair");
  int mem[SINGLE ? 1 : KMAX];
  int k = 1;
  if constexpr (SINGLE)
    mem[0] = L;
  else
    k = gather_members(pairs, L, mem);
  R drho = 0, ux = 0, uy = 0, uz = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    drho += g[q];
    if (cx(q) > 0) ux += g[q];
    if (cx(q) < 0) ux -= g[q];
    if (cy(q) > 0) uy += g[q];
    if (cy(q) < 0) uy -= g[q];
    if (cz(q) > 0) uz += g[q];
    if (cz(q) < 0) uz -= g[q];
  }
  const R baseU = eq_base<R>(drho, ux, uy, uz);
  const R lp = (R)I.lam_p, lm = (R)I.lam_m;
  const R fx = (R)I.fext[0], fy = (R)I.fext[1], fz = (R)I.fext[2];
  const R fu = fmac<R>(uz, fz, fmac<R>(uy, fy, ux * fx));
  // weights, normalised where several particles share the cell and sum above 1
  double Braw = 0.0;
  for (int m = 0; m < k; ++m) Braw += pairs.B[mem[m]];
  const bool normalise = Braw > 1.0;
  const double inv = normalise ? 1.0 / Braw : 1.0;
  double Bsum = 0.0;
  R acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0;
  const int x = c % I.nx, yz = c / I.nx, y = yz % I.ny, z = yz / I.ny;
  const R omit = (R)1 - (R)(1.0 / I.tau);
  const int Mv = M ? M : I.psm_m;
  for (int m = 0; m < (SINGLE ? 1 : k); ++m) {
    const int pm = pairs.p[mem[m]];
    const double Bm = normalise ? pairs.B[mem[m]] * inv : pairs.B[mem[m]];
    Bsum += Bm;
    double r[3];
    r[0] = min_image(((double)x + 0.5) - P.X[3 * pm + 0], (double)I.nx);
    r[1] = min_image(((double)y + 0.5) - P.X[3 * pm + 1], (double)I.ny);
    r[2] = min_image(((double)z + 0.5) - P.X[3 * pm + 2], (double)I.nz);
    const double* Up = P.U + 3 * pm;
    const double* Wp = P.Om + 3 * pm;
    const R vx = (R)(Up[0] + (Wp[1] * r[2] - Wp[2] * r[1]));
    const R vy = (R)(Up[1] + (Wp[2] * r[0] - Wp[0] * r[2]));
    const R vz = (R)(Up[2] + (Wp[0] * r[1] - Wp[1] * r[0]));
    const R baseV = eq_base<R>(drho, vx, vy, vz);
    R mv[3];
    if (Mv == 1)
      add_solid_operator<1, R>(g, acc, (R)Bm, baseU, ux, uy, uz, baseV, vx, vy, vz, omit, mv);
    else if (Mv == 2)
      add_solid_operator<2, R>(g, acc, (R)Bm, baseU, ux, uy, uz, baseV, vx, vy, vz, omit, mv);
    else
      add_solid_operator<3, R>(g, acc, (R)Bm, baseU, ux, uy, uz, baseV, vx, vy, vz, omit, mv);
    // F_s = B_s sum_q Omega_q c_qbar, T_s = (x_s - X_p) x F_s
    const double Fx = Bm * (double)mv[0], Fy = Bm * (double)mv[1], Fz = Bm * (double)mv[2];
    if constexpr (FT_REGS) {
      ft[0] = Fx;
      ft[1] = Fy;
      ft[2] = Fz;
      ft[3] = r[1] * Fz - r[2] * Fy;
      ft[4] = r[2] * Fx - r[0] * Fz;
      ft[5] = r[0] * Fy - r[1] * Fx;
    } else {
      double* o = pairs.out + mem[m];
      const long long s = pairs.ostride;
      o[0] = Fx;
      o[s] = Fy;
      o[2 * s] = Fz;
      o[3 * s] = r[1] * Fz - r[2] * Fy;
      o[4 * s] = r[2] * Fx - r[0] * Fz;
      o[5 * s] = r[0] * Fy - r[1] * Fx;
    }
  }
  const R omB = (R)(1.0 - Bsum);
  // fluid operator and forcing, then Eq. LBM_Collide_PSM:
  // out = g + (1 - B)(C + F) + sum_s B_s Omega_s
  {
    const R C0 = lp * (g[0] - (R)wq(0) * baseU);
    const R F0 = -(R)wq(0) * (R)3 * fu;
    out[0] = fmac<R>(omB, C0 + F0, g[0] + acc[0]);
#pragma unroll
    for (int qa = 1; qa < Q; qa += 2) {
      const int qb = qa + 1;
      const R w = (R)wq(qa);
      const R cu = dotc<R>(qa, ux, uy, uz);
      const R cf = dotc<R>(qa, fx, fy, fz);
      const R ea = geq1<R>(w, baseU, cu), eb = geq1<R>(w, baseU, -cu);
      const R gp = (R)0.5 * (g[qa] + g[qb]), gm = (R)0.5 * (g[qa] - g[qb]);
      const R ep = (R)0.5 * (ea + eb), em = (R)0.5 * (ea - eb);
      const R cp = lp * (gp - ep), cm = lm * (gm - em);
      const R Fp = w * fmac<R>((R)9 * cu, cf, (R)-3 * fu), Fm = w * ((R)3 * cf);
      out[qa] = fmac<R>(omB, (cp + cm) + (Fp + Fm), g[qa] + acc[qa]);
      out[qb] = fmac<R>(omB, (cp - cm) + (Fp - Fm), g[qb] + acc[qb]);
    }
  }
}

}  // namespace lbm
