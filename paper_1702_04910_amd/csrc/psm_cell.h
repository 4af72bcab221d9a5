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

// Equilibrium deviation, Eq. LBM_EQ minus w_q, for all q.
template <typename R>
__device__ __forceinline__ void geq_all(R drho, R ux, R uy, R uz, R (&e)[Q]) {
  const R base = drho - (R)1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const R cu = (R)cx(q) * ux + (R)cy(q) * uy + (R)cz(q) * uz;
    e[q] = (R)wq(q) * (base + cu * ((R)3 + (R)4.5 * cu));
  }
}

// g: pre-collision deviations of cell c (instance I), L: the cell's leader
// pair.  Writes the post-collision deviations to out and the six force/torque
// components of every member pair to pairs.out.
template <typename R>
__device__ __forceinline__ void psm_cell_collide(const R (&g)[Q], R (&out)[Q], const InstDev& I, const PartDev& P,
                                                 const PairDev& pairs, int L, int c) {
  int mem[KMAX];
  const int k = gather_members(pairs, L, mem);
  R drho = 0, ux = 0, uy = 0, uz = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    drho += g[q];
    ux += (R)cx(q) * g[q];
    uy += (R)cy(q) * g[q];
    uz += (R)cz(q) * g[q];
  }
  R eU[Q];
  geq_all<R>(drho, ux, uy, uz, eU);
  const R lp = (R)I.lam_p, lm = (R)I.lam_m;
  const R fx = (R)I.fext[0], fy = (R)I.fext[1], fz = (R)I.fext[2];
  const R fu = ux * fx + uy * fy + uz * fz;
  // weights, normalised where several particles share the cell and sum above 1
  double Bs[KMAX];
  double Bsum = 0.0;
  for (int m = 0; m < k; ++m) {
    Bs[m] = pairs.B[mem[m]];
    Bsum += Bs[m];
  }
  if (Bsum > 1.0) {
    for (int m = 0; m < k; ++m) Bs[m] = Bs[m] * (1.0 / Bsum);
    Bsum = 0.0;
    for (int m = 0; m < k; ++m) Bsum += Bs[m];
  }
  R acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0;
  const int x = c % I.nx, yz = c / I.nx, y = yz % I.ny, z = yz / I.ny;
  const R inv_tau = (R)(1.0 / I.tau);
  for (int m = 0; m < k; ++m) {
    const int pm = pairs.p[mem[m]];
    double r[3];
    r[0] = min_image(((double)x + 0.5) - P.X[3 * pm + 0], (double)I.nx);
    r[1] = min_image(((double)y + 0.5) - P.X[3 * pm + 1], (double)I.ny);
    r[2] = min_image(((double)z + 0.5) - P.X[3 * pm + 2], (double)I.nz);
    const double* Up = P.U + 3 * pm;
    const double* Wp = P.Om + 3 * pm;
    const double v0 = Up[0] + (Wp[1] * r[2] - Wp[2] * r[1]);
    const double v1 = Up[1] + (Wp[2] * r[0] - Wp[0] * r[2]);
    const double v2 = Up[2] + (Wp[0] * r[1] - Wp[1] * r[0]);
    R eV[Q];
    geq_all<R>(drho, (R)v0, (R)v1, (R)v2, eV);
    const R B = (R)Bs[m];
    R mx = 0, my = 0, mz = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int qb = opp(q);
      R om;
      if (I.psm_m == 1) om = (g[qb] - eU[qb]) - (g[q] - eV[q]);
      else if (I.psm_m == 2) om = (eV[q] - g[q]) + ((R)1 - inv_tau) * (g[q] - eU[q]);
      else om = (g[qb] - eV[qb]) - (g[q] - eV[q]);
      acc[q] += B * om;
      mx -= (R)cx(q) * om;
      my -= (R)cy(q) * om;
      mz -= (R)cz(q) * om;
    }
    // F_s = B_s sum_q Omega_q c_qbar, T_s = (x_s - X_p) x F_s
    const double Fx = Bs[m] * (double)mx, Fy = Bs[m] * (double)my, Fz = Bs[m] * (double)mz;
    double* o = pairs.out + mem[m];
    const long long s = pairs.ostride;
    o[0] = Fx;
    o[s] = Fy;
    o[2 * s] = Fz;
    o[3 * s] = r[1] * Fz - r[2] * Fy;
    o[4 * s] = r[2] * Fx - r[0] * Fz;
    o[5 * s] = r[0] * Fy - r[1] * Fx;
  }
  const R omB = (R)(1.0 - Bsum);
  // fluid operator and forcing, then Eq. LBM_Collide_PSM
  {
    const R base = drho - (R)1.5 * (ux * ux + uy * uy + uz * uz);
    const R C0 = lp * (g[0] - (R)wq(0) * base);
    const R F0 = -(R)wq(0) * (R)3 * fu;
    out[0] = g[0] + omB * C0 + acc[0] + omB * F0;
#pragma unroll
    for (int qa = 1; qa < Q; qa += 2) {
      const int qb = qa + 1;
      const R w = (R)wq(qa);
      const R cu = (R)cx(qa) * ux + (R)cy(qa) * uy + (R)cz(qa) * uz;
      const R cf = (R)cx(qa) * fx + (R)cy(qa) * fy + (R)cz(qa) * fz;
      const R gp = (R)0.5 * (g[qa] + g[qb]), gm = (R)0.5 * (g[qa] - g[qb]);
      const R ep = (R)0.5 * (eU[qa] + eU[qb]), em = (R)0.5 * (eU[qa] - eU[qb]);
      const R cp = lp * (gp - ep), cm = lm * (gm - em);
      const R Fp = w * ((R)9 * cu * cf - (R)3 * fu), Fm = w * ((R)3 * cf);
      out[qa] = g[qa] + omB * (cp + cm) + acc[qa] + omB * (Fp + Fm);
      out[qb] = g[qb] + omB * (cp - cm) + acc[qb] + omB * (Fp - Fm);
    }
  }
}

}  // namespace lbm
