"""Partially saturated cells method (Sec. 2.3), FP64, in deviation variables.

Solid collision operators (Eqs. PSM_M1..M3), with rho = rho_f of the cell
(carried as drho_f, see ``fluid``) and
v_s the particle surface velocity (Eq. bodyVelocity) at the cell centre; since
w_q = w_qbar every bracket f - f^eq equals g - g^eq:
  M1: Omega_q = [f_qbar - f^eq_qbar(rho,U)] - [f_q - f^eq_q(rho,v_s)]
  M2: Omega_q = [f^eq_q(rho,v_s) - f_q] + (1 - 1/tau)[f_q - f^eq_q(rho,U)]
  M3: Omega_q = [f_qbar - f^eq_qbar(rho,v_s)] - [f_q - f^eq_q(rho,v_s)]
Weights (Eqs. PSM_B1, PSM_B2): B1: B_s = eps_s; B2: B_s = eps_s (tau - 1/2) / ((1 - eps_s) + (tau - 1/2)).
Collision (Eqs. PSM, LBM_Collide_PSM):
  f~ = f + (1 - B) C^fluid + sum_s B_s Omega_s + (1 - B) F,   B = sum_s B_s.
C^fluid is BGK in the paper; the TRT operator is accepted as well.
Force and torque (Eqs. PSM_TotForce, PSM_TotTorque), applied at the cell centre x_s:
  F_s = sum_x B_s sum_q Omega_q c_qbar,  T_s = sum_x B_s (x_s - X_p) x sum_q Omega_q c_qbar.
Where several particles overlap one cell and sum_s B_s exceeds 1 (the paper is
silent), every B_s of that cell is divided by the sum.
"""
import numpy as np

from .fluid import moments, geq, forcing, fluid_operator
from .geometry import centre_disp
from .lattice import CF, OPP
from .rigid import surface_velocity


def weight(eps, tau, bsel):
    if bsel == 1:
        return eps.copy()
    t = tau - 0.5
    return eps * t / ((1.0 - eps) + t)


def solid_operator(gc, drho, U, vs, tau, msel):
    """Omega for cells given as columns: gc (19, n), drho (n,), U (3, n), vs (3, n)."""
    ge_u = geq(drho, U)
    ge_v = geq(drho, vs)
    if msel == 1:
        return (gc[OPP] - ge_u[OPP]) - (gc - ge_v)
    if msel == 2:
        return (ge_v - gc) + (1.0 - 1.0 / tau) * (gc - ge_u)
    if msel == 3:
        return (gc[OPP] - ge_v[OPP]) - (gc - ge_v)
    raise ValueError(msel)


def psm_collide(g, overlaps, parts, collision, tau, magic, fext, msel, bsel):
    """One PSM collision over the whole box.

    overlaps: list (one per particle) of (iz, iy, ix, eps) arrays.
    parts: list of dicts with keys X, U, Om (3-vectors).
    Returns (g_post, F (P,3), T (P,3), Bfield, sum_s B_s v_s field)."""
    shape = g.shape[1:]
    nz, ny, nx = shape
    drho, U = moments(g)
    Cf = fluid_operator(g, drho, U, collision, tau, magic)
    Fq = forcing(U, fext)

    Braw = np.zeros(shape)
    Bs_list = []
    for (iz, iy, ix, eps) in overlaps:
        Bs = weight(eps, tau, bsel)
        Bs_list.append(Bs)
        np.add.at(Braw, (iz, iy, ix), Bs)
    scale = np.where(Braw > 1.0, 1.0 / np.where(Braw > 1.0, Braw, 1.0), 1.0)

    B = np.zeros(shape)
    solid_sum = np.zeros_like(g)
    vB = np.zeros((3,) + shape)
    P = len(parts)
    F = np.zeros((P, 3))
    T = np.zeros((P, 3))
    for s, ((iz, iy, ix, eps), Bs) in enumerate(zip(overlaps, Bs_list)):
        if len(iz) == 0:
            continue
        Bs = Bs * scale[iz, iy, ix]
        p = parts[s]
        r = np.stack([centre_disp(ix, p["X"][0], nx), centre_disp(iy, p["X"][1], ny),
                      centre_disp(iz, p["X"][2], nz)], axis=-1)  # (n, 3) = x_s - X_p
        vs = surface_velocity(p["U"], p["Om"], r).T  # (3, n)
        gc = g[:, iz, iy, ix]
        om = solid_operator(gc, drho[iz, iy, ix], U[:, iz, iy, ix], vs, tau, msel)
        np.add.at(B, (iz, iy, ix), Bs)
        for q in range(19):
            np.add.at(solid_sum[q], (iz, iy, ix), Bs * om[q])
        for a in range(3):
            np.add.at(vB[a], (iz, iy, ix), Bs * vs[a])
        # sum_q Omega_q c_qbar = - sum_q Omega_q c_q
        mom = -(CF.T @ om)  # (3, n)
        fcell = Bs * mom  # (3, n)
        F[s] = fcell.sum(axis=1)
        T[s] = np.cross(r, fcell.T).sum(axis=0)
    gpost = g + (1.0 - B) * Cf + solid_sum + (1.0 - B) * Fq
    return gpost, F, T, B, vB


def psm_velocity(U, fext, B, vB):
    """Eq. MacVel_PSM: u = (1 - B)(U + f_ext/2) + sum_s B_s v_s."""
    f = np.asarray(fext, dtype=np.float64).reshape((3,) + (1,) * (U.ndim - 1))
    return (1.0 - B) * (U + 0.5 * f) + vB
