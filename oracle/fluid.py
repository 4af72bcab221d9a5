"""Lattice Boltzmann fluid core (Sec. 2.1), FP64, in deviation variables.

With g_q = f_q - w_q and sum_q w_q = 1, sum_q w_q c_q = 0, and the density
written as rho_f = rho0 + drho_f (Sec. 2.1, rho0 = 1):
  drho_f = sum_q g_q,   U = sum_q f_q c_q / rho0 = sum_q g_q c_q.
Equilibrium (Eq. LBM_EQ, rho0 = 1, c_s^2 = 1/3):
  f^eq_q = w_q (rho0 + drho_f + 3 c.U + 9/2 (c.U)^2 - 3/2 U.U),  so
  g^eq_q = f^eq_q - w_q = w_q (drho_f + 3 c.U + 9/2 (c.U)^2 - 3/2 U.U).
The fluctuation drho_f is carried as its own variable (never through 1 + drho_f).
Collision operators act on f - f^eq = g - g^eq, so they read identically in g.
All arrays are g[q, z, y, x]; vectors are U[a, z, y, x] with a = 0 (x), 1 (y), 2 (z).
"""
import numpy as np

from .lattice import CF, W, OPP, Q


def moments(g):
    """Density fluctuation drho_f = rho_f - rho0 and velocity U (the moment
    definitions after Eq. LBM_EQ)."""
    drho = g.sum(axis=0)
    U = np.tensordot(CF.T, g, axes=([1], [0]))  # (3, ...)
    return drho, U


def geq(drho, U, cu=None):
    """Deviation of the incompressible equilibrium, Eq. LBM_EQ, from w_q, as a
    function of the density fluctuation drho_f and the velocity U."""
    if cu is None:
        cu = np.tensordot(CF, U, axes=([1], [0]))  # (19, ...)
    uu = (U * U).sum(axis=0)
    wq = W.reshape((Q,) + (1,) * (cu.ndim - 1))
    return wq * ((drho - 1.5 * uu) + cu * (3.0 + 4.5 * cu))


def forcing(U, fext, cu=None):
    """Forcing operator, Eq. Forcing, with dt = 1 and c_s^2 = 1/3:
    F_q = w_q [ (c_q - U)/c_s^2 + (c_q.U) c_q / c_s^4 ] . f_ext
        = w_q [ 3 (c_q.f - U.f) + 9 (c_q.U)(c_q.f) ]."""
    fext = np.asarray(fext, dtype=np.float64)
    if cu is None:
        cu = np.tensordot(CF, U, axes=([1], [0]))  # c_q . U
    ex = (Q,) + (1,) * (cu.ndim - 1)
    cf = (CF @ fext).reshape(ex)  # c_q . f_ext
    uf = np.tensordot(fext, U, axes=([0], [0]))  # U . f_ext
    return W.reshape(ex) * (3.0 * (cf - uf) + 9.0 * cf * cu)


def tau_from_nu(nu):
    """Eq. Viscosity with dt = 1, c_s^2 = 1/3: nu = (tau - 1/2)/3."""
    return 3.0 * nu + 0.5


def trt_rates(tau, magic):
    """TRT relaxation rates (after Eq. MEM_TRT): lambda_+ = -1/tau and lambda_-
    from the magic parameter Lambda = (1/2 + 1/lambda_+)(1/2 + 1/lambda_-)."""
    lam_p = -1.0 / tau
    # (1/2 + 1/lam_m) = Lambda / (1/2 + 1/lam_p)
    inv_m = magic / (0.5 + 1.0 / lam_p) - 0.5
    lam_m = 1.0 / inv_m
    return lam_p, lam_m


def collide_bgk(g, tau, fext):
    """Eq. LBM_Collide with the BGK operator, Eq. LBM_SRT:
    f~ = f + (f^eq - f)/tau + F."""
    drho, U = moments(g)
    cu = np.tensordot(CF, U, axes=([1], [0]))
    return g + (geq(drho, U, cu) - g) / tau + forcing(U, fext, cu)


def collide_trt(g, lam_p, lam_m, fext):
    """Eq. LBM_Collide with the TRT operator, Eq. MEM_TRT:
    f~ = f + lambda_+ (f^+ - f^eq,+) + lambda_- (f^- - f^eq,-) + F,
    with f^+- = (f_q +- f_qbar)/2.  Since w_q = w_qbar, f - f^eq = g - g^eq and
    the split reads the same in g:  with n = g - g^eq,
    lambda_+ n^+ + lambda_- n^- = (lambda_+ + lambda_-)/2 n_q + (lambda_+ - lambda_-)/2 n_qbar."""
    drho, U = moments(g)
    cu = np.tensordot(CF, U, axes=([1], [0]))
    n = g - geq(drho, U, cu)
    c = (0.5 * (lam_p + lam_m)) * n + (0.5 * (lam_p - lam_m)) * n[OPP]
    return g + c + forcing(U, fext, cu)


def fluid_operator(g, drho, U, collision, tau, magic):
    """The collision operator C_q alone (no forcing): BGK, Eq. LBM_SRT, or TRT,
    Eq. MEM_TRT (same arithmetic as ``collide_bgk`` / ``collide_trt``).  Used as
    the fluid part of the PSM operator, Eq. PSM."""
    ge = geq(drho, U)
    if collision == "bgk":
        return (ge - g) / tau
    lam_p, lam_m = trt_rates(tau, magic)
    n = g - ge
    return (0.5 * (lam_p + lam_m)) * n + (0.5 * (lam_p - lam_m)) * n[OPP]


def collide(g, collision, tau, magic, fext):
    if collision == "bgk":
        return collide_bgk(g, tau, fext)
    lam_p, lam_m = trt_rates(tau, magic)
    return collide_trt(g, lam_p, lam_m, fext)


def stream(gt):
    """Eq. LBM_Stream on a periodic box: f_q(x + c_q, t+1) = f~_q(x, t)."""
    out = np.empty_like(gt)
    for q in range(Q):
        cx, cy, cz = (int(v) for v in CF[q])
        out[q] = np.roll(gt[q], shift=(cz, cy, cx), axis=(0, 1, 2))
    return out


def macroscopic_velocity(U, fext):
    """Eq. MacVel with rho0 = dt = 1: u = U + f_ext/2."""
    fext = np.asarray(fext, dtype=np.float64).reshape((3,) + (1,) * (U.ndim - 1))
    return U + 0.5 * fext
