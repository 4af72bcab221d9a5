"""Rigid-body update (Sec. 4.1: position and velocity advanced each step by an
explicit Euler integration of the acting forces), FP64.

Readings where the paper is silent:
* forward Euler for all three states, the position with the OLD velocity:
  U <- U + dt F_tot / m,  X <- X + dt U_old,  Omega <- Omega + dt T / I;
* solid sphere: V = pi D^3 / 6, m = rho_p V, I = m D^2 / 10;
* external force (rho_p - rho_f) V g + V f_ext: net gravity and the buoyancy of
  the fluid body force (the latter mirrors F_b of Sec. 3);
* dt is the number of LBM sweeps per rigid-body step (2 for MEM, Sec. 2.2.4).
"""
import math

import numpy as np


def sphere_volume(D):
    return math.pi * D ** 3 / 6.0


def euler_step(X, U, Om, F_h, T_h, D, rho_p, g, fext, dt, box):
    """One explicit Euler step of a single sphere.  Returns (X, U, Om) new."""
    V = sphere_volume(D)
    m = rho_p * V
    inertia = m * D * D / 10.0
    F_tot = np.asarray(F_h, dtype=np.float64) + (rho_p - 1.0) * V * np.asarray(g, dtype=np.float64) \
        + V * np.asarray(fext, dtype=np.float64)
    U_new = U + dt * F_tot / m
    X_new = np.mod(X + dt * U, np.asarray(box, dtype=np.float64))
    Om_new = Om + dt * np.asarray(T_h, dtype=np.float64) / inertia
    return X_new, U_new, Om_new


def surface_velocity(U, Om, r):
    """Eq. bodyVelocity: v(x) = U_p + Omega_p x (x - X_p), with r = x - X_p
    (arrays of shape (..., 3))."""
    r = np.asarray(r, dtype=np.float64)
    return np.asarray(U, dtype=np.float64) + np.cross(np.asarray(Om, dtype=np.float64), r)
