"""Momentum exchange method (Sec. 2.2), FP64, in deviation variables.

Owner field: -1 fluid, -2 - k a cell of static wall group k, p >= 0 a solid cell
of particle p (binary mapping: a cell is solid iff its centre is inside the sphere).

A link (x, q) joins a fluid cell x to a solid cell x + c_q.  After streaming,
f_qbar(x, t+1) is set by
  BB  (Eq. MEM_BB):  f_qbar = f~_q(x) - 2 w_q/c_s^2 v(x_b).c_q,            x_b = x + c_q/2
  CLI (Eq. MEM_CLI): f_qbar = f~_q(x) + k0 f~_q(x - c_q) - k0 f~_qbar(x)
                              - alpha w_q/c_s^2 v(x_b).c_q,                  x_b = x + delta_q c_q
with k0 = (1 - 2 delta)/(1 + 2 delta), alpha = 4/(1 + 2 delta).  In deviation
variables the w terms cancel (w_q = w_qbar and 1 + k0 - k0 = 1), so the same
expressions hold for g.  Reading (the paper is silent): where x - c_q is not a
fluid cell, CLI falls back to BB for that link.  Static-wall links always use BB
with the wall velocity.

Link force (Eq. MEM_Force, dx = dt = 1):
  F^q = (c_q - v) f~_q(x, t) - (c_qbar - v) f_qbar(x, t+1) = (c_q - v) f~_q + (c_q + v) f_qbar
      = 2 w_q c_q + (c_q - v) g~_q + (c_q + v) g_qbar          (f = w + g, w_q = w_qbar).
Totals, Eqs. MEM_TotForce/TotTorque: F = sum F^q, T = sum (x_b - X_p) x F^q.
The constant part 2 w_q c_q sums to zero over the links of one closed body:
every lattice line that enters the body along c_q leaves it along c_qbar, and
both links lie on that line, so their constant forces cancel and so do their
torques ((x_b - x'_b) is parallel to c_q).  The totals are therefore formed
from the deviation part only, which keeps them accurate to the rounding of the
deviations rather than of w_q.  This needs each body's solid run on every
lattice line to be bounded by fluid cells (particles not in contact; the
paper defines no contact model); ``check_link_balance`` verifies the
necessary per-direction link balance.

Static wall groups carry one of two rules.  A velocity wall is bounce-back
with the wall velocity (Eq. MEM_BB); with a wall velocity normal to the wall it
is the velocity inflow of the settling-sphere frame (Sec. 4.1).  An outflow
group is the pressure anti-bounce-back of that frame (Sec. 4.1, after Ginzburg):
  f_qbar(x, t+1) = -f~_q(x, t) + 2 f^eq,+_q(rho_out, u(x, t)),
with f^eq,+ the even part of Eq. LBM_EQ, w_q (rho + 9/2 (c_q.u)^2 - 3/2 u.u)
(rho0 = 1 in the nonlinear terms), and u(x, t) the velocity of Eq. MacVel in
the fluid cell x at time t (before its collision).  In deviation variables
(w_q = w_qbar):
  g_qbar = -g~_q + 2 w_q (rho_out - 1 + 9/2 (c_q.u)^2 - 3/2 u.u).

Refill (Sec. 2.2.3, Eq. MEM_Reconstruction).  Readings (parity unpinned where
noted):
* normal n = (x - X_p)/|x - X_p| from the new particle position; q_n maximises
  n . c_q/|c_q| (normalised velocities); ties go to the largest velocity vector in
  lexicographic (c_x, c_y, c_z) order -- parity unpinned;
* sources x + k c_qn (k = 1, 2, 3) must be fluid cells that were fluid before
  the remap; with three: 3 f1 - 3 f2 + f3, with two: 2 f1 - f2, with one: f1,
  with none: f^eq(rho_bar, v(x)) where rho_bar is the mean density of the old-fluid
  neighbours among the 18 directions (rho0 if there are none; carried as the
  mean fluctuation) -- parity unpinned;
* velocity constraint: in the orthogonal D3Q19 moment basis the momentum rows
  are c_qa with norm sum_q c_qa^2 = 10, so f_q += c_q.(j* - j)/10 sets the
  momentum j = sum f c to j* and leaves every other orthogonal moment unchanged;
  j* = v(x) - f_ext/2 so that Eq. MacVel gives u = v.
"""
import math

import numpy as np

from .geometry import centre_disp, link_delta
from .lattice import CF, W, OPP, C
from .fluid import geq
from .rigid import surface_velocity

FLUID = -1
WALL = -2  # wall group k is stored as WALL - k
SQRT1_2 = 0.7071067811865476  # 1/sqrt(2) rounded to double


def build_links(owner, parts, radii, box_shape, v_walls, wall_outflow=None):
    """All links (x fluid, q) with x + c_q solid; returns a dict of arrays."""
    nz, ny, nx = box_shape
    fluid = owner == FLUID
    rec = {k: [] for k in ("iz", "iy", "ix", "q", "p")}
    for q in range(1, 19):
        cx, cy, cz = (int(v) for v in C[q])
        nb = np.roll(owner, shift=(-cz, -cy, -cx), axis=(0, 1, 2))  # owner[x + c_q]
        sel = fluid & (nb != FLUID)
        iz, iy, ix = np.nonzero(sel)
        rec["iz"].append(iz); rec["iy"].append(iy); rec["ix"].append(ix)
        rec["q"].append(np.full(len(iz), q)); rec["p"].append(nb[sel])
    L = {k: np.concatenate(v).astype(np.int64) for k, v in rec.items()}
    n = len(L["q"])
    c = CF[L["q"]]  # (n, 3)
    delta = np.full(n, 0.5)
    d = np.stack([L["ix"] + 0.5, L["iy"] + 0.5, L["iz"] + 0.5], axis=-1).astype(np.float64)
    X = np.zeros((n, 3))
    Ul = np.zeros((n, 3))
    Oml = np.zeros((n, 3))
    isp = L["p"] >= 0
    for p in np.unique(L["p"][isp]):
        s = L["p"] == p
        Xp = parts[p]["X"]
        dp = np.stack([centre_disp(L["ix"][s], Xp[0], nx), centre_disp(L["iy"][s], Xp[1], ny),
                       centre_disp(L["iz"][s], Xp[2], nz)], axis=-1)
        d[s] = dp
        delta[s] = link_delta(dp, c[s], radii[p])
        X[s] = Xp
        Ul[s] = parts[p]["U"]
        Oml[s] = parts[p]["Om"]
    # CLI needs x - c_q to be a fluid cell
    bz = np.mod(L["iz"] - C[L["q"], 2], nz)
    by = np.mod(L["iy"] - C[L["q"], 1], ny)
    bx = np.mod(L["ix"] - C[L["q"], 0], nx)
    L["cli_ok"] = owner[bz, by, bx] == FLUID
    L["bz"], L["by"], L["bx"] = bz, by, bx
    L["delta"] = delta
    L["d"] = d  # x - X_p (particle links only)
    L["is_particle"] = isp
    L["U"], L["Om"] = Ul, Oml
    vw = np.zeros((n, 3))
    outflow = np.zeros(n, bool)
    rho_out = np.ones(n)
    for k, v in enumerate(v_walls):
        sel = L["p"] == WALL - k
        vw[sel] = v
        if wall_outflow is not None and wall_outflow[k] is not None:
            outflow[sel] = True
            rho_out[sel] = wall_outflow[k]
    L["v_wall"] = vw
    L["outflow"] = outflow
    L["rho_out"] = rho_out
    return L


def link_boundary(gt, gn, L, scheme, g=None, fext=None):
    """Apply BB/CLI on every link (the outflow rule on outflow wall links, which
    needs the pre-collision PDFs g and the body force for u(x, t)) and return
    per-link (F^q, T^q)."""
    n = len(L["q"])
    if n == 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    q = L["q"]
    qb = OPP[q]
    c = CF[q]
    iz, iy, ix = L["iz"], L["iy"], L["ix"]
    use_cli = (scheme == "cli") & L["cli_ok"] & L["is_particle"]
    delta = np.where(use_cli, L["delta"], 0.5)
    arm = L["d"] + delta[:, None] * c  # x_b - X_p
    v = np.where(L["is_particle"][:, None], surface_velocity(L["U"], L["Om"], arm) if n else 0.0,
                 L["v_wall"])
    vc = (v * c).sum(axis=1)
    wq = W[q]
    gtq = gt[q, iz, iy, ix]
    bb = gtq - 6.0 * wq * vc
    k0 = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta)
    alpha = 4.0 / (1.0 + 2.0 * delta)
    cli = gtq + k0 * gt[q, L["bz"], L["by"], L["bx"]] - k0 * gt[qb, iz, iy, ix] - 3.0 * alpha * wq * vc
    val = np.where(use_cli, cli, bb)
    out = L["outflow"]
    if out.any():
        gc = g[:, iz[out], iy[out], ix[out]]  # f(x, t) of the links' fluid cells
        u = (CF.T @ gc).T + 0.5 * np.asarray(fext, dtype=np.float64)  # Eq. MacVel, (n_out, 3)
        cu = (c[out] * u).sum(axis=1)
        uu = (u * u).sum(axis=1)
        val = val.copy()
        val[out] = -gtq[out] + 2.0 * wq[out] * ((L["rho_out"][out] - 1.0) + 4.5 * cu * cu - 1.5 * uu)
    gn[qb, iz, iy, ix] = val
    Fq = (c - v) * gtq[:, None] + (c + v) * val[:, None]
    Tq = np.cross(arm, Fq)
    return Fq, Tq


def check_link_balance(L, P):
    """Per particle, the number of links along c_q equals that along c_qbar."""
    for p in range(P):
        qs = L["q"][L["p"] == p]
        cnt = np.bincount(qs, minlength=19)
        if not np.array_equal(cnt, cnt[OPP]):
            raise ValueError("unbalanced links for particle %d: particles in contact are not supported" % p)


def refill_cell(g, owner, newmask, cell, Xp, Up, Omp, fext, box_shape, equilibrium=False):
    """PDF reconstruction of one newly uncovered cell (iz, iy, ix); returns g (19,).
    equilibrium=True skips the extrapolation: every uncovered cell takes the
    last fallback, f^eq(rho_bar, v(x)) (then the same velocity constraint)."""
    nz, ny, nx = box_shape
    iz, iy, ix = cell
    d = np.array([float(centre_disp(ix, Xp[0], nx)), float(centre_disp(iy, Xp[1], ny)),
                  float(centre_disp(iz, Xp[2], nz))])
    best = None
    for q in range(1, 19):
        c = C[q]
        dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2]
        score = dc if (c * c).sum() == 1 else dc * SQRT1_2
        key = (score, int(c[0]), int(c[1]), int(c[2]))
        if best is None or key > best[0]:
            best = (key, q)
    qn = best[1]
    cn = C[qn]

    def ok(z, y, x):
        return owner[z, y, x] == FLUID and not newmask[z, y, x]

    src = []
    for k in (1, 2, 3):
        z, y, x = (iz + k * cn[2]) % nz, (iy + k * cn[1]) % ny, (ix + k * cn[0]) % nx
        if equilibrium or not ok(z, y, x):
            break
        src.append(g[:, z, y, x])
    v = surface_velocity(Up, Omp, d)
    if len(src) == 3:
        out = 3.0 * src[0] - 3.0 * src[1] + src[2]
    elif len(src) == 2:
        out = 2.0 * src[0] - src[1]
    elif len(src) == 1:
        out = src[0].copy()
    else:
        drhos = []
        for q in range(1, 19):
            c = C[q]
            z, y, x = (iz + c[2]) % nz, (iy + c[1]) % ny, (ix + c[0]) % nx
            if ok(z, y, x):
                drhos.append(g[:, z, y, x].sum())
        drho_bar = float(np.mean(drhos)) if drhos else 0.0
        out = geq(np.array(drho_bar), v.reshape(3))
    j = CF.T @ out
    jstar = v - 0.5 * np.asarray(fext, dtype=np.float64)
    out = out + (CF @ (jstar - j)) / 10.0
    return out
