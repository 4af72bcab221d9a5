"""Helpers shared by the GPU parity tests: build the same case on the oracle
and on the HIP library (through the C-ABI), and compare them."""
import sys

import numpy as np

from oracle.lattice import C as ORACLE_C
from oracle.sim import OracleSim
from paper_1702_04910_amd import lbmps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def perm_gpu_to_oracle():
    gc = lbmps.velocities()
    perm = np.array([int(np.nonzero((ORACLE_C == gc[q]).all(axis=1))[0][0]) for q in range(19)])
    return perm


def gpu_to_oracle(g):
    perm = perm_gpu_to_oracle()
    out = np.empty_like(g)
    out[perm] = g
    return out


def oracle_to_gpu(g):
    perm = perm_gpu_to_oracle()
    return g[perm]


def make_pair(nx, ny, nz, nu, coupling="none", collision="trt", psm_m=1, psm_b=1, f_ext=(0, 0, 0),
              gravity=(0, 0, 0), precision="fp64", eps_n=8, eps_mode=0, parts=None, g0=None, n_sub=0,
              walls=None, tile_rows=0, block_threads=0, grid_blocks=0, sweep_flags=0, refill="extrapolation"):
    """parts: dict(X, U, Om, D, rho, fixed) lists; walls: list of (mask, v)."""
    ora = OracleSim(nx, ny, nz, nu, collision=collision, coupling=coupling, psm_m=psm_m, psm_b=psm_b, fext=f_ext,
                    gravity=gravity, n_sub=(n_sub or None), eps_n=eps_n, eps_recursive=(eps_mode == 1),
                    eps_estimator={3: "edge", 4: "distance"}.get(eps_mode), refill=refill)
    np_ = len(parts["D"]) if parts else 0
    dmax = max(parts["D"]) if parts else 0.0
    cfg = lbmps.make_config(nx, ny, nz, nu, collision=collision, coupling=coupling, psm_m=psm_m, psm_b=psm_b,
                            n_sub=n_sub, eps_n=eps_n, eps_mode=eps_mode, precision=precision,
                            max_particles=np_, max_diameter=dmax, f_ext=f_ext, gravity=gravity,
                            tile_rows=tile_rows, block_threads=block_threads, grid_blocks=grid_blocks,
                            sweep_flags=sweep_flags, refill=refill)
    sim = lbmps.Sim(cfg)
    if g0 is None:
        ora.init_equilibrium()
        sim.init_equilibrium()
    else:
        ora.set_pdfs(g0)
        sim.set_pdfs(oracle_to_gpu(g0))
    for (mask, v) in (walls or []):
        ora.set_static_solid(mask, v)
        sim.set_static_solid(mask, v)
    if parts:
        args = (parts["X"], parts["U"], parts["Om"], parts["D"], parts["rho"], parts["fixed"])
        ora.set_particles(*args)
        sim.set_particles(*args)
        if g0 is not None:
            ora.set_pdfs(g0)  # masks the solid cells again
    return ora, sim


def pdf_error(ora, sim):
    """max |g_gpu - g_oracle| / max |g_oracle| over fluid cells (canonical PDFs)."""
    go = ora.get_pdfs()
    gg = gpu_to_oracle(sim.get_pdfs())
    fluid = ora.owner == -1
    scale = np.abs(go[:, fluid]).max()
    return np.abs(gg[:, fluid] - go[:, fluid]).max() / scale, scale


def force_errors(ora, sim, inst=0):
    po = ora.particles()
    pg = sim.particles(inst)
    out = []
    for i in range(len(po["F"])):
        R = 0.5 * ora.parts[i]["D"]
        nF = np.linalg.norm(po["F"][i])
        eF = np.linalg.norm(pg["F"][i] - po["F"][i]) / nF
        eT = np.linalg.norm(pg["T"][i] - po["T"][i]) / (R * nF)
        out.append((eF, eT, nF))
    return out, po, pg


def link_set_errors(ora, sim):
    """Compare the MEM particle link sets: the sorted (cell, q, particle)
    triples must be equal (a discrete event); returns max |delta_gpu -
    delta_oracle| over the links.  Raises AssertionError on a set mismatch."""
    nz, ny, nx = ora.shape
    Lo = ora.links
    sel = Lo["p"] >= 0
    inv = np.empty(19, np.int64)
    inv[perm_gpu_to_oracle()] = np.arange(19)  # oracle q -> library q
    key_o = ((((Lo["iz"][sel] * ny + Lo["iy"][sel]) * nx + Lo["ix"][sel]) * 19 + inv[Lo["q"][sel]]) * 64
             + Lo["p"][sel])
    L = sim.links()
    key_g = (L["cell"].astype(np.int64) * 19 + L["q"]) * 64 + L["p"]
    oo, og = np.argsort(key_o), np.argsort(key_g)
    assert len(key_o) == len(key_g), (len(key_o), len(key_g))
    assert np.array_equal(key_o[oo], key_g[og])
    return float(np.abs(Lo["delta"][sel][oo] - L["delta"][og]).max()) if len(key_o) else 0.0


def overlap_set_check(ora, sim):
    """The PSM overlap lists (cell, particle, eps_s) must be equal exactly."""
    nz, ny, nx = ora.shape
    ko, eo = [], []
    for p, (iz, iy, ix, eps) in enumerate(ora.overlaps):
        ko.append(((iz * ny + iy) * nx + ix).astype(np.int64) * 64 + p)
        eo.append(eps)
    ko = np.concatenate(ko) if ko else np.zeros(0, np.int64)
    eo = np.concatenate(eo) if eo else np.zeros(0)
    ov = sim.overlaps()
    kg = ov["cell"].astype(np.int64) * 64 + ov["p"]
    o1, o2 = np.argsort(ko), np.argsort(kg)
    assert np.array_equal(ko[o1], kg[o2])
    assert np.array_equal(eo[o1], ov["eps"][o2])
