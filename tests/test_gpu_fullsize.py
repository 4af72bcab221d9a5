"""Parity at full size, in the launch configuration the benchmark times.

The 192x192x384 settling-sphere box (14.16 M cells) with the autotuned sweep
launch shape, started from a seeded random state.  The oracle cannot sweep
the whole box in seconds, but after two sweeps a fluid cell depends only on
its 5x5x5 neighbourhood: the oracle runs that neighbourhood as a periodic
5x5x5 box (the wrap only corrupts cells two away from the centre, which the
centre no longer sees) and its centre is compared with the library's.  The
sampled cells lie away from the sphere (no link or overlap within reach),
spread over the box including its periodic faces."""
import numpy as np
import pytest

from oracle.sim import OracleSim
from paper_1702_04910_amd import autotune, inputs, lbmps
from gpu_util import gpu_to_oracle, oracle_to_gpu, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _samples(shape, X, R, n, seed):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    out = []
    faces = [(0, None, None), (nz - 1, None, None), (None, 0, None), (None, ny - 1, None), (None, None, 0),
             (None, None, nx - 1)]
    while len(out) < n:
        z, y, x = int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))
        if len(out) < 2 * len(faces):  # cells on the periodic faces first
            fz, fy, fx = faces[len(out) % len(faces)]
            z = fz if fz is not None else z
            y = fy if fy is not None else y
            x = fx if fx is not None else x
        d = np.array([x + 0.5, y + 0.5, z + 0.5]) - X
        d -= np.array([nx, ny, nz]) * np.round(d / np.array([nx, ny, nz]))
        if np.linalg.norm(d) > R + 6:
            out.append((z, y, x))
    return out


@pytest.mark.parametrize("precision,coupling", [("fp32", "mem_cli"), ("fp32", "psm"), ("fp64", "mem_cli")])
def test_full_size_sampled_cells(precision, coupling):
    inp = inputs.c2_scale(0)
    nx, ny, nz = inp["nx"], inp["ny"], inp["nz"]
    best = autotune.tune(nx, ny, nz, precision)
    shape = {k: best[k] for k in ("tile_rows", "block_threads", "grid_blocks", "sweep_flags")}
    say("full size", precision, coupling, shape)
    cfg = lbmps.make_config(nx, ny, nz, inp["nu"], collision="trt", coupling=coupling, psm_m=3, psm_b=2, n_sub=2,
                            eps_n=8, eps_mode=lbmps.EPS_RECURSIVE, precision=precision, max_particles=1,
                            max_diameter=inp["D"], f_ext=inp["f_ext"], gravity=inp["gravity"], **shape)
    sim = lbmps.Sim(cfg)
    g0 = inputs.random_pdfs((nz, ny, nx), 1e-3, seed=21)  # oracle velocity order
    sim.set_pdfs(oracle_to_gpu(g0))
    sim.set_particles([inp["X"]], [[0, 0, 0]], [[0, 0, 0]], [inp["D"]], [inp["rho"]], [False])
    sim.step(2)
    g2 = sim.get_pdfs()
    sim.close()
    cells = _samples((nz, ny, nx), inp["X"], 0.5 * inp["D"], 120, seed=22)
    scale = np.abs(g0).max()
    worst = 0.0
    for (z, y, x) in cells:
        iz = (np.arange(z - 2, z + 3)) % nz
        iy = (np.arange(y - 2, y + 3)) % ny
        ix = (np.arange(x - 2, x + 3)) % nx
        sub = g0[:, iz][:, :, iy][:, :, :, ix]
        ora = OracleSim(5, 5, 5, inp["nu"], collision="trt", fext=inp["f_ext"])
        ora.set_pdfs(sub)
        ora.step(2)
        want = ora.get_pdfs()[:, 2, 2, 2]
        got = gpu_to_oracle(g2[:, z, y, x][:, None])[:, 0]
        worst = max(worst, float(np.abs(got - want).max() / scale))
    say("  %d sampled cells, max relative error %.3e" % (len(cells), worst))
    assert worst < TOL[precision]


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_full_size_work_beside_the_sweep_is_bitwise_identical(coupling):
    """The full-size box in the timed launch shape with a fast sphere: eight
    sweeps in one call (remap or rebuild beside the next sweep, refilled cells
    re-swept) equal four calls of one rigid-body step each (in order), bit
    for bit."""
    inp = inputs.c2_scale(0)
    nx, ny, nz = inp["nx"], inp["ny"], inp["nz"]
    best = autotune.tune(nx, ny, nz, "fp32")
    shape = {k: best[k] for k in ("tile_rows", "block_threads", "grid_blocks", "sweep_flags")}
    say("full size beside the sweep", coupling, shape)
    cfg = lbmps.make_config(nx, ny, nz, inp["nu"], collision="trt", coupling=coupling, psm_m=3, psm_b=2, n_sub=2,
                            eps_n=8, eps_mode=lbmps.EPS_RECURSIVE, precision="fp32", max_particles=1,
                            max_diameter=inp["D"], f_ext=inp["f_ext"], gravity=inp["gravity"], **shape)
    out = []
    for per_call in (2, 8):
        sim = lbmps.Sim(cfg)
        sim.init_equilibrium()
        sim.set_particles([inp["X"]], [[0.05, -0.03, -0.2]], [[0.0, 0.004, 0.0]], [inp["D"]], [inp["rho"]],
                          [False])
        for k in range(8 // per_call):
            sim.step(per_call)
        out.append((sim.get_pdfs().astype(np.float32), sim.particles()))
        sim.close()
    (ga, pa), (gb, pb) = out
    assert np.array_equal(ga, gb)
    for key in ("F", "T", "U", "Omega", "X"):
        assert np.array_equal(pa[key], pb[key]), key
    say("  sphere moved by %s" % (pb["X"][0] - np.asarray(inp["X"])))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_mass_and_momentum(precision):
    """Periodic fluid at full size: mass is conserved and the momentum grows
    by N f_ext per sweep (Eq. Forcing has exactly these moments)."""
    inp = inputs.c2_scale(0)
    nx, ny, nz = inp["nx"], inp["ny"], inp["nz"]
    N = nx * ny * nz
    best = autotune.tune(nx, ny, nz, precision)
    shape = {k: best[k] for k in ("tile_rows", "block_threads", "grid_blocks", "sweep_flags")}
    f = (1e-6, -5e-7, 2e-7)
    cfg = lbmps.make_config(nx, ny, nz, inp["nu"], collision="trt", precision=precision, f_ext=f, **shape)
    sim = lbmps.Sim(cfg)
    g0 = inputs.random_pdfs((nz, ny, nx), 1e-3, seed=23)
    sim.set_pdfs(oracle_to_gpu(g0))
    gs = sim.get_pdfs()  # as stored
    c = lbmps.velocities().astype(np.float64)
    m0 = gs.sum()
    j0 = np.einsum("qa,q->a", c, gs.reshape(19, -1).sum(axis=1))
    k = 4
    sim.step(k)
    g = sim.get_pdfs()
    sim.close()
    m1 = g.sum()
    j1 = np.einsum("qa,q->a", c, g.reshape(19, -1).sum(axis=1))
    dj = j1 - j0 - k * N * np.array(f)
    # rounding: FP32 stores are unbiased to ~6e-8 of |g| each (random walk over
    # 19 N k values), FP64 to ~1e-16
    u = 6e-8 if precision == "fp32" else 1.2e-16
    tol = 10 * u * np.abs(g0).max() * np.sqrt(19.0 * N * k) + 1e-12
    say("  %s: mass drift %.3e, momentum drift %s (tol %.2e)" % (precision, m1 - m0, dj, tol))
    assert abs(m1 - m0) < tol
    assert np.all(np.abs(dj) < tol + 1e-9 * k * N * np.abs(f).max())


def test_full_size_many_spheres_psm_modes_agree():
    """2000 moving spheres in 512^3 (PSM-M3B2, FP32, flat 8^3 solid fractions)
    with the autotuned sweep launch: the staged mode (the default here, the
    spheres cover ~4.5 % of the cells) and the separate overlap pass give the
    same forces, torques and motion bit for bit after two rigid-body steps."""
    wl = inputs.c5_learned(0)
    L = wl["nx"]
    n_p = len(wl["D"])
    best = autotune.tune(L, L, L, "fp32")
    flags = best["sweep_flags"] & ~(lbmps.SWEEP_PSM_FUSED | lbmps.SWEEP_PSM_SEPARATE | lbmps.SWEEP_PSM_STAGED)
    res = []
    for mode in (0, lbmps.SWEEP_PSM_SEPARATE):
        say("512^3, 2000 spheres, psm mode flag", mode, "launch", best)
        cfg = lbmps.make_config(L, L, L, wl["nu"], collision="trt", coupling="psm", psm_m=3, psm_b=2, n_sub=2,
                                eps_n=8, eps_mode=lbmps.EPS_FLAT, precision="fp32", max_particles=n_p,
                                max_diameter=20.0, f_ext=wl["f_ext"], gravity=wl["gravity"],
                                tile_rows=best["tile_rows"], block_threads=best["block_threads"],
                                grid_blocks=best["grid_blocks"], sweep_flags=flags | mode)
        sim = lbmps.Sim(cfg)
        sim.init_equilibrium()
        z = [[0.0, 0.0, 0.0]] * n_p
        sim.set_particles(wl["X"], z, z, wl["D"], [wl["rho"]] * n_p, [False] * n_p)
        sim.step(4)
        res.append(sim.particles())
        sim.close()
        del sim
    a, b = res
    for k in ("F", "T", "U", "Omega", "X"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(np.isfinite(a["F"])) and np.abs(a["F"]).max() > 0
