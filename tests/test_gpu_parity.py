"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances (relative, see the metric helpers):
FP64 storage 1e-12, FP32 storage 1e-5."""
import numpy as np
import pytest

from paper_1702_04910_amd import inputs
from gpu_util import make_pair, pdf_error, force_errors, say, gpu_to_oracle, link_set_errors, overlap_set_check

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("collision", ["trt", "bgk"])
def test_fluid_sweep_ragged_box(precision, collision):
    # ragged box (not a multiple of any tile), random state, body force
    nx, ny, nz = 37, 23, 19
    g0 = inputs.random_pdfs((nz, ny, nx), 1e-3, seed=5)
    say("fluid", precision, collision)
    ora, sim = make_pair(nx, ny, nz, 0.07, collision=collision, f_ext=(1e-5, -2e-5, 3e-5), precision=precision, g0=g0)
    ora.step(10)
    sim.step(10)
    e, _ = pdf_error(ora, sim)
    say("  e_f =", e)
    assert e < TOL[precision]


@pytest.mark.parametrize("tile_rows,block,grid", [(1, 64, 0), (3, 128, 0), (0, 256, 7)])
def test_fluid_sweep_launch_shapes(tile_rows, block, grid):
    nx, ny, nz = 40, 12, 9
    g0 = inputs.random_pdfs((nz, ny, nx), 1e-3, seed=6)
    say("launch", tile_rows, block, grid)
    ora, sim = make_pair(nx, ny, nz, 0.05, f_ext=(1e-5, 0, 0), g0=g0, tile_rows=tile_rows, block_threads=block,
                         grid_blocks=grid)
    ora.step(4)
    sim.step(4)
    e, _ = pdf_error(ora, sim)
    assert e < 1e-12


def _c1_parts(seed=0):
    c = inputs.c1_plain(seed)
    return c, dict(X=[c["X"]], U=[[0, 0, 0]], Om=[[0, 0, 0]], D=[c["D"]], rho=[1.5], fixed=[True])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nu", [0.01, 0.1])
def test_c1_psm_m1b1_trt(precision, nu):
    c, parts = _c1_parts(0)
    say("c1 PSM M1B1 TRT", precision, nu)
    ora, sim = make_pair(c["nx"], c["ny"], c["nz"], nu, coupling="psm", collision="trt", psm_m=1, psm_b=1,
                         f_ext=c["f_ext"], precision=precision, eps_n=8, parts=parts)
    # overlap list is a discrete event: compare exactly
    ov = sim.overlaps()
    iz, iy, ix, eps = ora.overlaps[0]
    cells_o = (iz * c["ny"] + iy) * c["nx"] + ix
    order = np.argsort(ov["cell"])
    assert np.array_equal(np.sort(cells_o), ov["cell"][order])
    assert np.array_equal(eps[np.argsort(cells_o)], ov["eps"][order])
    for k in range(4):
        ora.step(25)
        sim.step(25)
        (eF, eT, nF), = force_errors(ora, sim)[0]
        e, _ = pdf_error(ora, sim)
        say("  t=%d e_f=%.3e e_F=%.3e e_T=%.3e |F|=%.3e" % (ora.time, e, eF, eT, nF))
        assert e < TOL[precision] and eF < TOL[precision] and eT < TOL[precision]


@pytest.mark.parametrize("m,b,collision", [(2, 2, "trt"), (3, 2, "trt"), (1, 1, "bgk"), (3, 2, "bgk")])
def test_c1_psm_variants(m, b, collision):
    c, parts = _c1_parts(1)
    say("c1 PSM", m, b, collision)
    ora, sim = make_pair(c["nx"], c["ny"], c["nz"], 1.0 / 30.0, coupling="psm", collision=collision, psm_m=m, psm_b=b,
                         f_ext=c["f_ext"], parts=parts)
    ora.step(30)
    sim.step(30)
    (eF, eT, nF), = force_errors(ora, sim)[0]
    e, _ = pdf_error(ora, sim)
    say("  e_f=%.3e e_F=%.3e e_T=%.3e" % (e, eF, eT))
    assert e < 1e-12 and eF < 1e-12 and eT < 1e-12
    # Eq. MacVel_PSM fields
    ro, uo = ora.fields()
    rg, ug = sim.fields()
    assert np.abs(ug - uo).max() < 1e-12 * np.abs(uo).max()
    assert np.abs(rg - ro).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("coupling", ["mem_bb", "mem_cli"])
def test_c1_box_mem_fixed_sphere(precision, coupling):
    c, parts = _c1_parts(2)
    say("c1 MEM", coupling, precision)
    ora, sim = make_pair(c["nx"], c["ny"], c["nz"], 0.1, coupling=coupling, collision="trt", f_ext=c["f_ext"],
                         precision=precision, parts=parts)
    ed = link_set_errors(ora, sim)
    say("  links %d, max |delta error| %.1e" % (len(ora.links["q"]), ed))
    assert ed <= 1e-15
    for k in range(2):
        ora.step(50)
        sim.step(50)
        (eF, eT, nF), = force_errors(ora, sim)[0]
        e, _ = pdf_error(ora, sim)
        say("  t=%d e_f=%.3e e_F=%.3e e_T=%.3e |F|=%.3e" % (ora.time, e, eF, eT, nF))
        assert e < TOL[precision] and eF < TOL[precision] and eT < TOL[precision]


def _velocity_and_path_errors(po, pg, X0):
    """Relative sphere-velocity error and position error per unit path length."""
    eU = np.linalg.norm(pg["U"][0] - po["U"][0]) / np.linalg.norm(po["U"][0])
    eX = np.abs(pg["X"] - po["X"]).max() / max(1.0, float(np.linalg.norm(po["X"][0] - X0)))
    return eU, eX


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("coupling", ["mem_bb", "mem_cli"])
def test_moving_mem_sphere_with_refill(coupling, precision):
    # a sphere pushed through the box: cells are uncovered (refill) and covered;
    # the link set is compared exactly and delta_q to 1e-15 after every chunk
    # (the remap of the last rigid-body step); FP32 storage is the timed path
    # (there the positions differ at the force tolerance, and delta with them)
    say("moving MEM", coupling, precision)
    X0 = np.array([16.3, 15.8, 20.2])
    parts = dict(X=[X0], U=[[0.01, -0.005, 0.0]], Om=[[0.0, 0.001, 0.0]], D=[7.0], rho=[1.5], fixed=[False])
    ora, sim = make_pair(32, 32, 40, 0.05, coupling=coupling, collision="trt", f_ext=(0, 0, 1e-6),
                         gravity=(0, 0, -1e-3), parts=parts, precision=precision)
    tol = TOL[precision]
    for k in range(5):
        ora.step(40)
        sim.step(40)
        errs, po, pg = force_errors(ora, sim)
        eF, eT, nF = errs[0]
        e, _ = pdf_error(ora, sim)
        eU, eX = _velocity_and_path_errors(po, pg, X0)
        ed = link_set_errors(ora, sim)
        say("  t=%d refilled=%d links=%d e_f=%.3e e_F=%.3e e_T=%.3e e_U=%.3e eX=%.3e e_delta=%.1e"
            % (ora.time, ora.refilled, int((ora.links["p"] >= 0).sum()), e, eF, eT, eU, eX, ed))
        assert e < tol and eF < tol and eT < tol and eU < tol
        assert eX < (1e-13 if precision == "fp64" else tol)
        assert ed <= (1e-15 if precision == "fp64" else 1e-5)
    assert ora.refilled > 20


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_moving_mem_sphere_with_equilibrium_refill(precision):
    # the equilibrium reconstruction of uncovered cells (every cell takes the
    # last fallback of Sec. 2.2.3) against the oracle's
    say("moving MEM, equilibrium refill", precision)
    X0 = np.array([16.3, 15.8, 20.2])
    parts = dict(X=[X0], U=[[0.01, -0.005, 0.0]], Om=[[0.0, 0.001, 0.0]], D=[7.0], rho=[1.5], fixed=[False])
    ora, sim = make_pair(32, 32, 40, 0.05, coupling="mem_cli", collision="trt", f_ext=(0, 0, 1e-6),
                         gravity=(0, 0, -1e-3), parts=parts, precision=precision, refill="equilibrium")
    tol = TOL[precision]
    for k in range(3):
        ora.step(40)
        sim.step(40)
        errs, po, pg = force_errors(ora, sim)
        eF, eT, nF = errs[0]
        e, _ = pdf_error(ora, sim)
        say("  t=%d refilled=%d e_f=%.3e e_F=%.3e e_T=%.3e" % (ora.time, ora.refilled, e, eF, eT))
        assert e < tol and eF < tol and eT < tol
        assert link_set_errors(ora, sim) <= (1e-15 if precision == "fp64" else 1e-5)
    assert ora.refilled > 10


@pytest.mark.parametrize("coupling,precision", [("mem_cli", "fp64"), ("mem_cli", "fp32"), ("mem_cli", "fp16"),
                                                ("mem_cli", "bf16"), ("psm", "fp64"), ("psm", "fp16"),
                                                ("psm_staged", "fp64"), ("psm_staged", "fp32")])
def test_overlapped_remap_is_bitwise_identical(coupling, precision):
    # Within one step call the MEM remap (then the refilled cells are
    # re-swept) or the PSM list rebuild (the sweep beside it leaves every
    # overlapped cell to the overlap kernel, also when staged values are
    # configured) runs beside the next sweep; one rigid-body step per call
    # runs it in order.  Both give the same bits.
    from paper_1702_04910_amd import lbmps

    say("overlapped remap", coupling, precision)
    parts = dict(X=[[10.3, 11.8, 12.2], [20.4, 12.6, 11.1]], U=[[0.04, -0.02, 0.03], [-0.03, 0.01, 0.02]],
                 Om=[[0.0, 0.002, 0.0], [0.001, 0.0, 0.0]], D=[7.0, 6.3], rho=[1.5, 1.3], fixed=[False, False])
    flags = {"psm": lbmps.SWEEP_PSM_SEPARATE, "psm_staged": lbmps.SWEEP_PSM_STAGED}.get(coupling, 0)
    coupling = coupling.split("_staged")[0]
    runs = []
    for per_call in (2, 24):
        ora, sim = make_pair(30, 24, 24, 0.05, coupling=coupling, collision="trt", psm_m=3, psm_b=2,
                             f_ext=(1e-6, 0, 0), gravity=(0, 0, -1e-4), parts=parts, n_sub=2, eps_n=4,
                             precision=precision, sweep_flags=flags)
        for k in range(24 // per_call):
            sim.step(per_call)
        runs.append((sim.get_pdfs(), sim.particles()))
        if precision == "fp64" and per_call == 24:
            ora.step(24)
            e, _ = pdf_error(ora, sim)
            say("  oracle: refilled=%d e_f=%.2e" % (ora.refilled, e))
            assert e < 1e-12
            if coupling == "mem_cli":
                assert ora.refilled > 10
        sim.close()
    (ga, pa), (gb, pb) = runs
    assert np.array_equal(ga, gb)
    for key in ("X", "U", "Omega", "F", "T"):
        assert np.array_equal(pa[key], pb[key]), key


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("m,b,n_sub", [(1, 1, 1), (2, 2, 1), (3, 2, 2)])
def test_moving_psm_sphere(m, b, n_sub, precision):
    # overlap lists compared exactly after every chunk (FP64; with FP32
    # storage the positions differ at the force tolerance, which may move a
    # sample point across the surface, so only the forces are compared)
    say("moving PSM", m, b, n_sub, precision)
    X0 = np.array([16.3, 15.8, 20.2])
    parts = dict(X=[X0], U=[[0.01, -0.005, 0.0]], Om=[[0.0, 0.001, 0.0]], D=[7.0], rho=[1.5], fixed=[False])
    ora, sim = make_pair(32, 32, 40, 0.05, coupling="psm", collision="bgk", psm_m=m, psm_b=b, f_ext=(0, 0, 1e-6),
                         gravity=(0, 0, -1e-3), parts=parts, eps_n=4, n_sub=n_sub, precision=precision)
    tol = TOL[precision]
    for k in range(4):
        ora.step(26)
        sim.step(26)
        errs, po, pg = force_errors(ora, sim)
        eF, eT, nF = errs[0]
        e, _ = pdf_error(ora, sim)
        eU, eX = _velocity_and_path_errors(po, pg, X0)
        say("  t=%d e_f=%.3e e_F=%.3e e_T=%.3e e_U=%.3e eX=%.3e" % (ora.time, e, eF, eT, eU, eX))
        assert e < tol and eF < tol and eT < tol and eU < tol
        assert eX < (1e-13 if precision == "fp64" else tol)
        if precision == "fp64":
            overlap_set_check(ora, sim)


def test_psm_two_particles_sharing_cells():
    # two spheres closer than a cell: cells overlapped by both (weights normalised)
    say("PSM shared cells")
    parts = dict(X=[[10.2, 12.1, 12.3], [17.4, 12.6, 12.0]], U=[[0, 0, 0], [0, 0, 0]], Om=[[0, 0, 0], [0, 0, 0]],
                 D=[7.0, 6.5], rho=[1.5, 1.5], fixed=[True, True])
    ora, sim = make_pair(28, 24, 24, 0.05, coupling="psm", collision="trt", psm_m=3, psm_b=2,
                         f_ext=(1e-5, 0, 0), parts=parts, eps_n=8)
    ora.step(20)
    sim.step(20)
    errs, po, pg = force_errors(ora, sim)
    e, _ = pdf_error(ora, sim)
    say("  e_f=%.3e" % e, errs)
    assert e < 1e-12
    for eF, eT, _ in errs:
        assert eF < 1e-12 and eT < 1e-12


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [4, 16])
def test_overlap_fractions_exact(mode, n):
    say("overlaps", mode, n)
    rng = np.random.default_rng(11)
    X = rng.uniform(9, 11, 3)
    parts = dict(X=[X], U=[[0, 0, 0]], Om=[[0, 0, 0]], D=[9.3], rho=[1.5], fixed=[True])
    ora, sim = make_pair(21, 22, 23, 0.05, coupling="psm", parts=parts, eps_n=n, eps_mode=mode)
    ov = sim.overlaps()
    iz, iy, ix, eps = ora.overlaps[0]
    cells_o = (iz * 22 + iy) * 21 + ix
    o1, o2 = np.argsort(cells_o), np.argsort(ov["cell"])
    assert np.array_equal(cells_o[o1], ov["cell"][o2])
    assert np.array_equal(eps[o1], ov["eps"][o2])


def test_poiseuille_walls_on_gpu():
    say("walls")
    H = 10
    nz = H + 2
    bottom = np.zeros((nz, 2, 4), bool)
    bottom[0] = True
    top = np.zeros((nz, 2, 4), bool)
    top[-1] = True
    ora, sim = make_pair(4, 2, nz, 0.1, collision="trt", f_ext=(1e-6, 0, 0),
                         walls=[(bottom, (0, 0, 0)), (top, (1e-3, 0, 0))])
    ora.step(200)
    sim.step(200)
    e, _ = pdf_error(ora, sim)
    assert e < 1e-12


@pytest.mark.parametrize("m,b,precision", [(3, 2, "fp64"), (1, 1, "fp64"), (2, 2, "fp16"), (3, 2, "bf16")])
def test_psm_collision_modes_agree_bitwise(m, b, precision):
    # the same moving case with PSM cells collided inside the sweep, in the
    # overlap pass after the sweep and staged by the overlap pass before it:
    # identical bits, and (FP64) all on the oracle
    from paper_1702_04910_amd import lbmps

    parts = dict(X=[[10.2, 12.1, 12.3], [17.4, 12.6, 12.0]], U=[[0.01, 0, 0], [-0.005, 0.004, 0]],
                 Om=[[0, 0, 0.001], [0, 0, 0]], D=[7.0, 6.5], rho=[1.5, 1.3], fixed=[False, False])
    sims = []
    names = {lbmps.SWEEP_PSM_FUSED: "inside sweep", lbmps.SWEEP_PSM_SEPARATE: "separate pass",
             lbmps.SWEEP_PSM_STAGED: "staged"}
    for flags in (lbmps.SWEEP_PSM_FUSED, lbmps.SWEEP_PSM_SEPARATE, lbmps.SWEEP_PSM_STAGED):
        say("PSM", names[flags], m, b)
        ora, sim = make_pair(28, 24, 24, 0.05, coupling="psm", collision="trt", psm_m=m, psm_b=b,
                             f_ext=(1e-5, 0, 0), gravity=(0, 0, -1e-4), parts=parts, eps_n=4, n_sub=2,
                             sweep_flags=flags, precision=precision)
        sim.step(24)
        if precision == "fp64":
            ora.step(24)
            errs, po, pg = force_errors(ora, sim)
            e, _ = pdf_error(ora, sim)
            assert e < 1e-12
            for eF, eT, _ in errs:
                assert eF < 1e-12 and eT < 1e-12
        sims.append(sim)
    a = sims[0]
    pa = a.particles()
    for b_ in sims[1:]:
        assert np.array_equal(a.get_pdfs(), b_.get_pdfs())
        pb = b_.particles()
        for k in ("F", "T", "U", "X"):
            assert np.array_equal(pa[k], pb[k])


@pytest.mark.parametrize("mode", [3, 4])  # edge intersection, surface distance
def test_closed_form_estimators(mode):
    say("estimator", mode)
    parts = dict(X=[[10.3, 11.2, 10.9]], U=[[0.01, 0, -0.005]], Om=[[0, 0.001, 0]], D=[9.3], rho=[1.5],
                 fixed=[False])
    ora, sim = make_pair(24, 22, 26, 0.05, coupling="psm", collision="trt", psm_m=2, psm_b=2, f_ext=(1e-5, 0, 0),
                         parts=parts, eps_n=16, eps_mode=mode, n_sub=2)
    ov = sim.overlaps()
    iz, iy, ix, eps = ora.overlaps[0]
    cells_o = (iz * 22 + iy) * 24 + ix
    o1, o2 = np.argsort(cells_o), np.argsort(ov["cell"])
    assert np.array_equal(cells_o[o1], ov["cell"][o2])
    assert np.array_equal(eps[o1], ov["eps"][o2])
    for k in range(2):
        ora.step(20)
        sim.step(20)
        (eF, eT, _), = force_errors(ora, sim)[0]
        e, _ = pdf_error(ora, sim)
        say("  t=%d e_f=%.2e e_F=%.2e e_T=%.2e" % (ora.time, e, eF, eT))
        assert e < 1e-12 and eF < 1e-12 and eT < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_sweep_launch_variants_are_bitwise_identical(precision):
    from paper_1702_04910_amd import lbmps

    nx, ny, nz = 37, 23, 19
    g0 = inputs.random_pdfs((nz, ny, nx), 1e-3, seed=25)
    out = []
    # and the caps on resident workgroups per CU (LDS reservation only)
    for flags in (0, lbmps.SWEEP_OCC6, lbmps.SWEEP_OCC6 | lbmps.SWEEP_NT_LOADS, lbmps.SWEEP_WG_CAP3,
                  lbmps.SWEEP_WG_CAP2 | lbmps.SWEEP_NT_LOADS):
        ora, sim = make_pair(nx, ny, nz, 0.07, collision="trt", f_ext=(1e-5, -2e-5, 3e-5), precision=precision,
                             g0=g0, sweep_flags=flags)
        sim.step(6)
        out.append(sim.get_pdfs())
        sim.close()
    for o in out[1:]:
        assert np.array_equal(out[0], o)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_cell_quad_sweep_is_bitwise_identical(precision):
    # four x-adjacent cells per thread (nx a multiple of 4, several 8-byte
    # words per row and the periodic wrap of the staged words), tiles of one
    # and of several rows, with a moving MEM sphere on top of the sweep
    from paper_1702_04910_amd import lbmps

    nx, ny, nz = 44, 23, 21
    parts = dict(X=[[20.3, 11.8, 10.1]], U=[[0.01, -0.004, 0.006]], Om=[[0.0, 0.001, 0.0]], D=[7.4], rho=[1.5],
                 fixed=[False])
    out = []
    Q4 = lbmps.SWEEP_CELL_QUADS
    for rows, flags in ((1, 0), (1, Q4), (3, Q4 | lbmps.SWEEP_NT_LOADS | lbmps.SWEEP_WG_CAP2), (5, Q4)):
        say("cell quads", precision, rows, flags)
        ora, sim = make_pair(nx, ny, nz, 0.05, coupling="mem_cli", collision="trt", f_ext=(1e-5, 0, 2e-6),
                             gravity=(0, 0, -1e-4), parts=parts, precision=precision, n_sub=2, sweep_flags=flags,
                             tile_rows=rows)
        sim.step(8)
        out.append((sim.get_pdfs(), sim.particles()))
        sim.close()
    for g, p in out[1:]:
        assert np.array_equal(out[0][0], g)
        for k in ("F", "T", "U", "X"):
            assert np.array_equal(out[0][1][k], p[k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
def test_cell_pair_sweep_is_bitwise_identical(precision):
    # two x-adjacent cells per thread (even nx), with a moving MEM sphere so
    # that links and refill run on top of the sweep; the FP64 run is also
    # checked against the oracle
    from paper_1702_04910_amd import lbmps

    nx, ny, nz = 38, 23, 21
    parts = dict(X=[[17.3, 11.8, 10.1]], U=[[0.01, -0.004, 0.006]], Om=[[0.0, 0.001, 0.0]], D=[7.4], rho=[1.5],
                 fixed=[False])
    out = []
    for flags in (0, lbmps.SWEEP_CELL_PAIRS, lbmps.SWEEP_CELL_PAIRS | lbmps.SWEEP_NT_LOADS | lbmps.SWEEP_WG_CAP2):
        say("cell pairs", precision, flags)
        ora, sim = make_pair(nx, ny, nz, 0.05, coupling="mem_cli", collision="trt", f_ext=(1e-5, 0, 2e-6),
                             gravity=(0, 0, -1e-4), parts=parts, precision=precision, n_sub=2, sweep_flags=flags)
        sim.step(8)
        if precision == "fp64":
            ora.step(8)
            e, _ = pdf_error(ora, sim)
            assert e < 1e-12
        out.append((sim.get_pdfs(), sim.particles()))
        sim.close()
    for g, p in out[1:]:
        assert np.array_equal(out[0][0], g)
        for k in ("F", "T", "U", "X"):
            assert np.array_equal(out[0][1][k], p[k]), k
