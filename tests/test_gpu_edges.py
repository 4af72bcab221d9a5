"""Edge cases of the coupled path on the GPU against the FP64 oracle: no
particles, spheres straddling the periodic faces while they move, several
MEM spheres at once, the largest sphere the library accepts, cell centres
exactly on a sphere surface, and the argument checks of set_particles."""
import numpy as np
import pytest

from paper_1702_04910_amd import lbmps
from gpu_util import make_pair, pdf_error, force_errors, say, link_set_errors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_coupling_without_particles_is_the_fluid_sweep(coupling):
    say("no particles", coupling)
    parts = dict(X=[], U=[], Om=[], D=[], rho=[], fixed=[])
    ora, sim = make_pair(20, 18, 16, 0.05, coupling=coupling, f_ext=(1e-5, 0, 0), n_sub=2)
    sim.set_particles([], [], [], [], [], [])
    ora.step(6)
    sim.step(6)
    e, _ = pdf_error(ora, sim)
    assert e < 1e-12
    sim.close()


@pytest.mark.parametrize("coupling,m,b", [("mem_cli", 1, 1), ("mem_bb", 1, 1), ("psm", 2, 2)])
def test_sphere_crossing_periodic_faces(coupling, m, b):
    # centred near a box corner, moving across the x and z faces
    say("periodic crossing", coupling)
    parts = dict(X=[[0.4, 23.7, 31.6]], U=[[-0.02, 0.01, 0.02]], Om=[[0.001, 0.0, -0.002]], D=[6.5], rho=[1.5],
                 fixed=[False])
    ora, sim = make_pair(24, 24, 32, 0.05, coupling=coupling, collision="trt", psm_m=m, psm_b=b,
                         f_ext=(1e-6, 0, 0), gravity=(0, 0, -1e-4), parts=parts, eps_n=4, n_sub=2)
    for k in range(3):
        ora.step(30)
        sim.step(30)
        errs, po, pg = force_errors(ora, sim)
        eF, eT, _ = errs[0]
        e, _ = pdf_error(ora, sim)
        eX = np.abs(pg["X"] - po["X"]).max()
        say("  t=%d X=%s e_f=%.2e e_F=%.2e e_T=%.2e" % (ora.time, pg["X"][0], e, eF, eT))
        assert e < 1e-12 and eF < 1e-12 and eT < 1e-12 and eX < 1e-13
    # it has wrapped through x = 0 and z = 32
    assert pg["X"][0][0] > 12 and pg["X"][0][2] < 12
    sim.close()


def test_several_mem_spheres():
    say("several MEM spheres")
    parts = dict(X=[[8.2, 8.7, 9.1], [22.5, 9.3, 10.0], [15.1, 22.6, 20.4]],
                 U=[[0.01, 0, 0], [0, -0.01, 0.005], [0, 0, 0]], Om=[[0, 0, 0.001], [0, 0, 0], [0.002, 0, 0]],
                 D=[7.0, 6.2, 8.4], rho=[1.5, 1.2, 2.0], fixed=[False, False, True])
    ora, sim = make_pair(30, 30, 30, 0.05, coupling="mem_cli", collision="trt", f_ext=(1e-6, 0, 0),
                         gravity=(0, 0, -2e-4), parts=parts, n_sub=2)
    for k in range(2):
        ora.step(40)
        sim.step(40)
        errs, po, pg = force_errors(ora, sim)
        e, _ = pdf_error(ora, sim)
        say("  t=%d e_f=%.2e" % (ora.time, e), [("%.1e" % a, "%.1e" % b) for a, b, _ in errs])
        assert e < 1e-12
        for eF, eT, _ in errs:
            assert eF < 1e-12 and eT < 1e-12
        assert np.abs(pg["X"] - po["X"]).max() < 1e-13
        assert link_set_errors(ora, sim) <= 1e-15
    sim.close()


def test_mem_cli_falls_back_to_bounce_back_in_narrow_gaps():
    # Two spheres one fluid cell apart along x, and a fixed sphere one fluid
    # cell above a static wall: fluid cells with a solid cell on both sides of
    # a link, where CLI takes the bounce-back rule for that link.
    say("MEM-CLI narrow gaps")
    nx, ny, nz = 30, 24, 24
    wall = np.zeros((nz, ny, nx), bool)
    wall[0] = True
    parts = dict(X=[[10.5, 12.3, 11.7], [18.9, 12.1, 11.9], [5.0, 5.0, 5.2]],
                 U=[[0.002, 0, 0], [-0.002, 0.001, 0], [0, 0, 0]], Om=[[0, 0, 0.001], [0, 0, 0], [0, 0, 0]],
                 D=[7.0, 7.0, 6.0], rho=[1.5, 1.2, 2.0], fixed=[False, False, True])
    ora, sim = make_pair(nx, ny, nz, 0.05, coupling="mem_cli", collision="trt", f_ext=(1e-6, 0, 0),
                         gravity=(0, 0, -1e-5), parts=parts, n_sub=2, walls=[(wall, (0, 0, 0))])
    L = ora.links
    fallback = L["is_particle"] & ~L["cli_ok"]
    say("  particle links %d, of them with x - c_q solid: %d" % (int(L["is_particle"].sum()), int(fallback.sum())))
    assert fallback.sum() >= 2  # the case is exercised
    for k in range(3):
        ora.step(20)
        sim.step(20)
        errs, po, pg = force_errors(ora, sim)
        e, _ = pdf_error(ora, sim)
        say("  t=%d e_f=%.2e" % (ora.time, e), [("%.1e" % a, "%.1e" % b) for a, b, _ in errs])
        assert e < 1e-12
        for eF, eT, _ in errs:
            assert eF < 1e-12 and eT < 1e-12
        assert np.abs(pg["X"] - po["X"]).max() < 1e-13
    sim.close()


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_largest_sphere(coupling):
    # D = 58: bounding boxes of 64 cells per axis, the library's limit
    say("largest sphere", coupling)
    parts = dict(X=[[32.3, 31.8, 33.1]], U=[[0, 0, 0]], Om=[[0, 0, 0]], D=[58.0], rho=[1.5], fixed=[True])
    ora, sim = make_pair(66, 64, 68, 0.1, coupling=coupling, collision="trt", psm_m=3, psm_b=2,
                         f_ext=(1e-6, 0, 0), parts=parts, eps_n=2, n_sub=2)
    ora.step(4)
    sim.step(4)
    (eF, eT, _), = force_errors(ora, sim)[0]
    e, _ = pdf_error(ora, sim)
    say("  e_f=%.2e e_F=%.2e e_T=%.2e" % (e, eF, eT))
    assert e < 1e-12 and eF < 1e-12 and eT < 1e-12
    sim.close()


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_cell_centres_on_the_surface(coupling):
    # X at a cell centre and an integer radius: the cell centres at distance
    # exactly R are inside (the <= convention), the same on both sides
    say("centres on the surface", coupling)
    parts = dict(X=[[12.5, 12.5, 12.5]], U=[[0, 0, 0]], Om=[[0, 0, 0]], D=[8.0], rho=[1.5], fixed=[True])
    ora, sim = make_pair(25, 25, 25, 0.05, coupling=coupling, collision="trt", psm_m=1, psm_b=1,
                         f_ext=(1e-6, 2e-6, 0), parts=parts, eps_n=4, n_sub=2)
    if coupling == "mem_cli":
        assert link_set_errors(ora, sim) <= 1e-15
    ora.step(10)
    sim.step(10)
    (eF, eT, _), = force_errors(ora, sim)[0]
    e, _ = pdf_error(ora, sim)
    assert e < 1e-12 and eF < 1e-12 and eT < 1e-12
    sim.close()


def test_set_particles_argument_checks():
    cfg = lbmps.make_config(20, 20, 20, 0.05, coupling="mem_cli", max_particles=2, max_diameter=6.0)
    sim = lbmps.Sim(cfg)
    ok = dict(X=[[10, 10, 10]], U=[[0, 0, 0]], Om=[[0, 0, 0]], D=[5.0], rho=[1.5], fixed=[False])

    def call(**kw):
        a = dict(ok, **kw)
        sim.set_particles(a["X"], a["U"], a["Om"], a["D"], a["rho"], a["fixed"])

    call()
    for bad in (dict(D=[7.0]), dict(D=[0.0]), dict(rho=[0.0]), dict(X=[[np.nan, 1, 1]]), dict(U=[[np.inf, 0, 0]])):
        with pytest.raises(lbmps.LbmpsError) as ei:
            call(**bad)
        assert ei.value.status == -1
    with pytest.raises(lbmps.LbmpsError):  # more than max_particles
        sim.set_particles([[5, 5, 5]] * 3, [[0, 0, 0]] * 3, [[0, 0, 0]] * 3, [4.0] * 3, [1.5] * 3, [False] * 3)
    with pytest.raises(lbmps.LbmpsError):  # steps must be a multiple of n_sub (2 for MEM)
        sim.step(3)
    call()  # still usable after rejected calls
    sim.step(2)
    sim.sync()
    sim.close()


def test_sampled_sweep_timing():
    # every third sweep launch is timed; a negative stride is rejected
    cfg = lbmps.make_config(32, 24, 16, 0.05)
    sim = lbmps.Sim(cfg)
    sim.init_equilibrium()
    sim.set_timing(True, 3)
    sim.step(10)
    ms, n = sim.timing()
    assert n == 4 and ms > 0  # launches 0, 3, 6, 9
    with pytest.raises(lbmps.LbmpsError):
        sim.set_timing(True, -2)
    sim.set_timing(True)
    sim.step(5)
    assert sim.timing()[1] == 5
    sim.set_timing(False)
    sim.close()


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_unstable_rigid_step_is_reported_and_not_taken(coupling):
    # A sphere set moving at two cells per sweep: its first rigid-body step
    # (two sweeps) would move it by four cells.  The library reports
    # LBMPS_EUNSTABLE and leaves the sphere where it was, so every index
    # derived from its position stays inside the box.
    say("unstable rigid step", coupling)
    cfg = lbmps.make_config(24, 24, 24, 0.05, coupling=coupling, psm_m=2, psm_b=2, n_sub=2, eps_n=4,
                            max_particles=1, max_diameter=6.0)
    sim = lbmps.Sim(cfg)
    sim.init_equilibrium()
    X = [11.3, 12.2, 12.7]
    sim.set_particles([X], [[2.0, 0.0, 0.0]], [[0, 0, 0]], [6.0], [1.5], [False])
    sim.step(2)
    with pytest.raises(lbmps.LbmpsError) as ei:
        sim.sync()
    assert ei.value.status == -4
    with pytest.raises(lbmps.LbmpsError):  # the flag stays set
        sim.particles()
    sim.close()

