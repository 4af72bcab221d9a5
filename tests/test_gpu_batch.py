"""Batched form on the GPU: instances advanced together in one launch equal
the same instances run alone, bit for bit; graph replay equals eager steps."""
import numpy as np
import pytest

from paper_1702_04910_amd import inputs, lbmps
from gpu_util import say

pytestmark = pytest.mark.gpu


def _cfg(d, dmax, tile_cells=256, grid=0, precision="fp32", flags=0):
    return lbmps.make_config(d["nx"], d["ny"], d["nz"], d["nu"], collision="trt", coupling=d["coupling"],
                             psm_m=d["psm_m"], psm_b=d["psm_b"], n_sub=2, eps_n=8, eps_mode=lbmps.EPS_RECURSIVE,
                             precision=precision, max_particles=1, max_diameter=dmax, f_ext=d["f_ext"],
                             gravity=d["gravity"], tile_rows=max(1, tile_cells // d["nx"]), grid_blocks=grid,
                             sweep_flags=flags)


def _setup(sim, i, d):
    sim.init_equilibrium(inst=i)
    sim.set_particles([d["X"]], [[0, 0, 0]], [[0, 0, 0]], [d["D"]], [d["rho"]], [False], inst=i)


def _small_batch(seed=3):
    out = []
    for k, (D, cp, m, b) in enumerate([(8.0, "mem_cli", 0, 0), (8.0, "psm", 3, 2), (6.0, "mem_cli", 0, 0),
                                       (6.0, "psm", 2, 2)]):
        box = (int(5 * D), int(5 * D), int(10 * D))
        d = inputs.settling_sphere(seed + k, D, box, nu=0.1 * D / 250.0, re=250.0, rho_ratio=1.5)
        d.update(coupling=cp, psm_m=m or 1, psm_b=b or 1)
        out.append(d)
    return out


@pytest.mark.parametrize("flags", [0, lbmps.SWEEP_PSM_FUSED, lbmps.SWEEP_PSM_STAGED,
                                   lbmps.SWEEP_CELL_PAIRS | lbmps.SWEEP_WG_CAP2 | lbmps.SWEEP_NT_LOADS])
def test_batched_instances_equal_solo_runs_bitwise(flags):
    insts = _small_batch()
    dmax = max(d["D"] for d in insts)
    say("batch of", len(insts), "flags", flags)
    batch = lbmps.Sim([_cfg(d, dmax, grid=512, flags=flags) for d in insts])
    for i, d in enumerate(insts):
        _setup(batch, i, d)
    batch.step(40)
    for i, d in enumerate(insts):
        say("  solo", i, d["coupling"])
        solo = lbmps.Sim(_cfg(d, dmax))
        _setup(solo, 0, d)
        solo.step(40)
        assert np.array_equal(solo.get_pdfs(), batch.get_pdfs(i))
        ps, pb = solo.particles(), batch.particles(i)
        for k in ("F", "T", "U", "Omega", "X"):
            assert np.array_equal(ps[k], pb[k]), k
        solo.close()
    batch.close()


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_batch_of_one_coupling_with_work_beside_the_sweep(coupling):
    # a batch of MEM-only (PSM-only) instances runs its remaps (list rebuilds)
    # beside the next sweep within one step call; each instance equals its
    # solo run stepped one rigid-body step per call (in order), bit for bit
    insts = [d for d in _small_batch() if d["coupling"] == coupling]
    dmax = max(d["D"] for d in insts)
    say("one-coupling batch", coupling, len(insts))
    flags = lbmps.SWEEP_PSM_SEPARATE if coupling == "psm" else 0
    batch = lbmps.Sim([_cfg(d, dmax, flags=flags) for d in insts])
    for i, d in enumerate(insts):
        _setup(batch, i, d)
    batch.step(40)
    for i, d in enumerate(insts):
        solo = lbmps.Sim(_cfg(d, dmax, flags=flags))
        _setup(solo, 0, d)
        for k in range(20):
            solo.step(2)
        assert np.array_equal(solo.get_pdfs(), batch.get_pdfs(i))
        ps, pb = solo.particles(), batch.particles(i)
        for k in ("F", "T", "U", "Omega", "X"):
            assert np.array_equal(ps[k], pb[k]), k
        solo.close()
    batch.close()


def test_graph_replay_equals_eager_steps():
    import torch

    insts = _small_batch(7)[:2]
    dmax = max(d["D"] for d in insts)
    st_e, st_g = torch.cuda.Stream(), torch.cuda.Stream()
    eager = lbmps.Sim([_cfg(d, dmax) for d in insts], stream=st_e)
    graph = lbmps.Sim([_cfg(d, dmax) for d in insts], stream=st_g)
    for i, d in enumerate(insts):
        _setup(eager, i, d)
        _setup(graph, i, d)
    for rep in range(4):
        say("  replay", rep)
        eager.step(4)
        graph.step_graph(4)
        eager.sync()
        graph.sync()
        for i in range(len(insts)):
            assert np.array_equal(eager.get_pdfs(i), graph.get_pdfs(i))
            pe, pg = eager.particles(i), graph.particles(i)
            assert np.array_equal(pe["X"], pg["X"]) and np.array_equal(pe["F"], pg["F"])
    # eager steps interleaved with replays keep agreeing
    eager.step(2)
    graph.step(2)
    eager.step(4)
    graph.step_graph(4)
    for i in range(len(insts)):
        assert np.array_equal(eager.get_pdfs(i), graph.get_pdfs(i))
    eager.close()
    graph.close()


def test_graph_needs_period_multiple():
    import torch

    insts = _small_batch(9)[:1]
    sim = lbmps.Sim([_cfg(insts[0], insts[0]["D"])], stream=torch.cuda.Stream())
    _setup(sim, 0, insts[0])
    with pytest.raises(lbmps.LbmpsError):
        sim.step_graph(3)
    sim.close()


def test_mixed_batch_instances_match_their_oracle_runs():
    # A batch of MEM-CLI, PSM-M3B2 and MEM-BB instances of different box
    # sizes, each with a moving sphere (FP64 storage): every instance against
    # its own FP64 oracle run at 1e-12 (PDFs, force, torque), positions to 1e-13.
    from oracle.sim import OracleSim
    from gpu_util import oracle_to_gpu, gpu_to_oracle

    specs = [(26, 24, 30, "mem_cli", 3, 2, [12.3, 11.6, 18.2], [0.01, -0.004, 0.0], 6.6, 1.4),
             (24, 22, 28, "psm", 3, 2, [11.4, 10.7, 15.9], [-0.006, 0.008, 0.002], 7.0, 1.5),
             (22, 26, 24, "mem_bb", 3, 2, [10.8, 13.1, 12.5], [0.0, 0.005, -0.01], 5.8, 1.25)]
    dmax = max(s[8] for s in specs)
    cfgs, oras = [], []
    for (nx, ny, nz, cp, m, b, X, U, D, rho) in specs:
        f = (1e-6, 0.0, 5e-7)
        g = (0.0, 0.0, -2e-4)
        cfgs.append(lbmps.make_config(nx, ny, nz, 0.06, collision="trt", coupling=cp, psm_m=m, psm_b=b, n_sub=2,
                                      eps_n=4, precision="fp64", max_particles=1, max_diameter=dmax, f_ext=f,
                                      gravity=g))
        o = OracleSim(nx, ny, nz, 0.06, collision="trt", coupling=cp, psm_m=m, psm_b=b, fext=f, gravity=g, n_sub=2,
                      eps_n=4)
        o.init_equilibrium()
        o.set_particles([X], [U], [[0.0, 0.001, 0.0]], [D], [rho], [False])
        oras.append(o)
    batch = lbmps.Sim(cfgs)
    for i, (nx, ny, nz, cp, m, b, X, U, D, rho) in enumerate(specs):
        batch.init_equilibrium(inst=i)
        batch.set_particles([X], [U], [[0.0, 0.001, 0.0]], [D], [rho], [False], inst=i)
    for chunk in range(3):
        batch.step(12)
        for i, o in enumerate(oras):
            o.step(12)
            go = o.get_pdfs()
            gg = gpu_to_oracle(batch.get_pdfs(i))
            fluid = o.owner == -1
            e = np.abs(gg[:, fluid] - go[:, fluid]).max() / np.abs(go[:, fluid]).max()
            po, pg = o.particles(), batch.particles(i)
            nF = np.linalg.norm(po["F"][0])
            eF = np.linalg.norm(pg["F"][0] - po["F"][0]) / nF
            eT = np.linalg.norm(pg["T"][0] - po["T"][0]) / (0.5 * specs[i][8] * nF)
            eX = np.abs(pg["X"][0] - po["X"][0]).max()
            say("  t=%d inst %d (%s): e_f=%.2e e_F=%.2e e_T=%.2e eX=%.2e" % (o.time, i, specs[i][3], e, eF, eT, eX))
            assert e < 1e-12 and eF < 1e-12 and eT < 1e-12 and eX < 1e-13
    batch.close()
