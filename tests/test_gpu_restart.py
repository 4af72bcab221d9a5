"""Checkpoint and restart through the C-ABI, and graph replay of the
coupled step with moving particles (including the learned solid fraction,
whose network inference is captured with the rebuild)."""
import numpy as np
import pytest

from paper_1702_04910_amd import inputs, lbmps
from gpu_util import say

pytestmark = pytest.mark.gpu


def _cfg(coupling, **kw):
    base = dict(collision="trt", coupling=coupling, psm_m=3, psm_b=2, n_sub=2, eps_n=8, precision="fp32",
                max_particles=2, max_diameter=8.0, f_ext=(1e-6, 0, 0), gravity=(0, 0, -5e-4))
    base.update(kw)
    return lbmps.make_config(40, 36, 48, 0.05, **base)


PARTS = dict(X=[[12.3, 17.2, 30.1], [27.6, 18.4, 20.3]], U=[[0.004, 0, 0], [0, 0.003, -0.002]],
             Om=[[0, 0, 0.001], [0.001, 0, 0]], D=[7.5, 6.8], rho=[1.5, 1.3], fixed=[False, False])


def _start(sim):
    sim.init_equilibrium()
    p = PARTS
    sim.set_particles(p["X"], p["U"], p["Om"], p["D"], p["rho"], p["fixed"])


@pytest.mark.parametrize("coupling", ["mem_cli", "psm"])
def test_checkpoint_restart_continues_bitwise(coupling):
    say("restart", coupling)
    a = lbmps.Sim(_cfg(coupling))
    _start(a)
    a.step(30)
    g = a.get_pdfs()
    st = a.particles()
    a.step(30)
    want_g, want_p = a.get_pdfs(), a.particles()
    a.close()
    # restore into a fresh context: PDFs, then the particle state at the same
    # rigid-body step boundary (positions, velocities)
    b = lbmps.Sim(_cfg(coupling))
    b.set_pdfs(g)
    b.set_particles(st["X"], st["U"], st["Omega"], PARTS["D"], PARTS["rho"], PARTS["fixed"])
    b.step(30)
    assert np.array_equal(b.get_pdfs(), want_g)
    pb = b.particles()
    for k in ("X", "U", "Omega", "F", "T"):
        assert np.array_equal(pb[k], want_p[k]), k
    b.close()


@pytest.mark.parametrize("mode", ["psm_flat", "psm_learned", "mem_cli"])
def test_graph_replay_moving_particles(mode):
    import torch

    say("graph replay", mode)
    coupling = "mem_cli" if mode == "mem_cli" else "psm"
    kw = dict(eps_mode=lbmps.EPS_LEARNED, eps_n=16) if mode == "psm_learned" else {}
    sims = [lbmps.Sim(_cfg(coupling, **kw), stream=torch.cuda.Stream()) for _ in range(2)]
    params = None
    if mode == "psm_learned":  # a quickly trained network for R in [3, 4.2]
        n = 32768
        m = lbmps.Mlp(n)
        m.set_samples(inputs.eps_training_cells(5, n, r_min=3.0, r_max=4.2))
        m.set_params(inputs.mlp_init(5))
        m.label(16)
        mult, add = inputs.affine_orders(5, n, 8)
        m.train(mult, add, batch=512, lr=2e-3)
        params = m.params()
        m.close()
    for s in sims:
        s.init_equilibrium()
        if params is not None:
            s.set_eps_model(params, 3.0, 4.2)
        p = PARTS
        s.set_particles(p["X"], p["U"], p["Om"], p["D"], p["rho"], p["fixed"])
    eager, graph = sims
    for rep in range(3):
        eager.step(8)
        graph.step_graph(8)
        eager.sync()
        graph.sync()
        assert np.array_equal(eager.get_pdfs(), graph.get_pdfs())
        pe, pg = eager.particles(), graph.particles()
        for k in ("X", "U", "F"):
            assert np.array_equal(pe[k], pg[k]), (rep, k)
    for s in sims:
        s.close()
