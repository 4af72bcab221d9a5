"""Workload for hardware-counter runs of the sweep kernel (run it under
``rocprofv3 --pmc FETCH_SIZE`` and again under ``--pmc WRITE_SIZE``).

It launches, in this order:
  * a plain device-to-device copy of COPY_BYTES (torch's copy kernel), five
    times: the calibration of the counters (bytes read and written are known);
  * the sweep kernel of the primary workload (settling sphere D = 24 in a
    192x192x384 periodic box, MEM-CLI, FP32 deviation storage unless
    --precision says otherwise, autotuned launch shape), SWEEPS times after a
    short warm-up.

The per-dispatch counter values of both kernels, and the source hash that
names the sweep kernel they were taken on, go into the text summary under
profiles/ that the benchmark reads (its ``traffic`` field).

    python -m paper_1702_04910_amd.counters [--shape ROWS,BLOCK,GRID,FLAGS]

Without --shape the launch shape comes from the autotuner (which launches
its own timing sweeps first).
"""
import hashlib
import os
import sys

COPY_BYTES = 1 << 30
SWEEPS = 20

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_SOURCES = ("csrc/sweep.hip", "csrc/common.h", "csrc/psm_cell.h", "csrc/kernels.h")


def sweep_source_hash():
    """SHA-256 over the sources of the sweep kernel (counter values are void
    once they change)."""
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main(argv=None):
    import argparse

    import torch

    from . import inputs, lbmps
    from .autotune import tune

    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()

    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", default=None, help="tile_rows,block_threads,grid_blocks,sweep_flags")
    ap.add_argument("--precision", default="fp32", choices=("fp64", "fp32", "fp16", "bf16"),
                    help="storage precision of the primary workload's sweep")
    ap.add_argument("--workload", default="primary", choices=("primary", "spheres"),
                    help="spheres: 2000 moving spheres in 512^3, PSM-M3B2, flat 8^3 solid fractions")
    args = ap.parse_args(argv)
    if args.workload == "spheres":
        return spheres(args)
    inp = inputs.c2_scale(0)
    keys = ("tile_rows", "block_threads", "grid_blocks", "sweep_flags")
    if args.shape:
        shape = dict(zip(keys, (int(v) for v in args.shape.split(","))))
    else:
        best = tune(inp["nx"], inp["ny"], inp["nz"], args.precision)
        shape = {k: best[k] for k in keys}
    cfg = lbmps.make_config(inp["nx"], inp["ny"], inp["nz"], inp["nu"], collision="trt", coupling="mem_cli",
                            n_sub=2, precision=args.precision, max_particles=1, max_diameter=inp["D"], f_ext=inp["f_ext"],
                            gravity=inp["gravity"], **shape)
    sim = lbmps.Sim(cfg)
    sim.init_equilibrium()
    sim.set_particles([inp["X"]], [[0, 0, 0]], [[0, 0, 0]], [inp["D"]], [inp["rho"]], [False])
    sim.step(4)
    sim.step(SWEEPS)
    sim.sync()
    sim.close()
    print("counters workload done: copy %d B x5, %d sweeps of %dx%dx%d %s, shape %s, sweep source %s"
          % (COPY_BYTES, SWEEPS, inp["nx"], inp["ny"], inp["nz"], args.precision, shape, sweep_source_hash()),
          flush=True)
    return 0


def spheres(args):
    """The learned-solid-fraction workload with exact (flat 8^3) solid
    fractions: 4 sweeps after 2 warm-up sweeps (PSM collide, overlap rebuilds)."""
    from . import inputs, lbmps

    wl = inputs.c5_learned(0)
    L, n = wl["nx"], len(wl["D"])
    keys = ("tile_rows", "block_threads", "grid_blocks", "sweep_flags")
    shape = dict(zip(keys, (int(v) for v in (args.shape or "1,256,0,1").split(","))))
    cfg = lbmps.make_config(L, L, L, wl["nu"], collision="trt", coupling="psm", psm_m=3, psm_b=2, n_sub=2, eps_n=8,
                            eps_mode=lbmps.EPS_FLAT, precision="fp32", max_particles=n, max_diameter=20.0,
                            f_ext=wl["f_ext"], gravity=wl["gravity"], **shape)
    sim = lbmps.Sim(cfg)
    sim.init_equilibrium()
    z = [[0.0, 0.0, 0.0]] * n
    sim.set_particles(wl["X"], z, z, wl["D"], [wl["rho"]] * n, [False] * n)
    sim.step(2)
    sim.step(4)
    sim.sync()
    ov = sim.overlaps()
    sim.close()
    import numpy as np

    cells, per_cell = np.unique(ov["cell"], return_counts=True)
    print("counters workload done: %d spheres in %d^3, PSM-M3B2 flat 8^3, 6 sweeps, shape %s; %d particle-cell "
          "pairs, %d overlapped cells (%d shared)" % (n, L, shape, len(ov["cell"]), len(cells),
                                                       int((per_cell > 1).sum())), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
