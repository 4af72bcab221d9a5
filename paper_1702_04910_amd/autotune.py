"""Launch-shape autotuner for the sweep kernel.

For a box shape and storage precision it times the sweep kernel (HIP events
recorded by the library around every launch) over a grid of launch shapes:
rows per tile (sized by the LDS staging they need), workgroup size, a
persistent grid or one workgroup per tile, plain or non-temporal loads, the
six-wave build, a cap on the sweep workgroups resident per CU (fewer
concurrent streams can raise the achieved HBM bandwidth) and one, two or four
cells per thread.  The timing instance
is a coupling-free copy of the box (the sweep kernel does not depend on the
coupling); one instance per row count, the other parameters switched with
set_launch.  Results are cached in a JSON file keyed by the device name, shape
and precision; shapes tuned on an MI355X ship with the package
(tuned_shapes.json, written by this tuner, with the hash of the sweep sources
they were timed on) and are used when the cache has no entry and the sources
are unchanged, so a fresh machine of the same kind does not time them again.

    python -m paper_1702_04910_amd.autotune 192 192 384 fp32
"""
import json
import os
import sys
import time

from . import lbmps

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbmps", "sweep_tuning.json")
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


def _shipped():
    """Shipped shapes, when they were tuned on the current sweep sources."""
    from .counters import sweep_source_hash

    try:
        doc = json.load(open(SHIPPED))
    except (OSError, ValueError):
        return {}
    return doc.get("shapes", {}) if doc.get("sweep_source") == sweep_source_hash() else {}


def _key(nx, ny, nz, precision):
    """Cache key: the GPU's architecture and compute-unit count (not its
    marketing name, which depends on the driver's name table), box, precision."""
    import torch

    prop = torch.cuda.get_device_properties(0)
    arch = getattr(prop, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return "%s|%dCU|%dx%dx%d|%s" % (arch.split(":")[0], prop.multi_processor_count, nx, ny, nz, precision)


# where the last tune() result came from: "cache", "shipped" or "timed"
LAST_SOURCE = None


CAPS = (0, lbmps.SWEEP_WG_CAP3, lbmps.SWEEP_WG_CAP2)


def _cells_per_thread(nx, s, flags):
    """Flags for one, two (even nx) or four (2-byte storage, nx a multiple of
    4) cells per sweep thread; neither with the six-wave build (bit 3)."""
    if flags & lbmps.SWEEP_OCC6:
        return (0,)
    out = [0]
    if nx % 2 == 0:
        out.append(lbmps.SWEEP_CELL_PAIRS)
    if s == 2 and nx % 4 == 0:
        out.append(lbmps.SWEEP_CELL_QUADS)
    return tuple(out)


def candidates(nx, precision):
    """Launch shapes to time, grouped by tile_rows (one timing instance each)."""
    s = lbmps.STORAGE_BYTES[lbmps.PRECISION[precision]]
    max_rows = max(1, 65536 // (10 * s * nx))
    rows = sorted({max(1, min(max_rows, t // nx)) for t in (256, 512, 1024, 2048, 4096)})
    out = []
    for r in rows:
        for block in (128, 256):
            for grid in (0, 2048):
                for flags in ((0, 1, 8, 9) if s < 8 else (0, 1)):  # + six-wave build (bit 3) for 4/2-byte storage
                    for cap in CAPS:
                        for cells in _cells_per_thread(nx, s, flags):
                            out.append(dict(tile_rows=r, block_threads=block, grid_blocks=grid,
                                            sweep_flags=flags | cap | cells))
    return out


def _time_launches(sim, shapes, sweeps, warmup):
    """Microseconds per sweep launch for each shape, on one instance."""
    out = []
    for sh in shapes:
        sim.set_launch(sh["block_threads"], sh["grid_blocks"], sh["sweep_flags"])
        sim.step(warmup)
        sim.sync()
        sim.set_timing(True)
        sim.step(sweeps)
        ms, n = sim.timing()
        sim.set_timing(False)
        out.append(ms / n * 1e3)
    return out


def time_shape(nx, ny, nz, precision, shape, sweeps=20, warmup=4):
    cfg = lbmps.make_config(nx, ny, nz, 0.05, precision=precision, **shape)
    sim = lbmps.Sim(cfg)
    try:
        sim.init_equilibrium()
        return _time_launches(sim, [shape], sweeps, warmup)[0]
    finally:
        sim.close()


def tune(nx, ny, nz, precision, sweeps=20, cache=CACHE, force=False, verbose=False):
    """Best launch shape for the box; returns dict(tile_rows, block_threads,
    grid_blocks, sweep_flags, us)."""
    key = _key(nx, ny, nz, precision)
    db = {}
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
        except ValueError:
            db = {}
    global LAST_SOURCE
    if key in db and not force:
        LAST_SOURCE = "cache"
        return db[key]
    if not force:
        ship = _shipped()
        if key in ship:
            LAST_SOURCE = "shipped"
            return ship[key]
    LAST_SOURCE = "timed"
    best = None
    cands = candidates(nx, precision)
    for r in sorted({c["tile_rows"] for c in cands}):
        group = [c for c in cands if c["tile_rows"] == r]
        sim = lbmps.Sim(lbmps.make_config(nx, ny, nz, 0.05, precision=precision, **group[0]))
        try:
            sim.init_equilibrium()
            times = _time_launches(sim, group, sweeps, 4)
        finally:
            sim.close()
        for shape, us in zip(group, times):
            if verbose:
                print("  %s -> %.1f us" % (shape, us), file=sys.stderr, flush=True)
            if best is None or us < best["us"]:
                best = dict(shape, us=us)
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = best
        tmp = cache + ".tmp%d" % os.getpid()
        json.dump(db, open(tmp, "w"), indent=1)
        os.replace(tmp, cache)
    return best


def tune_batch(make_sim, tile_cells=(256, 288, 384, 512, 1024), grids=(0, 1024, 2048, 4096), sweeps=10,
               verbose=False):
    """Launch shape for a batched context.  make_sim(tile_cells) must return a
    ready Sim whose configurations use rows = max(1, tile_cells // nx) (288 and
    384 give two rows of the 144-wide boxes and two to four of the 96-wide
    ones, among the fastest tiles of those widths alone).  Times
    the batched sweep for each tile size x grid x load kind; returns the best
    dict(tile_cells, block_threads, grid_blocks, sweep_flags, us)."""
    best = None
    for tc in tile_cells:
        sim = make_sim(tc)
        try:
            for grid in grids:
                for flags in [f | cap | pr for f in (0, 1, 8, 9) for cap in CAPS
                              for pr in ((0,) if f & 8 else (0, lbmps.SWEEP_CELL_PAIRS, lbmps.SWEEP_CELL_QUADS))]:
                    try:
                        sim.set_launch(256, grid, flags)
                    except lbmps.LbmpsError:  # cell pairs / quads need every instance's nx even / 2-byte storage
                        continue
                    sim.set_timing(True)
                    sim.step(sweeps)
                    ms, n = sim.timing()
                    sim.set_timing(False)
                    us = ms / n * 1e3
                    if verbose:
                        print("  tile %d grid %d flags %d -> %.1f us" % (tc, grid, flags, us), file=sys.stderr,
                              flush=True)
                    if best is None or us < best["us"]:
                        best = dict(tile_cells=tc, block_threads=256, grid_blocks=grid, sweep_flags=flags, us=us)
        finally:
            sim.close()
    return best


if __name__ == "__main__":
    nx, ny, nz = (int(v) for v in sys.argv[1:4])
    prec = sys.argv[4] if len(sys.argv) > 4 else "fp32"
    t0 = time.time()
    r = tune(nx, ny, nz, prec, force=True, verbose=True)
    print(json.dumps(r), "(%.1f s)" % (time.time() - t0))
