"""Host-side logic that needs no GPU: the launch tuner's candidate shapes, the
source hash that ties committed hardware counters to the sweep sources, and
the benchmark's refusal of multi-GPU runs."""
import os
import subprocess
import sys

import pytest

from paper_1702_04910_amd import autotune, counters, lbmps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("nx,precision", [(192, "fp32"), (512, "fp32"), (192, "fp16"), (512, "bf16"), (38, "fp16"),
                                         (37, "fp32"), (96, "fp64")])
def test_tuner_candidates_are_valid_configurations(nx, precision):
    cands = autotune.candidates(nx, precision)
    assert len(cands) == len({tuple(sorted(c.items())) for c in cands})  # no duplicates
    s = lbmps.STORAGE_BYTES[lbmps.PRECISION[precision]]
    for c in cands:
        f = c["sweep_flags"]
        cfg = lbmps.make_config(nx, 16, 16, 0.05, precision=precision, **c)
        assert lbmps.workspace_bytes(cfg) > 0, c  # the library accepts it
        assert c["tile_rows"] * nx * 10 * s <= 65536  # LDS staging fits
        assert not (f & lbmps.SWEEP_CELL_PAIRS and (nx % 2 or f & lbmps.SWEEP_OCC6))
        assert not (f & lbmps.SWEEP_CELL_QUADS and (nx % 4 or s != 2 or f & (lbmps.SWEEP_OCC6 | lbmps.SWEEP_CELL_PAIRS)))
        assert not (f & lbmps.SWEEP_OCC6 and s == 8)  # six-wave build only for 4- and 2-byte storage
        assert (f & (lbmps.SWEEP_WG_CAP3 | lbmps.SWEEP_WG_CAP2)) != (lbmps.SWEEP_WG_CAP3 | lbmps.SWEEP_WG_CAP2)
    # every option is offered where it applies
    flags = {c["sweep_flags"] for c in cands}
    assert any(f & lbmps.SWEEP_WG_CAP2 for f in flags) and any(f & lbmps.SWEEP_WG_CAP3 for f in flags)
    assert any(f & lbmps.SWEEP_CELL_PAIRS for f in flags) == (nx % 2 == 0)
    assert any(f & lbmps.SWEEP_CELL_QUADS for f in flags) == (nx % 4 == 0 and s == 2)


def test_counter_hash_follows_the_sweep_sources():
    h = counters.sweep_source_hash()
    assert len(h) == 16 and h == counters.sweep_source_hash()
    # the hash covers every file the sweep kernel is compiled from
    src = open(os.path.join(ROOT, "paper_1702_04910_amd", "csrc", "sweep.hip")).read()
    for inc in ("common.h", "kernels.h", "psm_cell.h"):
        assert '#include "%s"' % inc in src
        assert "csrc/" + inc in counters.SWEEP_SOURCES


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_build_flags_keep_rounding_identical_across_kernels():
    # no packed FP32 and no mixed-precision FMAs (an FMA fused with the
    # conversion to FP16 storage rounds once, so its use would make the stored
    # bits depend on the kernel)
    from paper_1702_04910_amd import build

    flags = " ".join(build.CFLAGS)
    assert "-packed-fp32-ops" in flags and "-fma-mix-insts" in flags


def test_dominant_frequency_of_a_sampled_oscillation():
    # the frame driver's DFT frequency estimate (Tab. 3's f): a sine of known
    # frequency plus noise and an offset, sampled every quarter time unit
    import numpy as np

    from paper_1702_04910_amd.settling import dominant_frequency

    rng = np.random.default_rng(3)
    t = np.arange(0.0, 150.0, 0.25)
    for f in (0.0415, 0.071, 0.2):
        v = 0.12 + 0.02 * np.sin(2 * np.pi * f * t + 1.0) + 1e-3 * rng.standard_normal(len(t))
        assert abs(dominant_frequency(t, v) - f) < 0.002
    assert dominant_frequency(t[:5], t[:5]) is None
