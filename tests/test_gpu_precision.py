"""16-bit storage forms (FP16 / BF16 deviations g = f - w_q, collision in
FP32) against the FP64 oracle.

Tolerance, derived from the arithmetic: starting from a state the storage
holds exactly, one sweep computes in FP32 (relative error ~1e-7) and rounds
once on store (FP16: to nearest even).  So every stored value equals the oracle's
FP64 result rounded once to the storage type, except where the FP32 and FP64
values straddle a rounding midpoint: there the two differ by one unit in the
last place (plus the FP32 absolute error, ~2^-20 of the largest deviation,
where cancellation leaves a result far below its inputs: BF16 resolves such
tiny values, FP16 flushes them into its subnormal spacing).  MEM link slots
are rebuilt from post-collision values that were stored (rounded) first; up
to three of them, so those slots get 4 u of the largest deviation more.  Forces come from
the same FP32 arithmetic on exact inputs: FP32
accuracy for PSM.  MEM link forces use post-collision values that the push
sweep has already stored, i.e. rounded: each link term may carry up to
4 u |g| (the CLI rule combines three stored values), so the bound adds
4 sqrt(2) u n_links max|g| / |F| to the FP32 tolerance.  Over k sweeps each store adds at most half a unit, u = 2^-11
(FP16) or 2^-8 (BF16) of the value; collision damps the non-equilibrium part
and conserves the rest, so the error stays below 4 k u of the largest
deviation.

The values pushed by PSM-overlapped cells, and with BF16 storage every stored
post-collision value, are rounded stochastically (to one of the two neighbours
of the FP32 result, the upper with probability equal to the distance from the
lower in units of their spacing), so those are checked to lie within one
spacing of the exact value, with about a quarter of them not the nearest.

Over a long horizon the error of the sphere's velocity and force is measured
at full size by the benchmark (bench.py, precision forms)."""
import numpy as np
import pytest

from oracle import mlp as om
from paper_1702_04910_amd import inputs
from gpu_util import make_pair, gpu_to_oracle, force_errors, say

pytestmark = pytest.mark.gpu

KINDS = ["fp16", "bf16"]
UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def round_store(x, kind):
    if kind == "fp16":
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)
    return om.bf16(x)


def ulp_store(x, kind):
    """Spacing of the storage type at the rounded magnitude of x."""
    r = np.abs(round_store(x, kind))
    if kind == "fp16":
        return np.spacing(r.astype(np.float16)).astype(np.float64)
    b = r.astype(np.float32).view(np.uint32)
    nxt = (((b >> 16) + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return nxt - r


def _check_rounded_once(go, gg, mask, kind, extra=None, stochastic=None):
    """mask: [z, y, x] cells compared; extra: optional [q, z, y, x] absolute
    allowance added to the tolerance (values built from stored inputs);
    stochastic: optional [q, z, y, x] mask of the values pushed by overlapped
    PSM cells, which are rounded stochastically (with BF16 storage every value
    is): each must be one of the two neighbours of the exact value (within one
    spacing of it), and they are left out of the exact-match fraction."""
    sr = np.zeros(go.shape, bool) if stochastic is None else stochastic.copy()
    if kind == "bf16":  # BF16 storage rounds every post-collision value stochastically
        sr[:] = True
    slack = 2.0 ** -20 * np.abs(go[:, mask]).max()
    sel = mask[None, :, :, :] & ~sr
    if sel.any():
        ref = round_store(go[sel], kind)
        got = gg[sel]
        diff = np.abs(got - ref)
        tol = ulp_store(go[sel], kind) + slack
        if extra is not None:
            tol = tol + extra[sel]
        exact = float(np.mean(got == ref))
        say("  exact fraction %.5f, max diff / tolerance %.2f" % (exact, float((diff / tol).max())))
        assert np.all(diff <= tol)
        assert exact >= 0.99
    ssel = mask[None, :, :, :] & sr
    if ssel.any():
        x, y = go[ssel], gg[ssel]
        tol = ulp_store(x, kind) + slack + (extra[ssel] if extra is not None else 0.0)
        assert np.all(np.abs(y - x) <= tol)
        differs = float(np.mean(y != round_store(x, kind)))
        say("  %d stochastically rounded values, %.3f of them not the nearest" % (x.size, differs))
        assert 0.05 < differs < 0.5


@pytest.mark.parametrize("kind", KINDS)
def test_fluid_sweep_rounds_once(kind):
    nx, ny, nz = 37, 23, 19
    g0 = round_store(inputs.random_pdfs((nz, ny, nx), 1e-3, seed=15), kind)
    say("fluid one sweep", kind)
    ora, sim = make_pair(nx, ny, nz, 0.07, collision="trt", f_ext=(1e-5, -2e-5, 3e-5), precision=kind, g0=g0)
    assert np.array_equal(gpu_to_oracle(sim.get_pdfs()), g0)  # the storage holds the start exactly
    ora.step(1)
    sim.step(1)
    _check_rounded_once(ora.get_pdfs(), gpu_to_oracle(sim.get_pdfs()), ora.owner == -1, kind)
    sim.close()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("coupling,m,b", [("mem_cli", 1, 1), ("mem_bb", 1, 1), ("psm", 3, 2), ("psm", 1, 1)])
def test_coupled_sweep_rounds_once(kind, coupling, m, b):
    c = inputs.c1_plain(1)
    parts = dict(X=[c["X"]], U=[[1e-3, -2e-3, 5e-4]], Om=[[1e-4, 0, -2e-4]], D=[c["D"]], rho=[1.5], fixed=[True])
    shape = (c["nz"], c["ny"], c["nx"])
    g0 = round_store(inputs.random_pdfs(shape, 1e-4, seed=16), kind)
    say("coupled one sweep", kind, coupling, m, b)
    ora, sim = make_pair(c["nx"], c["ny"], c["nz"], 0.05, coupling=coupling, collision="trt", psm_m=m, psm_b=b,
                         f_ext=c["f_ext"], precision=kind, eps_n=8, parts=parts, g0=g0, n_sub=1)
    ora.step(1)
    sim.step(1)
    go = ora.get_pdfs()
    extra = None
    if coupling.startswith("mem"):
        # the link rule rewrites f_qbar(x) from post-collision values the push
        # sweep already stored (rounded): up to three such inputs
        from oracle.lattice import OPP
        L = ora.links
        extra = np.zeros_like(go)
        extra[OPP[L["q"]], L["iz"], L["iy"], L["ix"]] = 4 * UNIT[kind] * np.abs(go).max()
    stochastic = None
    if coupling == "psm":
        # values pushed by overlapped cells: cell + c_q, direction q
        from oracle.lattice import C
        iz, iy, ix, _ = ora.overlaps[0]
        stochastic = np.zeros(go.shape, bool)
        for q in range(19):
            stochastic[q, (iz + C[q, 2]) % shape[0], (iy + C[q, 1]) % shape[1], (ix + C[q, 0]) % shape[2]] = True
    _check_rounded_once(go, gpu_to_oracle(sim.get_pdfs()), ora.owner == -1, kind, extra, stochastic)
    (eF, eT, nF), = force_errors(ora, sim)[0]
    bound = 1e-5
    if coupling.startswith("mem"):
        gmax = max(np.abs(g0).max(), np.abs(ora.get_pdfs()).max())
        bound += 4 * np.sqrt(2.0) * UNIT[kind] * len(ora.links["q"]) * gmax / nF
    say("  e_F %.2e e_T %.2e (bound %.2e)" % (eF, eT, bound))
    assert eF < bound and eT < 1.5 * bound
    sim.close()


@pytest.mark.parametrize("kind", KINDS)
def test_error_growth_bounded_over_sweeps(kind):
    nx, ny, nz = 40, 24, 20
    k = 20
    g0 = round_store(inputs.random_pdfs((nz, ny, nx), 1e-3, seed=17), kind)
    ora, sim = make_pair(nx, ny, nz, 0.05, collision="trt", f_ext=(2e-5, 0, 0), precision=kind, g0=g0)
    ora.step(k)
    sim.step(k)
    go = ora.get_pdfs()
    gg = gpu_to_oracle(sim.get_pdfs())
    e = np.abs(gg - go).max() / np.abs(go).max()
    say("  %s after %d sweeps: e_f = %.3e (bound %.3e)" % (kind, k, e, 4 * k * UNIT[kind]))
    assert e <= 4 * k * UNIT[kind]
    sim.close()
