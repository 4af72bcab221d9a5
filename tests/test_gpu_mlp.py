"""Learned solid fraction on the GPU: labels against the oracle's exact
supersampling counts, the MFMA forward and backward passes against the
oracle's bfloat16-emulating FP64 reference, training, the estimator inside a
PSM context (exact cells, fallback, judge), and its cost against exact
supersampling."""
import math
import time

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import mlp as om
from paper_1702_04910_amd import inputs, lbmps
from gpu_util import say

pytestmark = pytest.mark.gpu


def _exact_eps(rd, n):
    out = np.empty(len(rd))
    for i, (R, dx, dy, dz) in enumerate(rd):
        out[i] = geo.eps_flat_counts(np.array([dx]), np.array([dy]), np.array([dz]), R, n)[0] / float(n) ** 3
    return out


def _params(seed):
    p = om.unpack(inputs.mlp_init(seed).astype(np.float64))
    rng = np.random.default_rng(seed + 7)
    p["b1"] = rng.standard_normal(om.NH) * 0.1
    p["b2"] = rng.standard_normal(om.NH) * 0.1
    return om.pack(p).astype(np.float32)


def test_labels_equal_oracle_supersampling():
    rd = inputs.eps_training_cells(1, 1500)
    m = lbmps.Mlp(len(rd))
    m.set_samples(rd)
    for n in (16, 5):
        say("label n =", n)
        m.label(n)
        got = m.targets()
        assert np.array_equal(got, _exact_eps(rd, n).astype(np.float32))
    m.close()


@pytest.mark.parametrize("n", [4999, 32, 1])
def test_forward_matches_bf16_reference(n):
    rd = inputs.eps_training_cells(2, n)
    blob = _params(3)
    m = lbmps.Mlp(n)
    m.set_samples(rd)
    m.set_params(blob)
    assert np.array_equal(m.params(), blob)
    y = m.predict()
    X = om.features(rd[:, 1:], rd[:, 0])
    ref, _ = om.forward(om.unpack(blob.astype(np.float64)), X, emulate_bf16=True)
    ref = np.clip(ref, 0.0, 1.0)
    say("forward max err", np.abs(y - ref).max())
    assert np.abs(y - ref).max() < 1e-3
    m.close()


@pytest.mark.parametrize("batch,b0", [(1000, 0), (77, 4950), (32, 13)])
def test_gradient_matches_oracle_backprop(batch, b0):
    n = 5000
    rd = inputs.eps_training_cells(4, n)
    blob = _params(5)
    m = lbmps.Mlp(n)
    m.set_samples(rd)
    m.set_params(blob)
    m.label(16)
    t = m.targets().astype(np.float64)
    mult, add = 1237, 411  # gcd(1237, 5000) = 1
    g = m.gradient(b0, batch, mult, add)
    idx = ((((b0 + np.arange(batch)) % n) * mult + add) % n)
    X = om.features(rd[idx, 1:], rd[idx, 0])
    p = om.unpack(blob.astype(np.float64))
    ge = om.pack(om.backward(p, X, t[idx], emulate_bf16=True))
    g64 = om.pack(om.backward(p, X, t[idx]))
    off = 0
    for name, shp in om.SIZES:
        k = int(np.prod(shp))
        a, b, c = g[off:off + k], ge[off:off + k], g64[off:off + k]
        scale = np.linalg.norm(b) + 1e-30
        say("  %s rel err vs bf16 ref %.2e, vs fp64 %.2e" % (name, np.linalg.norm(a - b) / scale,
                                                             np.linalg.norm(a - c) / (np.linalg.norm(c) + 1e-30)))
        assert np.linalg.norm(a - b) <= 1e-2 * scale, name
        assert np.linalg.norm(a - c) <= 5e-2 * (np.linalg.norm(c) + 1e-30), name
        off += k
    # a bad sample order is rejected
    with pytest.raises(lbmps.LbmpsError):
        m.gradient(0, batch, 10, 0)  # gcd(10, 5000) != 1
    m.close()


def _train(n=65536, seed=8):
    rd = inputs.eps_training_cells(seed, n)
    m = lbmps.Mlp(n)
    m.set_samples(rd)
    m.set_params(inputs.mlp_init(seed))
    m.label(16)
    t = m.targets()
    y0 = m.predict()
    mult, add = inputs.affine_orders(seed, n, 18)
    t0 = time.time()
    m.train(mult[:12], add[:12], batch=512, lr=2e-3)
    m.train(mult[12:], add[12:], batch=512, lr=5e-4)
    y1 = m.predict()
    dt = time.time() - t0
    return m, t, y0, y1, dt


@pytest.fixture(scope="module")
def trained():
    m, t, y0, y1, dt = _train()
    say("trained: rmse %.4f -> %.4f, mean |err| %.4f (%.1f s)" % (
        np.sqrt(np.mean((y0 - t) ** 2)), np.sqrt(np.mean((y1 - t) ** 2)), np.mean(np.abs(y1 - t)), dt))
    p = m.params()
    m.close()
    return dict(params=p, t=t, y0=y0, y1=y1)


def test_training_reduces_error(trained):
    t, y0, y1 = trained["t"], trained["y0"], trained["y1"]
    r0 = np.sqrt(np.mean((y0 - t) ** 2))
    r1 = np.sqrt(np.mean((y1 - t) ** 2))
    assert r1 < 0.05 * r0
    assert np.mean(np.abs(y1 - t)) < 0.015


def _psm_ctx(eps_mode, eps_n, box, X, D):
    cfg = lbmps.make_config(box, box, box, 0.05, coupling="psm", psm_m=2, psm_b=2, eps_n=eps_n, eps_mode=eps_mode,
                            precision="fp32", max_particles=len(D), max_diameter=float(max(D)))
    return lbmps.Sim(cfg)


def _sph(seed, box=64, n=4):
    rng = np.random.default_rng(seed)
    X = [np.array([16.0, 16.0, 16.0]) + rng.uniform(-0.5, 0.5, 3) + 32.0 * np.array([i & 1, (i >> 1) & 1, 0])
         for i in range(n)]
    D = list(rng.uniform(11.0, 21.0, n))
    return X, D


def _exact_bbox(shape, X, R, n):
    """Exact eps (flat n^3) of every cell of the sphere's bounding box: {cell: eps}."""
    nz, ny, nx = shape
    ix, iy, iz = (geo.bbox_range(X[0], R, nx), geo.bbox_range(X[1], R, ny), geo.bbox_range(X[2], R, nz))
    gz, gy, gx = [a.ravel() for a in np.meshgrid(iz, iy, ix, indexing="ij")]
    dcx, dcy, dcz = geo.centre_disp(gx, X[0], nx), geo.centre_disp(gy, X[1], ny), geo.centre_disp(gz, X[2], nz)
    out = {}
    for a in range(0, len(gx), 1000):
        cnt = geo.eps_flat_counts(dcx[a:a + 1000], dcy[a:a + 1000], dcz[a:a + 1000], R, n)
        for k, c in enumerate(cnt):
            i = a + k
            out[int((gz[i] * ny + gy[i]) * nx + gx[i])] = c / float(n) ** 3
    return out


def test_learned_context_exact_cells_and_judge(trained):
    X, D = _sph(21)
    sim = _psm_ctx(lbmps.EPS_LEARNED, 16, 64, X, D)
    sim.init_equilibrium()
    with pytest.raises(lbmps.LbmpsError):
        sim.set_particles(X, [[0, 0, 0]] * 4, [[0, 0, 0]] * 4, D, [1.5] * 4, [True] * 4)
    sim.set_eps_model(trained["params"], 5.5, 10.5)
    sim.set_particles(X, [[0, 0, 0]] * 4, [[0, 0, 0]] * 4, D, [1.5] * 4, [True] * 4)
    ov = sim.overlaps()
    mean_err, max_err, n_judged = sim.eps_judge(1)
    say("judge: mean %.4f max %.4f over %d" % (mean_err, max_err, n_judged))
    errs = []
    for p in range(4):
        exact = _exact_bbox((64, 64, 64), X[p], 0.5 * D[p], 16)
        sel = ov["p"] == p
        got = dict(zip(ov["cell"][sel].tolist(), ov["eps"][sel].tolist()))
        for c, e in exact.items():
            if e == 1.0:
                assert got.get(c) == 1.0  # cells entirely inside stay exact
            errs.append(abs(got.get(c, 0.0) - e))
        assert set(got) <= set(exact)
        assert all(0.0 < e <= 1.0 for e in got.values())
    errs = np.array(errs)
    # every nonzero error sits in a cut cell the judge recounts
    assert n_judged > 1000
    assert abs(errs.max() - max_err) < 1e-12
    assert abs(errs.sum() - mean_err * n_judged) < 1e-9 * max(1.0, errs.sum())
    assert mean_err < 0.02
    sim.close()


def test_learned_fallback_outside_radius_range_is_exact(trained):
    X, D = _sph(22)
    ref = _psm_ctx(lbmps.EPS_FLAT, 16, 64, X, D)
    ref.init_equilibrium()
    ref.set_particles(X, [[0, 0, 0]] * 4, [[0, 0, 0]] * 4, D, [1.5] * 4, [True] * 4)
    sim = _psm_ctx(lbmps.EPS_LEARNED, 16, 64, X, D)
    sim.init_equilibrium()
    sim.set_eps_model(trained["params"], 1.0, 2.0)  # no particle in range: all supersampled
    sim.set_particles(X, [[0, 0, 0]] * 4, [[0, 0, 0]] * 4, D, [1.5] * 4, [True] * 4)
    a, b = ref.overlaps(), sim.overlaps()
    assert np.array_equal(a["cell"], b["cell"]) and np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["eps"], b["eps"])
    ref.step(4)
    sim.step(4)
    assert np.array_equal(ref.get_pdfs(), sim.get_pdfs())
    ref.close()
    sim.close()


def test_learned_estimator_gain_over_exact_sampling(trained):
    """What the network gains: on the same 120 spheres its largest solid-
    fraction error against flat 16^3 supersampling (the reference) is smaller
    than that of flat 8^3 sampling, although it evaluates no sample point at
    all for the cut cells in its radius range (flat 8^3 tests 512 per cut cell,
    the reference 4096).  The
    rebuild times are printed; the timed comparison belongs to the benchmark
    (bench.py, learned form), not to this pass/fail test."""
    import torch

    wl = inputs.c5_learned(0, n=300)
    L = 256
    sel = np.all(wl["X"] < L, axis=1)
    X, D = wl["X"][sel][:120], wl["D"][sel][:120]
    eps, ms = {}, {}
    for name, mode, n in (("flat16", lbmps.EPS_FLAT, 16), ("flat8", lbmps.EPS_FLAT, 8),
                          ("learned", lbmps.EPS_LEARNED, 16)):
        cfg = lbmps.make_config(L, L, L, 0.01, coupling="psm", psm_m=3, psm_b=2, n_sub=2, eps_n=n, eps_mode=mode,
                                precision="fp32", max_particles=len(D), max_diameter=20.0)
        sim = lbmps.Sim(cfg)
        sim.init_equilibrium()
        if mode == lbmps.EPS_LEARNED:
            sim.set_eps_model(trained["params"], 5.5, 10.5)
        sim.set_particles(X, [[0, 0, 0]] * len(D), [[0, 0, 0]] * len(D), D, [1.5] * len(D), [False] * len(D))
        ov = sim.overlaps()
        eps[name] = {(int(p), int(c)): float(e) for p, c, e in zip(ov["p"], ov["cell"], ov["eps"])}
        if mode == lbmps.EPS_LEARNED:
            assert sim.eps_judge(1)[2] > 0.9 * sum(1 for e in eps[name].values() if e < 1.0)
        sim.sync()
        t0 = time.perf_counter()
        for _ in range(5):
            sim.rebuild_overlaps()
        sim.sync()
        ms[name] = (time.perf_counter() - t0) / 5 * 1e3
        sim.close()
        torch.cuda.empty_cache()
    ref = eps["flat16"]

    def err(other):
        keys = set(ref) | set(other)
        d = np.array([abs(ref.get(k, 0.0) - other.get(k, 0.0)) for k in keys
                      if 0.0 < ref.get(k, 0.0) < 1.0 or 0.0 < other.get(k, 0.0) < 1.0])
        return float(d.mean()), float(d.max())

    e8, el = err(eps["flat8"]), err(eps["learned"])
    say("eps error vs flat 16^3 (mean, max): flat 8^3 %s, network %s; rebuild ms %s"
        % (np.round(e8, 4), np.round(el, 4), {k: round(v, 3) for k, v in ms.items()}))
    # the network's worst cut cell is better than flat 8^3 sampling's, and its
    # mean error stays within the judge's bound
    assert el[1] < e8[1]
    assert el[0] < 0.01
