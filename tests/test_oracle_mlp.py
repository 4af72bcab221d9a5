"""Pins of the solid-fraction network's reference arithmetic (oracle/mlp.py):
bfloat16 rounding against hand-worked values and torch's conversion, the
FP64 backward pass against central finite differences, and the input
features against the cube symmetry they encode.  Pure CPU."""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle import mlp
from paper_1702_04910_amd import inputs


# ----------------------------------------------------------------------- bfloat16
def test_bf16_round_to_nearest_even_worked_values():
    u = 2.0 ** -7  # bf16 spacing just above 1
    cases = [
        (1.0, 1.0),
        (1.0 + u / 2, 1.0),                 # tie -> even (down)
        (1.0 + 3 * u / 2, 1.0 + 2 * u),     # tie -> even (up)
        (1.0 + u / 2 + 2.0 ** -20, 1.0 + u),  # just above the tie
        (1.0 + u / 2 - 2.0 ** -20, 1.0),      # just below the tie
        (-(1.0 + 3 * u / 2), -(1.0 + 2 * u)),
        (3.0, 3.0),
        (2.0 ** 100 * (1.0 + 2.0 ** -9), 2.0 ** 100),
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert mlp.bf16(np.array([x]))[0] == want, x


def test_bf16_matches_torch_conversion_of_float32():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), want)


# ----------------------------------------------------------------------- features
def test_features_are_cube_symmetric_and_sorted():
    rng = np.random.default_rng(11)
    d = rng.uniform(-6, 6, (200, 3))
    R = rng.uniform(3, 12, 200)
    x = mlp.features(d, R)
    assert x.shape == (200, mlp.NIN)
    r = np.linalg.norm(d, axis=1)
    assert np.allclose(x[:, 0], r - R, rtol=0, atol=1e-14)
    assert np.all(x[:, 1] >= x[:, 2]) and np.all(x[:, 2] >= x[:, 3]) and np.all(x[:, 3] >= 0)
    assert np.allclose((x[:, 1:4] ** 2).sum(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.array_equal(x[:, 4], 8.0 / R)
    assert np.all(x[:, 5:] == 0)
    for perm in ([1, 0, 2], [2, 1, 0], [1, 2, 0]):
        for signs in ([1, 1, 1], [-1, 1, 1], [1, -1, -1], [-1, -1, -1]):
            d2 = d[:, perm] * np.array(signs)
            assert np.array_equal(mlp.features(d2, R), x)
    # the supersampled fraction has the same symmetry (what makes the features sufficient)
    n = 8
    for k in range(20):
        base = geo.eps_flat_counts(d[k:k + 1, 0], d[k:k + 1, 1], d[k:k + 1, 2], R[k], n)
        d2 = -d[k:k + 1, [2, 0, 1]]
        assert geo.eps_flat_counts(d2[:, 0], d2[:, 1], d2[:, 2], R[k], n)[0] == base[0]


# ----------------------------------------------------------------------- backward
def _problem(seed, m=48):
    rng = np.random.default_rng(seed)
    p = mlp.unpack(inputs.mlp_init(seed).astype(np.float64))
    p["b1"] = rng.standard_normal(mlp.NH) * 0.1
    p["b2"] = rng.standard_normal(mlp.NH) * 0.1
    R = rng.uniform(4, 10, m)
    d = rng.uniform(-1, 1, (m, 3)) * R[:, None]
    X = mlp.features(d, R)
    t = rng.uniform(0, 1, m)
    return p, X, t


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_matches_central_differences(seed):
    p, X, t = _problem(seed)
    g = mlp.backward(p, X, t)
    blob = mlp.pack(p)
    gb = mlp.pack(g)
    rng = np.random.default_rng(seed + 100)
    # every bias and output weight, and a sample of the matrix entries
    sizes = {name: int(np.prod(s)) for name, s in mlp.SIZES}
    offs = np.cumsum([0] + [sizes[name] for name, _ in mlp.SIZES])
    idx = list(range(offs[1], offs[2])) + list(range(offs[3], offs[6]))  # b1; b2, W3, b3
    idx += list(rng.choice(np.arange(offs[0], offs[1]), 40, replace=False))
    idx += list(rng.choice(np.arange(offs[2], offs[3]), 80, replace=False))
    idx = sorted(set(int(i) for i in idx))
    h = 1e-6
    worst = 0.0
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (mlp.loss(mlp.unpack(bp), X, t) - mlp.loss(mlp.unpack(bm), X, t)) / (2 * h)
        worst = max(worst, abs(fd - gb[i]) / max(1e-3, np.abs(gb).max()))
    assert worst < 1e-7


def test_planted_error_in_backward_is_caught():
    """A dropped ReLU mask on layer 1 (a plausible slip) fails the check above."""
    p, X, t = _problem(3)
    g = mlp.backward(p, X, t)
    _, c = mlp.forward(p, X)
    dy = 2.0 * (mlp.forward(p, X)[0] - t) / len(t)
    dZ2 = np.outer(dy, p["W3"]) * (c["Z2"] > 0)
    wrong_W1 = (dZ2 @ p["W2"]).T @ X  # no [Z1 > 0] factor
    assert np.abs(wrong_W1 - g["W1"]).max() > 1e-3 * np.abs(g["W1"]).max()


def test_bf16_emulation_stays_close_to_fp64():
    p, X, t = _problem(4, m=256)
    y, _ = mlp.forward(p, X)
    yb, _ = mlp.forward(p, X, emulate_bf16=True)
    assert np.abs(yb - y).max() < 3e-2 * (np.abs(y).max() + 1)
    g = mlp.pack(mlp.backward(p, X, t))
    gb = mlp.pack(mlp.backward(p, X, t, emulate_bf16=True))
    assert np.linalg.norm(gb - g) < 2e-2 * np.linalg.norm(g)


def test_pack_roundtrip_and_size():
    p = mlp.unpack(inputs.mlp_init(0).astype(np.float64))
    blob = mlp.pack(p)
    assert blob.size == mlp.NPARAM == 4801
    q = mlp.unpack(blob)
    for name, _ in mlp.SIZES:
        assert np.array_equal(q[name], p[name])
