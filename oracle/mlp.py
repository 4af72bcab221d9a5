"""Reference forward and backward pass of the solid-fraction surrogate (the
learned estimate of eps_s for cells cut by a sphere surface), FP64.

The paper computes eps_s by supersampling (Sec. 2.3.2) and notes that its cost
may dominate (Sec. 2.3.4); the surrogate replaces the supersampling of cut
cells.  Its design is not from the paper (parity unpinned for the design
choices; the arithmetic is pinned by finite differences):

* features of a cell with centre displacement d = x_c - X_p from a sphere of
  radius R: the signed distance |d| - R of the cell centre from the surface,
  the direction cosines |d_k| / |d| sorted descending (the cube symmetry of
  the cell makes eps_s invariant under axis permutations and reflections), and
  8 / R (curvature relative to the cell size, scaled to O(1)); padded with
  zeros to 8 inputs;
* network 8 -> 64 -> 64 -> 1 with ReLU hidden layers, output clamped to [0, 1]
  only at inference;
* loss: mean squared error over a batch, L = (1/M) sum_n (y_n - t_n)^2.

``forward``/``backward`` optionally round the operands of the five matrix
products (layer 1, layer 2, dH1 = dZ2 W2, dW2 = dZ2^T H1, dW1 = dZ1^T X) to
bfloat16 (round to nearest even): X, W1, W2, H1, dZ2 and dZ1.  Biases, the
output layer, the bias gradients and every sum stay in full precision.
"""
import numpy as np

NIN = 8
NH = 64
# parameter blob layout (float32 on the device, float64 here)
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(blob):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(blob[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16(x):
    """Round to bfloat16 the way a float32 operand is rounded: float64 to float32
    (nearest even), then float32 to bfloat16 (nearest even, on the bit pattern);
    returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(d, R):
    """Inputs for displacements d (n, 3) and radii R (n,): (n, 8)."""
    d = np.asarray(d, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    s = -np.sort(-np.abs(d), axis=1)  # |d_k| sorted descending
    r = np.sqrt((s[:, 0] * s[:, 0] + s[:, 1] * s[:, 1]) + s[:, 2] * s[:, 2])
    cos = s / np.where(r > 0, r, np.inf)[:, None]
    x = np.zeros((len(R), NIN))
    x[:, 0] = r - R
    x[:, 1:4] = cos
    x[:, 4] = 8.0 / R
    return x


def forward(p, X, emulate_bf16=False):
    r = bf16 if emulate_bf16 else (lambda v: v)
    W1, W2 = r(p["W1"]), r(p["W2"])
    Xb = r(X)
    Z1 = Xb @ W1.T + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    H1b = r(H1)
    Z2 = H1b @ W2.T + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    y = H2 @ p["W3"] + p["b3"][0]
    return y, dict(Xb=Xb, Z1=Z1, H1b=H1b, Z2=Z2, H2=H2, W1=W1, W2=W2)


def loss(p, X, t, emulate_bf16=False):
    y, _ = forward(p, X, emulate_bf16)
    return np.mean((y - t) ** 2)


def backward(p, X, t, emulate_bf16=False):
    """Gradients of the batch-mean squared error with respect to every parameter."""
    r = bf16 if emulate_bf16 else (lambda v: v)
    y, c = forward(p, X, emulate_bf16)
    M = len(t)
    dy = 2.0 * (y - t) / M
    g = {}
    g["W3"] = c["H2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dZ2 = np.outer(dy, p["W3"]) * (c["Z2"] > 0)
    dZ2b = r(dZ2)
    g["W2"] = dZ2b.T @ c["H1b"]
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2b @ c["W2"]
    dZ1 = dH1 * (c["Z1"] > 0)
    g["W1"] = r(dZ1).T @ c["Xb"]
    g["b1"] = dZ1.sum(axis=0)
    return g
