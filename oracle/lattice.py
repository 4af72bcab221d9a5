"""D3Q19 lattice (Sec. 2.1: the 19-velocity cubic lattice, lattice units
dx = dt = rho0 = 1, c_s^2 = 1/3).

The paper cites the weights to Qian et al. without printing them; the standard
D3Q19 values are used: 1/3 for the rest velocity, 1/18 for the six axis
velocities and 1/36 for the twelve face diagonals.

The velocity ORDER here is the oracle's own (built by enumeration, sorted by
speed).  The GPU library uses its own, different order; tests match the two by
velocity vector, never by index.
"""
import numpy as np

CS2 = 1.0 / 3.0  # c_s^2 in lattice units


def _build():
    vel = []
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                if cx * cx + cy * cy + cz * cz <= 2:
                    vel.append((cx, cy, cz))
    vel.sort(key=lambda c: c[0] * c[0] + c[1] * c[1] + c[2] * c[2])  # stable: rest, axes, diagonals
    c = np.array(vel, dtype=np.int64)
    speed2 = (c * c).sum(axis=1)
    w = np.where(speed2 == 0, 1.0 / 3.0, np.where(speed2 == 1, 1.0 / 18.0, 1.0 / 36.0))
    opp = np.array([int(np.nonzero((c == -c[q]).all(axis=1))[0][0]) for q in range(len(c))])
    return c, w, opp


C, W, OPP = _build()
Q = 19
assert C.shape == (Q, 3)
CF = C.astype(np.float64)  # velocities as float, shape (19, 3), column 0 = x
