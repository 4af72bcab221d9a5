"""Shared driver of the Sec. 3 drag study (simple-cubic periodic sphere array):
L = 32, D = L/2 at the box centre, body force a = (1e-5, 0, 0), run until the
dimensionless drag C converges.  Works with any object exposing
``step(n)``, ``force_x()`` and ``mean_ux()``."""
import json
import math
import os

C_REF = 2.8402  # Sangani & Acrivos value quoted in Sec. 3
L_BOX = 32
D_SPHERE = 16.0
A_FORCE = 1e-5

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fig1_drag_error.json")

LABELS = {"mem_bb": "MEM BB", "mem_cli": "MEM CLI", (1, 1): "PSM M1B1", (2, 2): "PSM M2B2", (3, 2): "PSM M3B2"}


def paper_value(label, tau):
    series = json.load(open(_GOLD))["series"][label]
    for t, v in series:
        if abs(t - tau) < 1e-9:
            return v
    raise KeyError((label, tau))


def drag_C(force_x, mean_ux, nu):
    """C = a.(F_d + F_b)/|a| / (3 pi rho0 nu D u_bar), F_b = pi/6 D^3 a (Sec. 3)."""
    Fb = math.pi / 6.0 * D_SPHERE ** 3 * A_FORCE
    return (force_x + Fb) / (3.0 * math.pi * nu * D_SPHERE * mean_ux)


def run_to_convergence(sim, nu, chunk=100, rel=1e-5, max_steps=40000):
    prev = None
    steps = 0
    while steps < max_steps:
        sim.step(chunk)
        steps += chunk
        C = drag_C(sim.force_x(), sim.mean_ux(), nu)
        if prev is not None and abs(C - prev) < rel * abs(C):
            return C / C_REF - 1.0, steps
        prev = C
    return C / C_REF - 1.0, steps
