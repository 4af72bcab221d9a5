"""Shared driver of the Sec. 3 drag study (simple-cubic periodic sphere array):
L = 32, D = L/2 at the box centre, body force along x, run until the
dimensionless drag C has converged.

Reading of the forcing amplitude: Sec. 3 treats the flow as Stokes flow
(the reference C_ref is the creeping-flow value) and quotes a = 1e-5.  With
Eq. LBM_EQ's quadratic terms that holds at tau = 1.5 (Reynolds number u_bar D /
nu ~ 0.1) but not at small tau: a = 1e-5 at tau = 0.6 gives u_bar D / nu ~ 10,
where inertia raises C by ~4 % for every coupling alike, whereas the paper's
momentum-exchange curves stay flat down to tau = 0.55.  The drag study is
therefore run at the Reynolds number of the tau = 1.5 run for every tau:
a = 1e-5 (nu / nu_1.5)^2, which keeps u_bar D / nu fixed (u_bar ~ a / nu).  C
does not depend on a in the Stokes regime.

Convergence: C(t) approaches its limit like C_inf + A exp(-t / T) with
T = L^3 / (3 pi nu D C) (the mean flow's response time), i.e. ~240 steps at
tau = 1.5 and ~2400 at tau = 0.6.  C is sampled every `chunk` steps; the limit
is estimated by Aitken's delta-squared extrapolation of three consecutive
samples, and the run stops when two consecutive estimates agree.  The
tau = 0.6 run starts from the converged tau = 1.5 flow rescaled to the new
viscosity and force (Stokes flow: u ~ a / nu, pressure ~ a): the steady state
does not depend on the start, only the time to reach it does.
"""
import json
import math
import os

C_REF = 2.8402  # Sangani & Acrivos value quoted in Sec. 3
L_BOX = 32
D_SPHERE = 16.0
A_FORCE = 1e-5
NU_REF = 1.0 / 3.0  # tau = 1.5: the viscosity at which a = A_FORCE

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fig1_drag_error.json")

LABELS = {"mem_bb": "MEM BB", "mem_cli": "MEM CLI", (1, 1): "PSM M1B1", (2, 2): "PSM M2B2", (3, 2): "PSM M3B2"}
VARIANTS = {"MEM BB": ("mem_bb", 0, 0), "MEM CLI": ("mem_cli", 0, 0), "PSM M1B1": ("psm", 1, 1),
            "PSM M2B2": ("psm", 2, 2), "PSM M3B2": ("psm", 3, 2)}


def paper_value(label, tau):
    series = json.load(open(_GOLD))["series"][label]
    for t, v in series:
        if abs(t - tau) < 1e-9:
            return v
    raise KeyError((label, tau))


def force_density(nu):
    """Body force of the drag study at viscosity nu (fixed Reynolds number)."""
    return A_FORCE * (nu / NU_REF) ** 2


def drag_C(force_x, mean_ux, nu, a=A_FORCE):
    """C = a.(F_d + F_b)/|a| / (3 pi rho0 nu D u_bar), F_b = pi/6 D^3 a (Sec. 3)."""
    Fb = math.pi / 6.0 * D_SPHERE ** 3 * a
    return (force_x + Fb) / (3.0 * math.pi * nu * D_SPHERE * mean_ux)


def aitken(c0, c1, c2):
    """Limit of c0, c1, c2 taken as a geometric tail: c2 + d2 r / (1 - r) with
    the ratio r = d2 / d1 of the last two changes (Aitken's delta squared);
    None unless the tail is contracting and monotone (0 <= r < 0.95)."""
    d1, d2 = c1 - c0, c2 - c1
    if d1 == 0.0:
        return c2 if d2 == 0.0 else None
    r = d2 / d1
    if not 0.0 <= r < 0.95:
        return None
    return c2 + d2 * r / (1.0 - r)


def converge_C(step, measure, chunk, rel=2e-5, min_samples=4, max_steps=40000):
    """Sample C every chunk steps; stop when two consecutive Aitken estimates
    exist and agree to rel (relative).  Returns (C estimate, steps)."""
    cs, est, steps = [], [], 0
    while steps < max_steps:
        step(chunk)
        steps += chunk
        cs.append(measure())
        est.append(aitken(*cs[-3:]) if len(cs) >= 3 else None)
        if (len(cs) >= min_samples and est[-1] is not None and est[-2] is not None
                and abs(est[-1] - est[-2]) < rel * abs(est[-1])):
            return est[-1], steps
    raise RuntimeError("C did not converge in %d steps" % max_steps)


def run_oracle_variant(label):
    """Fig. 1 for one coupling variant on the FP64 oracle: the drag error
    C/C_ref - 1 at tau = 1.5, then at tau = 0.6 (warm-started from the
    tau = 1.5 flow).  Returns {tau: (error, steps)}."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fluid as fl
    from oracle.sim import OracleSim

    coupling, m, b = VARIANTS[label]
    coll = "trt" if coupling.startswith("mem") else "bgk"
    c = L_BOX / 2.0
    out = {}
    g_prev = None
    with threadpool_limits(limits=1):
        for tau, chunk in ((1.5, 100), (0.6, 500)):
            nu = (tau - 0.5) / 3.0
            a = force_density(nu)
            # forces averaged over two sweeps for every coupling (Sec. 4.1's
            # subcycles): under M3 a fully covered cell mirrors its
            # non-equilibrium part every sweep, so any interior deviation from
            # the particle velocity (the warm start leaves some) makes the
            # single-sweep force alternate without decay; the average of two
            # sweeps cancels that mode
            s = OracleSim(L_BOX, L_BOX, L_BOX, nu, collision=coll, coupling=coupling, psm_m=m, psm_b=b,
                          fext=(a, 0.0, 0.0), eps_n=8, n_sub=2)
            s.init_equilibrium()
            s.set_particles([[c, c, c]], [[0, 0, 0]], [[0, 0, 0]], [D_SPHERE], [1.0], [True])
            if g_prev is not None:
                # the tau = 1.5 Stokes flow rescaled: velocity ~ a / nu, pressure ~ a
                drho, U = fl.moments(g_prev[0])
                ku = (a / g_prev[1]) * (g_prev[2] / nu)
                kp = a / g_prev[1]
                s.set_pdfs(fl.geq(kp * drho, ku * U))

            def measure():
                return drag_C(s.F[0, 0], s.fields()[1][0].mean(), nu, a)

            C, steps = converge_C(s.step, measure, chunk)
            out[tau] = (C / C_REF - 1.0, steps)
            g_prev = (s.get_pdfs(), a, nu)
    return label, out
