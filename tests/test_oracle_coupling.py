"""Pins of the oracle's particle coupling (Secs. 2.2-2.3, 3, 4.1) against
closed forms, invariants, brute force and the values of Fig. 1.  Pure CPU."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import fluid as fl
from oracle import geometry as geo
from oracle import mem as mm
from oracle import psm as ps
from oracle import rigid as rb
from oracle.lattice import C, CF, W, OPP, Q
from oracle.sim import OracleSim


RNG = np.random.default_rng(99)


# --------------------------------------------------------------------------- geometry
def test_link_delta_lies_on_surface():
    R = 3.7
    for _ in range(200):
        q = int(RNG.integers(1, 19))
        c = CF[q]
        # pick a fluid point just outside along -c from a point inside
        inside = RNG.uniform(-0.5, 0.5, 3) * R * 0.3
        d = inside - c * RNG.uniform(0.0, 1.0)
        while geo.dist2(*d) <= R * R:
            d = d - c * 0.3
        # move until d + c is inside and d outside
        u = -d / np.linalg.norm(d)
        d = u * -(R + 0.4)
        if geo.dist2(*(d + c)) > R * R:
            continue
        delta = float(geo.link_delta(d, c, R))
        assert 0.0 < delta <= 1.0
        p = d + delta * c
        assert abs(math.sqrt(geo.dist2(*p)) - R) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_recursive_supersampling_equals_flat(n):
    R = 2.5 + RNG.uniform(0, 3)
    X = RNG.uniform(10, 11, 3)
    a = geo.overlap_cells((24, 24, 24), X, R, n, recursive=False)
    b = geo.overlap_cells((24, 24, 24), X, R, n, recursive=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def _cube_sphere_volume(cx, cy, cz, R):
    """Exact volume of the unit cube centred at displacement (cx, cy, cz) from the
    sphere centre intersected with the ball of radius R (2-D quadrature of the
    covered z-extent)."""
    def h(y, x):
        r2 = R * R - x * x - y * y
        if r2 <= 0:
            return 0.0
        s = math.sqrt(r2)
        return max(0.0, min(cz + 0.5, s) - max(cz - 0.5, -s))
    v, err = integrate.dblquad(h, cx - 0.5, cx + 0.5, cy - 0.5, cy + 0.5, epsabs=1e-11, epsrel=1e-11)
    return v


def test_supersampling_converges_to_exact_cell_volume():
    R = 2.3
    for cell in [(1.7, 0.4, 0.9), (0.2, -2.1, 0.3), (1.1, 1.3, 0.8), (-1.9, 0.6, -0.7)]:
        exact = _cube_sphere_volume(*cell, R)
        errs = []
        for n in (16, 64):
            cnt = geo.eps_flat_counts(np.array([cell[0]]), np.array([cell[1]]), np.array([cell[2]]), R, n)[0]
            errs.append(abs(cnt / n ** 3 - exact))
        # a sample point is misclassified only within half a sample diagonal of the
        # surface: error <= (surface area in the cell <= 3) * sqrt(3)/(2n)
        assert errs[0] <= 3 * math.sqrt(3) / 32
        assert errs[1] <= 3 * math.sqrt(3) / 128
        assert errs[1] < 0.02


def test_total_solid_fraction_is_sphere_volume():
    R, n = 4.0, 8
    X = np.array([12.31, 11.77, 12.05])
    iz, iy, ix, eps = geo.overlap_cells((24, 24, 24), X, R, n)
    V = 4.0 / 3.0 * math.pi * R ** 3
    r = R * n  # sphere radius in units of the sample spacing
    # lattice-point count in a ball deviates from its volume by O(r^1.5)
    assert abs(eps.sum() - V) / V < 3 * r ** 1.5 / (4.0 / 3.0 * math.pi * r ** 3)


def test_symmetric_face_neighbours():
    R = 1.7
    X = np.array([8.5, 8.5, 8.5])  # a cell centre
    iz, iy, ix, eps = geo.overlap_cells((16, 16, 16), X, R, 8)
    e = {(z, y, x): v for z, y, x, v in zip(iz, iy, ix, eps)}
    faces = [e[(8, 8, 9)], e[(8, 8, 7)], e[(8, 9, 8)], e[(8, 7, 8)], e[(9, 8, 8)], e[(7, 8, 8)]]
    assert len(set(faces)) == 1
    assert e[(8, 8, 8)] == 1.0


# --------------------------------------------------------------------------- rigid body
def test_rigid_euler_constant_force_closed_form():
    X0 = np.array([5.0, 6.0, 7.0])
    U0 = np.array([1e-3, -2e-3, 0.0])
    Om0 = np.array([0.0, 1e-4, 0.0])
    F = np.array([1e-3, 2e-3, -3e-3])
    T = np.array([2e-4, 0.0, -1e-4])
    D, rho, dt = 6.0, 1.3, 2.0
    X, U, Om = X0.copy(), U0.copy(), Om0.copy()
    n = 25
    for _ in range(n):
        X, U, Om = rb.euler_step(X, U, Om, F, T, D, rho, np.zeros(3), np.zeros(3), dt, (100.0, 100.0, 100.0))
    m = rho * math.pi * D ** 3 / 6.0
    inertia = m * D * D / 10.0
    assert np.abs(U - (U0 + n * dt * F / m)).max() < 1e-15
    assert np.abs(X - (X0 + n * dt * U0 + dt * dt * F / m * n * (n - 1) / 2)).max() < 1e-13
    assert np.abs(Om - (Om0 + n * dt * T / inertia)).max() < 1e-16


@pytest.mark.parametrize("coupling", ["mem_bb", "mem_cli", "psm"])
def test_first_rigid_step_from_rest_is_reduced_gravity(coupling):
    # A sphere released from rest in fluid at rest feels no hydrodynamic force
    # in the first rigid-body step (f = w everywhere: no link force, and every
    # solid operator vanishes), so the explicit Euler step gives the reduced
    # gravity of Archimedes (Sec. 4.1): U_1 = dt (1 - rho_f/rho_p) g, X_1 = X_0;
    # the next step moves X by dt U_1.  (A sphere weighed with rho_p instead of
    # rho_p - rho_f, or without the fluid's buoyancy, fails.)
    g = np.array([1e-4, -2e-4, -3e-4])
    rho_p = 1.4
    s = OracleSim(18, 18, 18, nu=0.05, collision="trt", coupling=coupling, psm_m=3, psm_b=2, gravity=g, n_sub=2,
                  eps_n=4)
    s.init_equilibrium()
    X0 = np.array([9.3, 8.8, 9.1])
    s.set_particles([X0], [[0, 0, 0]], [[0, 0, 0]], [6.0], [rho_p], [False])
    s.step(2)
    P = s.particles()
    assert np.abs(P["F"]).max() == 0.0
    U1 = 2.0 * (1.0 - 1.0 / rho_p) * g
    assert np.abs(P["U"][0] - U1).max() < 1e-19
    assert np.array_equal(P["X"][0], X0)
    s.step(2)
    assert np.abs(s.particles()["X"][0] - (X0 + 2.0 * U1)).max() < 1e-15


def test_first_psm_step_from_rest_includes_body_force_buoyancy():
    # PSM with one sweep per rigid-body step: the solid operators read the
    # pre-collision PDFs, which are at rest in the first sweep, so the first
    # step's hydrodynamic force is zero and U_1 = [(rho_p - 1) V g + V f_ext]/m:
    # the fluid body force acts on the sphere's volume as on the fluid it
    # displaces (the buoyancy of Sec. 3's F_b); without it, U_1 = (1 - 1/rho_p) g.
    g = np.array([0.0, 0.0, -3e-4])
    f = np.array([2e-5, 0.0, 1e-4])
    rho_p = 1.25
    s = OracleSim(18, 18, 18, nu=0.05, collision="bgk", coupling="psm", psm_m=2, psm_b=2, gravity=g, fext=f,
                  n_sub=1, eps_n=4)
    s.init_equilibrium()
    s.set_particles([[9.3, 8.8, 9.1]], [[0, 0, 0]], [[0, 0, 0]], [6.0], [rho_p], [False])
    s.step(1)
    P = s.particles()
    assert np.abs(P["F"]).max() == 0.0
    assert np.abs(P["U"][0] - ((1.0 - 1.0 / rho_p) * g + f / rho_p)).max() < 1e-19


# --------------------------------------------------------------------------- MEM
def _mem_sim(scheme, nu=0.05, fext=(1e-5, 0, 0), n_sub=2, X=(8.3, 7.9, 8.2), U=(0, 0, 0), D=7.0):
    s = OracleSim(16, 16, 16, nu=nu, collision="trt", coupling=scheme, fext=fext, n_sub=n_sub)
    s.init_equilibrium()
    s.set_particles([X], [U], [[0, 0, 0]], [D], [1.5], [True])
    return s


def test_cli_at_half_delta_is_bounce_back_bitwise():
    a = _mem_sim("mem_bb")
    b = _mem_sim("mem_cli")
    b.links["delta"][:] = 0.5
    g0 = 1e-3 * RNG.standard_normal(a.g.shape)
    a.set_pdfs(g0)
    b.set_pdfs(g0)
    a.step(4)
    b.step(4)
    assert np.array_equal(a.g, b.g)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.T, b.T)


@pytest.mark.parametrize("scheme", ["mem_bb", "mem_cli"])
def test_comoving_uniform_flow_is_fixed_point(scheme):
    V = np.array([0.02, -0.01, 0.015])
    s = _mem_sim(scheme, fext=(0, 0, 0), U=V)
    g0 = fl.geq(np.zeros(s.shape), V.reshape(3, 1, 1, 1) * np.ones((3,) + s.shape))
    s.set_pdfs(g0)
    fluid = s.owner == mm.FLUID
    s.step(4)
    assert np.abs(s.g[:, fluid] - g0[:, fluid]).max() < 1e-16
    assert np.abs(s.F).max() < 1e-14


@pytest.mark.parametrize("scheme", ["mem_bb", "mem_cli"])
def test_mem_momentum_identity(scheme):
    # fixed sphere (v = 0): per sweep the fluid gains N_fluid f_ext and loses the link force
    s = _mem_sim(scheme, n_sub=1)
    g0 = 1e-3 * RNG.standard_normal(s.g.shape)
    s.set_pdfs(g0)
    fluid = s.owner == mm.FLUID
    for _ in range(3):
        P0 = np.einsum("qa,qn->a", CF, s.g[:, fluid])
        s.step(1)
        P1 = np.einsum("qa,qn->a", CF, s.g[:, fluid])
        expect = fluid.sum() * s.fext - s.F[0]
        # rounding of ~10^3 full-f link terms of size ~0.1: a few 1e-15 absolute
        assert np.abs((P1 - P0) - expect).max() < 1e-12 * np.abs(s.F[0]).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_constant_link_force_part_cancels(seed):
    # the 2 w_q c_q part of Eq. MEM_Force cancels over a closed body: exactly for the
    # force (integer link counts per direction), to rounding for the torque
    rng = np.random.default_rng(seed)
    s = _mem_sim("mem_cli", X=tuple(rng.uniform(6, 10, 3)), D=rng.uniform(4, 9))
    L = s.links
    cnt = np.bincount(L["q"], minlength=19)
    assert np.array_equal(cnt, cnt[OPP])
    c = CF[L["q"]]
    const = 2.0 * W[L["q"]][:, None] * c
    for delta in (np.full(len(L["q"]), 0.5), L["delta"]):
        arm = L["d"] + delta[:, None] * c
        assert np.abs(np.cross(arm, const).sum(0)).max() < 1e-13


# --------------------------------------------------------------------------- refill
def _refill_setup():
    shape = (12, 12, 12)
    owner = np.full(shape, mm.FLUID)
    newmask = np.zeros(shape, bool)
    cell = (6, 6, 3)  # (iz, iy, ix): normal towards -x from a sphere centred at larger x
    Xp = np.array([8.5, 6.5, 6.5])
    return shape, owner, newmask, cell, Xp


def test_refill_quadratic_extrapolation_exact_up_to_momentum():
    shape, owner, newmask, cell, Xp = _refill_setup()
    newmask[cell] = True
    ix = np.arange(12, dtype=float)
    coef = RNG.standard_normal((3, Q)) * 1e-3
    g = np.zeros((Q,) + shape)
    for q in range(Q):
        g[q] = (coef[0, q] + coef[1, q] * ix + coef[2, q] * ix * ix)[None, None, :]
    Up, Omp, f = np.array([0.01, 0.0, -0.02]), np.array([0.0, 1e-3, 0.0]), np.array([1e-5, 0, 0])
    out = mm.refill_cell(g, owner, newmask, cell, Xp, Up, Omp, f, shape)
    exact = g[:, 6, 6, 3]
    diff = out - exact
    # momentum set to j* = v - f/2, density and every moment orthogonal to c_a unchanged
    d = np.array([3.5 - 8.5, 0.0, 0.0])
    v = rb.surface_velocity(Up, Omp, d)
    assert np.abs(CF.T @ out - (v - 0.5 * f)).max() < 1e-17
    assert abs(diff.sum()) < 1e-17
    proj = CF @ np.linalg.lstsq(CF, diff, rcond=None)[0]
    assert np.abs(diff - proj).max() < 1e-17


def test_equilibrium_refill_is_equilibrium_of_mean_neighbour_density():
    # the equilibrium reconstruction: f^eq(rho_bar, v) with rho_bar the mean
    # density of the old-fluid neighbours (counted by brute force here), then
    # the velocity constraint, which with f_ext = 0 changes nothing
    shape, owner, newmask, cell, Xp = _refill_setup()
    newmask[cell] = True
    owner[6, 7, 3] = 4  # one solid neighbour, one more newly uncovered one
    newmask[5, 6, 3] = True
    g = 1e-3 * RNG.standard_normal((Q,) + shape)
    Up, Omp = np.array([0.01, 0.0, -0.02]), np.array([0.0, 1e-3, 0.0])
    out = mm.refill_cell(g, owner, newmask, cell, Xp, Up, Omp, np.zeros(3), shape, equilibrium=True)
    drhos = []
    for q in range(1, Q):
        z, y, x = (cell[0] + C[q, 2]) % 12, (cell[1] + C[q, 1]) % 12, (cell[2] + C[q, 0]) % 12
        if owner[z, y, x] == mm.FLUID and not newmask[z, y, x]:
            drhos.append(g[:, z, y, x].sum())
    assert len(drhos) == 16
    d = np.array([cell[2] + 0.5 - Xp[0], cell[1] + 0.5 - Xp[1], cell[0] + 0.5 - Xp[2]])
    v = Up + np.cross(Omp, d)
    w = W
    cu = C @ v
    expect = w * (np.mean(drhos) + 3 * cu + 4.5 * cu * cu - 1.5 * (v @ v))
    assert np.abs(out - expect).max() < 1e-17


def test_refill_linear_fallback_exact_for_linear_field():
    shape, owner, newmask, cell, Xp = _refill_setup()
    newmask[cell] = True
    owner[6, 6, 0] = 5  # third source cell is solid -> linear extrapolation
    ix = np.arange(12, dtype=float)
    coef = RNG.standard_normal((2, Q)) * 1e-3
    g = np.zeros((Q,) + shape)
    for q in range(Q):
        g[q] = (coef[0, q] + coef[1, q] * ix)[None, None, :]
    out = mm.refill_cell(g, owner, newmask, cell, Xp, np.zeros(3), np.zeros(3), np.zeros(3), shape)
    diff = out - g[:, 6, 6, 3]
    proj = CF @ np.linalg.lstsq(CF, diff, rcond=None)[0]
    assert np.abs(diff - proj).max() < 1e-17 and abs(diff.sum()) < 1e-17


# --------------------------------------------------------------------------- PSM
def _psm_sim(m, b, coll="bgk", nu=0.05, U=(0, 0, 0), Om=(0, 0, 0), fext=(1e-5, 0, 0)):
    s = OracleSim(16, 16, 16, nu=nu, collision=coll, coupling="psm", psm_m=m, psm_b=b, fext=fext, eps_n=4)
    s.init_equilibrium()
    s.set_particles([[8.3, 7.9, 8.2]], [U], [Om], [7.0], [1.5], [True])
    return s


@pytest.mark.parametrize("coll", ["bgk", "trt"])
def test_psm_without_particles_is_fluid_sweep_bitwise(coll):
    a = OracleSim(10, 8, 6, nu=0.07, collision=coll, coupling="psm", fext=(1e-5, 2e-5, 0))
    b = OracleSim(10, 8, 6, nu=0.07, collision=coll, coupling="none", fext=(1e-5, 2e-5, 0))
    g0 = 1e-3 * RNG.standard_normal(a.g.shape)
    a.set_pdfs(g0)
    b.set_pdfs(g0)
    a.set_particles([], [], [], [], [], [])
    a.step(3)
    b.step(3)
    assert np.array_equal(a.g, b.g)


@pytest.mark.parametrize("m,k", [(1, 1), (2, 1), (3, 2)])
def test_solid_operator_mass_and_closed_form_force(m, k):
    n = 40
    g = 1e-2 * RNG.standard_normal((Q, n))
    rho, U = fl.moments(g)
    vs = 0.02 * RNG.standard_normal((3, n))
    om = ps.solid_operator(g, rho, U, vs, 0.8, m)
    # operands are ~1e-2: 19-term sums carry a few 1e-17 of rounding
    assert np.abs(om.sum(0)).max() < 1e-15
    mom = -(CF.T @ om)  # sum_q Omega_q c_qbar
    assert np.abs(mom - k * (U - vs)).max() < 1e-15


def test_m2_with_solid_at_fluid_velocity_is_bgk():
    # Eq. PSM_M2 with v_s = U: the bracket (1 - 1/tau)[f - f^eq(rho, U)] and
    # f^eq(rho, v_s) - f combine to (f^eq - f)/tau, the BGK operator of
    # Eq. LBM_SRT (a wrong coefficient on the bracket, e.g. 1 - tau or 1/tau,
    # gives another multiple of f^eq - f)
    n = 30
    g = 1e-2 * RNG.standard_normal((Q, n))
    rho, U = fl.moments(g)
    for tau in (0.6, 0.8, 1.7):
        om = ps.solid_operator(g, rho, U, U, tau, 2)
        # operands ~1e-2: a few units in the last place of rounding
        assert np.abs(om - (fl.geq(rho, U) - g) / tau).max() < 1e-16


@pytest.mark.parametrize("coll", ["bgk", "trt"])
def test_fully_covered_m2b2_cell_relaxes_as_bgk(coll):
    # Through the whole PSM step: a cell inside the sphere has eps_s = 1, so
    # B2 = 1 (Eq. PSM_B2) and Eq. LBM_Collide_PSM keeps only the solid term;
    # with the particle moving at that cell's fluid velocity, M2 is BGK there
    # (without the forcing, which is weighted by 1 - B = 0), whatever the fluid
    # operator.  Pins B2 at eps = 1, the (1 - B) weights and M2's coefficient.
    s = OracleSim(16, 16, 16, nu=0.1, collision=coll, coupling="psm", psm_m=2, psm_b=2, fext=(1e-5, 2e-5, 0),
                  eps_n=4)
    g0 = 1e-3 * RNG.standard_normal((Q, 16, 16, 16))
    rho, U = fl.moments(g0)
    cell = (8, 8, 8)  # (z, y, x): centre (8.5, 8.5, 8.5), 0.43 from the sphere centre
    s.set_particles([[8.3, 7.9, 8.2]], [U[:, 8, 8, 8]], [[0, 0, 0]], [7.0], [1.5], [True])
    iz, iy, ix, eps = s.overlaps[0]
    k = np.nonzero((iz == 8) & (iy == 8) & (ix == 8))[0]
    assert len(k) == 1 and eps[k[0]] == 1.0
    gt, F, T, B, vB = ps.psm_collide(g0, s.overlaps, s.parts, coll, s.tau, s.magic, s.fext, 2, 2)
    assert B[cell] == 1.0
    expect = g0[:, 8, 8, 8] + (fl.geq(rho, U)[:, 8, 8, 8] - g0[:, 8, 8, 8]) / s.tau
    assert np.abs(gt[:, 8, 8, 8] - expect).max() < 1e-17


@pytest.mark.parametrize("m,b", [(1, 1), (2, 2), (3, 2)])
def test_psm_force_torque_closed_form(m, b):
    s = _psm_sim(m, b, U=(1e-3, 0, -2e-3), Om=(0, 1e-4, 2e-4))
    g0 = 1e-3 * RNG.standard_normal(s.g.shape)
    s.set_pdfs(g0)
    rho, U = fl.moments(s.g)
    k = 2.0 if m == 3 else 1.0
    iz, iy, ix, eps = s.overlaps[0]
    Bs = ps.weight(eps, s.tau, b)
    p = s.parts[0]
    r = np.stack([geo.centre_disp(ix, p["X"][0], 16), geo.centre_disp(iy, p["X"][1], 16),
                  geo.centre_disp(iz, p["X"][2], 16)], -1)
    vs = rb.surface_velocity(p["U"], p["Om"], r)
    fc = k * Bs[:, None] * (U[:, iz, iy, ix].T - vs)
    s.step(1)
    assert np.abs(s.F[0] - fc.sum(0)).max() < 1e-15
    assert np.abs(s.T[0] - np.cross(r, fc).sum(0)).max() < 1e-14


@pytest.mark.parametrize("m,b", [(1, 1), (2, 2), (3, 2)])
def test_psm_comoving_uniform_flow_is_fixed_point(m, b):
    V = np.array([0.02, 0.01, -0.01])
    s = _psm_sim(m, b, U=V, fext=(0, 0, 0))
    g0 = fl.geq(np.zeros(s.shape), V.reshape(3, 1, 1, 1) * np.ones((3,) + s.shape))
    s.set_pdfs(g0)
    s.step(2)
    assert np.abs(s.g - g0).max() < 1e-17
    assert np.abs(s.F).max() < 1e-15


@pytest.mark.parametrize("m,b", [(1, 1), (2, 2), (3, 2)])
def test_psm_momentum_identity(m, b):
    s = _psm_sim(m, b)
    s.set_pdfs(1e-3 * RNG.standard_normal(s.g.shape))
    P0 = np.einsum("qa,qzyx->a", CF, s.g)
    iz, iy, ix, eps = s.overlaps[0]
    B = np.zeros(s.shape)
    B[iz, iy, ix] = ps.weight(eps, s.tau, b)
    s.step(1)
    P1 = np.einsum("qa,qzyx->a", CF, s.g)
    expect = (1.0 - B).sum() * s.fext - s.F[0]
    assert np.abs((P1 - P0) - expect).max() < 1e-14


def test_psm_is_bgk_with_modified_relaxation_time():
    # Sec. 4.6: (1-B) C^BGK = (f^eq - f)/tau_PSM with tau_PSM = tau/(1-B)
    s = _psm_sim(3, 2)
    g = 1e-3 * RNG.standard_normal(s.g.shape)
    gt, F, T, B, vB = ps.psm_collide(g, s.overlaps, s.parts, "bgk", s.tau, s.magic, s.fext, 3, 2)
    rho, U = fl.moments(g)
    solid_sum = gt - (g + (1 - B) * fl.fluid_operator(g, rho, U, "bgk", s.tau, s.magic) + (1 - B) * fl.forcing(U, s.fext))
    mask = B < 1.0
    tau_psm = s.tau / (1.0 - B[mask])
    alt = g[:, mask] + (fl.geq(rho, U)[:, mask] - g[:, mask]) / tau_psm + solid_sum[:, mask] + \
        (1 - B[mask]) * fl.forcing(U, s.fext)[:, mask]
    assert np.abs(alt - gt[:, mask]).max() < 1e-17
