"""Pins of the oracle's fluid core (Sec. 2.1) against closed forms, invariants
and analytic flows.  Pure CPU."""
import math

import numpy as np
import pytest

from oracle import fluid as fl
from oracle.lattice import C, CF, W, OPP, Q
from oracle.sim import OracleSim

RNG = np.random.default_rng(1234)


def test_lattice_isotropy():
    # sum w = 1, sum w c = 0, sum w c c = I/3, 4th-order isotropy = delta-delta/9
    assert abs(W.sum() - 1.0) < 1e-15
    assert np.abs(W @ CF).max() == 0.0
    M2 = np.einsum("q,qa,qb->ab", W, CF, CF)
    assert np.abs(M2 - np.eye(3) / 3.0).max() < 1e-15
    M4 = np.einsum("q,qa,qb,qc,qd->abcd", W, CF, CF, CF, CF)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(M4 - iso).max() < 1e-15
    assert (OPP[OPP] == np.arange(Q)).all()
    assert (C[OPP] == -C).all()
    assert sorted((C * C).sum(1).tolist()) == [0] + [1] * 6 + [2] * 12


def _rand_state(n, scale=1e-2):
    g = scale * RNG.standard_normal((Q, n))
    return g


def test_equilibrium_moments():
    rho = 1.0 + 0.01 * RNG.standard_normal(50)
    U = 0.05 * RNG.standard_normal((3, 50))
    ge = fl.geq(rho - 1.0, U)
    feq = ge + W[:, None]
    assert np.abs(feq.sum(0) - rho).max() < 1e-15
    assert np.abs(CF.T @ feq - U).max() < 1e-15
    Pi = np.einsum("qa,qb,qn->abn", CF, CF, feq)
    exact = rho[None, None, :] / 3.0 * np.eye(3)[:, :, None] + U[:, None, :] * U[None, :, :]
    assert np.abs(Pi - exact).max() < 1e-15


def test_forcing_moments():
    U = 0.05 * RNG.standard_normal((3, 40))
    f = np.array([1e-3, -2e-3, 5e-4])
    F = fl.forcing(U, f)
    assert np.abs(F.sum(0)).max() < 1e-18
    assert np.abs(CF.T @ F - f[:, None]).max() < 1e-18
    Pi = np.einsum("qa,qb,qn->abn", CF, CF, F)
    exact = U[:, None, :] * f[None, :, None] + f[:, None, None] * U[None, :, :]
    assert np.abs(Pi - exact).max() < 1e-18


@pytest.mark.parametrize("coll", ["bgk", "trt"])
def test_collision_conservation_and_fixed_point(coll):
    g = _rand_state(64)
    f = np.array([1e-4, 2e-4, -3e-4])
    tau = 0.73
    gt = fl.collide(g, coll, tau, 3.0 / 16.0, f)
    rho0, U0 = fl.moments(g)
    rho1, U1 = fl.moments(gt)
    assert np.abs(rho1 - rho0).max() < 1e-15
    assert np.abs(U1 - U0 - f[:, None]).max() < 1e-15
    # equilibrium is a fixed point without forcing
    drho = 0.01 * RNG.standard_normal(64)
    U = 0.03 * RNG.standard_normal((3, 64))
    ge = fl.geq(drho, U)
    assert np.abs(fl.collide(ge, coll, tau, 3.0 / 16.0, np.zeros(3)) - ge).max() < 1e-16


def test_trt_relaxes_symmetric_and_antisymmetric_parts():
    g = _rand_state(32)
    tau, magic = 0.9, 3.0 / 16.0
    lp, lm = fl.trt_rates(tau, magic)
    assert abs((0.5 + 1 / lp) * (0.5 + 1 / lm) - magic) < 1e-15
    rho, U = fl.moments(g)
    n = g - fl.geq(rho, U)
    gt = fl.collide_trt(g, lp, lm, np.zeros(3))
    n1 = gt - fl.geq(rho, U)
    sym, anti = 0.5 * (n + n[OPP]), 0.5 * (n - n[OPP])
    sym1, anti1 = 0.5 * (n1 + n1[OPP]), 0.5 * (n1 - n1[OPP])
    assert np.abs(sym1 - (1 + lp) * sym).max() < 1e-16
    assert np.abs(anti1 - (1 + lm) * anti).max() < 1e-16
    # with Lambda = (tau - 1/2)^2 both rates equal -1/tau: TRT is BGK
    lp2, lm2 = fl.trt_rates(tau, (tau - 0.5) ** 2)
    assert abs(lm2 - lp2) < 1e-14
    assert np.abs(fl.collide_trt(g, lp2, lm2, np.zeros(3)) - fl.collide_bgk(g, tau, np.zeros(3))).max() < 1e-16


def test_stream_moves_single_population():
    nz, ny, nx = 5, 6, 7
    for q in range(Q):
        gt = np.zeros((Q, nz, ny, nx))
        gt[q, 4, 5, 6] = 1.0  # at the upper corner: every moving velocity wraps
        out = fl.stream(gt)
        z, y, x = (4 + C[q, 2]) % nz, (5 + C[q, 1]) % ny, (6 + C[q, 0]) % nx
        assert out[q, z, y, x] == 1.0 and out.sum() == 1.0


def test_periodic_momentum_grows_by_body_force():
    s = OracleSim(8, 6, 10, nu=0.05, collision="trt", fext=(1e-5, -2e-5, 3e-5))
    g0 = 1e-3 * RNG.standard_normal((Q, 10, 6, 8))
    s.set_pdfs(g0)
    N = 8 * 6 * 10
    P0 = np.einsum("qa,qzyx->a", CF, s.g)
    M0 = s.g.sum()
    s.step(7)
    P1 = np.einsum("qa,qzyx->a", CF, s.g)
    assert np.abs(P1 - P0 - 7 * N * s.fext).max() < 1e-15 * N * 10
    assert abs(s.g.sum() - M0) < 1e-14


def _shear_wave_nu_error(L, tau, coll):
    nu = (tau - 0.5) / 3.0
    s = OracleSim(4, 4, L, nu=nu, collision=coll)
    z = np.arange(L) + 0.5
    k = 2 * math.pi / L
    u = np.zeros((3, L, 4, 4))
    u[0] = (1e-4 * np.sin(k * z))[:, None, None]
    s.set_pdfs(fl.geq(np.zeros((L, 4, 4)), u))
    amp = []
    t_marks = [int(0.2 * L * L / (nu * 4 * math.pi ** 2)), int(0.7 * L * L / (nu * 4 * math.pi ** 2))]
    t = 0
    for tm in t_marks:
        s.step(tm - t)
        t = tm
        _, uu = s.fields()
        amp.append(2.0 / L * np.sum(uu[0, :, 0, 0] * np.sin(k * z)))
    nu_eff = math.log(amp[0] / amp[1]) / (k * k * (t_marks[1] - t_marks[0]))
    return abs(nu_eff - nu) / nu


def test_shear_wave_viscous_decay_second_order():
    # Eq. Viscosity: a shear wave decays as exp(-nu k^2 t); the lattice error is O(k^2)
    e16 = _shear_wave_nu_error(16, 0.8, "bgk")
    e32 = _shear_wave_nu_error(32, 0.8, "bgk")
    assert e32 < 3e-3
    assert 3.5 < e16 / e32 < 4.5  # second order: halving dx divides the error by ~4


def _channel(coll, tau, H, f=0.0, v_top=0.0, max_steps=20000):
    nu = (tau - 0.5) / 3.0
    nz = H + 2
    s = OracleSim(2, 2, nz, nu=nu, collision=coll, fext=(f, 0.0, 0.0))
    s.init_equilibrium()
    bottom = np.zeros((nz, 2, 2), bool)
    bottom[0] = True
    top = np.zeros((nz, 2, 2), bool)
    top[-1] = True
    s.set_static_solid(bottom, (0.0, 0.0, 0.0))
    s.set_static_solid(top, (v_top, 0.0, 0.0))
    prev = None
    while s.time < max_steps:
        s.step(100)
        ux = s.fields()[1][0, 1:-1, 0, 0]
        if prev is not None and np.abs(ux - prev).max() <= 1e-15 * np.abs(ux).max():
            break
        prev = ux.copy()
    sdist = np.arange(1, H + 1) + 0.5 - 1.0  # distance from the half-way wall at z = 1
    return ux, sdist, nu


@pytest.mark.parametrize("tau", [0.7, 1.4])
def test_poiseuille_exact_with_trt_magic_3_16(tau):
    # half-way bounce-back walls with TRT, Lambda = 3/16 (Sec. 2.1, Sec. 3) place the
    # wall exactly: the discrete Poiseuille profile equals the parabola
    f = 1e-7
    ux, sd, nu = _channel("trt", tau, 10, f=f)
    exact = f / (2 * nu) * sd * (10 - sd)
    assert np.abs(ux - exact).max() / exact.max() < 1e-9


def test_poiseuille_bgk_depends_on_tau():
    # with BGK the wall location moves with tau (Sec. 2.1): error grows with tau
    f = 1e-7
    errs = []
    for tau in (0.8, 1.5):
        ux, sd, nu = _channel("bgk", tau, 10, f=f)
        exact = f / (2 * nu) * sd * (10 - sd)
        errs.append(np.abs(ux - exact).max() / exact.max())
    assert errs[0] > 1e-4 and errs[1] > 3 * errs[0]


@pytest.mark.parametrize("coll", ["bgk", "trt"])
def test_couette_linear_profile_exact(coll):
    # moving-wall bounce-back, Eq. MEM_BB, reproduces the linear Couette profile
    vw = 1e-3
    ux, sd, nu = _channel(coll, 0.9, 8, v_top=vw)
    exact = vw * sd / 8.0
    assert np.abs(ux - exact).max() / vw < 1e-12
