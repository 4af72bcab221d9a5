"""Pins of the oracle's settling-sphere frame boundaries (Sec. 4.1): the
velocity inflow (bounce-back with the inflow velocity, Eq. MEM_BB) at the
bottom and the pressure outflow (anti-bounce-back with f^eq,+(rho_out, u)) at
the top, periodic in x and y.  Pure CPU."""
import numpy as np
import pytest

from oracle import fluid as fl
from oracle.lattice import C, W
from oracle.sim import OracleSim


def _channel(nx, ny, nz, u, rho_out=1.0, nu=0.1, collision="trt"):
    s = OracleSim(nx, ny, nz, nu, collision=collision, coupling="none")
    inflow = np.zeros((nz, ny, nx), bool)
    inflow[0] = True
    out = np.zeros((nz, ny, nx), bool)
    out[-1] = True
    s.set_static_solid(inflow, (0.0, 0.0, u))
    s.set_outflow(out, rho_out)
    return s


@pytest.mark.parametrize("collision", ["trt", "bgk"])
def test_plug_flow_is_a_fixed_point(collision):
    # uniform f^eq(rho_out, u_inf): the inflow rule returns f^eq_qbar
    # (f^eq_qbar - f^eq_q = -6 w_q c_q.u) and so does the outflow rule
    # (-f^eq_q + 2 f^eq,+_q = f^eq,+_q - f^eq,-_q = f^eq_qbar)
    u = 0.04
    for rho_out in (1.0, 1.02):
        s = _channel(6, 5, 14, u, rho_out, collision=collision)
        s.init_equilibrium(rho_out, (0.0, 0.0, u))
        g0 = s.g.copy()
        s.step(30)
        fluid = s.owner == -1
        assert np.abs(s.g[:, fluid] - g0[:, fluid]).max() < 1e-16


def test_perturbed_channel_returns_to_plug_flow_at_outflow_density():
    # from a perturbed state at density 1, the channel relaxes to the plug flow
    # with the outflow's density rho_out (the inflow fixes the velocity only)
    u, rho_out = 0.03, 1.01
    s = _channel(8, 8, 18, u, rho_out)
    s.init_equilibrium(1.0, (0.0, 0.0, u))
    rng = np.random.default_rng(3)
    s.set_pdfs(s.g + 1e-4 * rng.standard_normal(s.g.shape))
    s.step(6000)
    fluid = s.owner == -1
    ones = np.ones((3,) + s.shape)
    target = fl.geq(np.full(s.shape, rho_out - 1.0), np.array([0.0, 0.0, u]).reshape(3, 1, 1, 1) * ones)
    assert np.abs(s.g[:, fluid] - target[:, fluid]).max() < 1e-9


def test_mass_flux_through_every_plane_equals_inflow_at_steady_state():
    # With an obstacle in the channel, at steady state the mass crossing every
    # half plane between two fluid planes per step (populations moving up
    # minus populations moving down, between fluid cells) equals the inflow:
    # the inflow rule lets u_inf per cell and step into the box (its
    # populations with c_z = +1 exceed the reflected ones by 6 w_q u_inf, and
    # sum_{c_z = 1} w_q = 1/6), and no mass is created or lost elsewhere,
    # the outflow included.
    u = 0.02
    nx, ny, nz = 8, 8, 16
    s = _channel(nx, ny, nz, u, 1.0, nu=0.1)
    block = np.zeros((nz, ny, nx), bool)
    block[7:9, 3:5, 2:5] = True
    s.set_static_solid(block, (0.0, 0.0, 0.0))
    s.init_equilibrium(1.0, (0.0, 0.0, u))
    s.step(5000)
    fluid = s.owner == -1
    f = s.g + W.reshape(19, 1, 1, 1)
    for z in range(1, nz - 2):  # the half plane between z and z + 1
        flux = 0.0
        for q in range(19):
            cx, cy, cz = (int(v) for v in C[q])
            if cz == 0:
                continue
            pair = np.roll(fluid, shift=(cz, cy, cx), axis=(0, 1, 2)) & fluid  # x - c_q and x fluid
            if cz == 1:
                flux += f[q, z + 1][pair[z + 1]].sum()
            else:
                flux -= f[q, z][pair[z]].sum()
        assert abs(flux / (u * nx * ny) - 1.0) < 1e-11, z
