"""Time-stepping drivers: Alg. 1 (LBM with momentum exchange coupling) and
Alg. 2 (LBM with partially saturated cells coupling), FP64, plain and literal.

State: the canonical PDFs f(x, t) (post-stream, post-boundary, pre-collision)
held as deviations g = f - w.  Solid MEM cells are not updated and are reported
as g = 0.

One call of ``step(n)`` advances n LBM time steps:
* MEM: in groups of n_sub sweeps (n must be a multiple of n_sub), each sweep =
  collide (fluid cells) -> stream -> BB/CLI on every link -> link forces; the
  forces are averaged over the n_sub sweeps, the rigid bodies advance with
  dt = n_sub, and the particle mapping is updated with refill of uncovered cells.
* PSM: every sweep = solid fractions from the current positions -> PSM collide
  -> stream -> force/torque; every n_sub sweeps (default 1, Alg. 2) the forces
  are averaged, the rigid bodies advance with dt = n_sub and the solid
  fractions are recomputed.  (Sec. 4.1 obtains the sphere forces of the
  settling benchmark from two averaged subcycles; with M3, whose force is
  2 sum B (U - v), a single sweep per rigid-body step makes the fluid inside
  fully covered cells and the sphere exchange an alternating momentum that
  grows by (1 + 2 rho_f/rho_p) per step, so moving M3 runs use n_sub = 2.)
* none: collide -> stream.
Static walls (half-way bounce-back with a wall velocity, or the outflow rule of
the settling-sphere frame, Sec. 4.1) are applied after the stream in every mode.
"""
import numpy as np

from . import fluid as fl
from . import geometry as geo
from . import mem as mm
from . import psm as ps
from . import rigid as rb


class OracleSim:
    def __init__(self, nx, ny, nz, nu, collision="trt", magic=3.0 / 16.0, coupling="none",
                 psm_m=1, psm_b=1, fext=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0), n_sub=None,
                 eps_n=8, eps_recursive=False, eps_estimator=None, refill="extrapolation"):
        self.shape = (nz, ny, nx)
        self.box = np.array([nx, ny, nz], dtype=np.float64)
        self.nu = float(nu)
        self.tau = fl.tau_from_nu(nu)
        self.collision = collision
        self.magic = float(magic)
        self.coupling = coupling
        self.msel, self.bsel = psm_m, psm_b
        self.fext = np.asarray(fext, dtype=np.float64)
        self.gravity = np.asarray(gravity, dtype=np.float64)
        if n_sub is None:
            n_sub = 2 if coupling.startswith("mem") else 1
        self.n_sub = n_sub
        self.eps_n = eps_n
        self.eps_recursive = eps_recursive
        self.eps_estimator = eps_estimator  # None (supersampling), 'edge' or 'distance'
        self.refill_equilibrium = refill == "equilibrium"  # else the extrapolation of Sec. 2.2.3
        self.g = np.zeros((19,) + self.shape)
        self.owner = np.full(self.shape, mm.FLUID, dtype=np.int64)
        self.v_walls = []
        self.wall_outflow = []  # per wall group: None (velocity wall) or rho_out (outflow)
        self.parts = []
        self.F = np.zeros((0, 3))
        self.T = np.zeros((0, 3))
        self.links = None
        self.overlaps = []
        self._remap(initial=True)
        self.time = 0
        self.refilled = 0

    # --- set-up -------------------------------------------------------------
    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        U = np.asarray(u, dtype=np.float64).reshape(3, 1, 1, 1) * np.ones((3,) + self.shape)
        self.g = fl.geq(np.full(self.shape, float(rho) - 1.0), U)
        self._mask_solid()

    def set_pdfs(self, g):
        self.g = np.array(g, dtype=np.float64).reshape((19,) + self.shape)
        self._mask_solid()

    def get_pdfs(self):
        return self.g.copy()

    def set_static_solid(self, mask, v_wall=(0.0, 0.0, 0.0)):
        """Add one group of static wall cells moving with velocity v_wall
        (half-way bounce-back, Eq. MEM_BB)."""
        self.owner[np.asarray(mask, dtype=bool)] = mm.WALL - len(self.v_walls)
        self.v_walls.append(np.asarray(v_wall, dtype=np.float64))
        self.wall_outflow.append(None)
        self._remap(initial=True)

    def set_outflow(self, mask, rho_out=1.0):
        """Add one group of outflow cells: the fluid cells next to them get the
        pressure anti-bounce-back of Sec. 4.1 with density rho_out."""
        self.owner[np.asarray(mask, dtype=bool)] = mm.WALL - len(self.v_walls)
        self.v_walls.append(np.zeros(3))
        self.wall_outflow.append(float(rho_out))
        self._remap(initial=True)

    def set_viscosity(self, nu):
        """New kinematic viscosity (Eq. Viscosity gives tau); the calibration
        of Sec. 4.1 adjusts it between runs."""
        self.nu = float(nu)
        self.tau = fl.tau_from_nu(nu)

    def set_gravity(self, g):
        self.gravity = np.asarray(g, dtype=np.float64)

    def set_particles(self, X, U, Om, D, rho_p, fixed):
        self.parts = []
        for i in range(len(D)):
            self.parts.append(dict(X=np.mod(np.asarray(X[i], dtype=np.float64), self.box),
                                   U=np.asarray(U[i], dtype=np.float64),
                                   Om=np.asarray(Om[i], dtype=np.float64), D=float(D[i]),
                                   rho=float(rho_p[i]), fixed=bool(fixed[i])))
        P = len(self.parts)
        self.F = np.zeros((P, 3))
        self.T = np.zeros((P, 3))
        self._remap(initial=True)

    # --- geometry -----------------------------------------------------------
    def _radii(self):
        return [p["D"] / 2.0 for p in self.parts]

    def _mask_solid(self):
        self.g[:, self.owner != mm.FLUID] = 0.0

    def _remap(self, initial=False):
        """Binary mapping (MEM) or solid fractions (PSM) from current positions."""
        if self.coupling.startswith("mem"):
            old = self.owner.copy()
            new = np.where(old <= mm.WALL, old, mm.FLUID)
            for p, part in enumerate(self.parts):
                m = geo.solid_cells(self.shape, part["X"], part["D"] / 2.0)
                new[m & (new == mm.FLUID)] = p
            self.owner = new
            if not initial:
                newly = (old >= 0) & (new == mm.FLUID)
                cells = np.argwhere(newly)
                gnew = self.g.copy()
                for (iz, iy, ix) in cells:
                    p = old[iz, iy, ix]
                    part = self.parts[p]
                    gnew[:, iz, iy, ix] = mm.refill_cell(self.g, new, newly, (iz, iy, ix), part["X"], part["U"],
                                                         part["Om"], self.fext, self.shape,
                                                         equilibrium=self.refill_equilibrium)
                self.g = gnew
                self.refilled += len(cells)
            self._mask_solid()
        else:
            self.overlaps = [geo.overlap_cells(self.shape, p["X"], p["D"] / 2.0, self.eps_n, self.eps_recursive,
                                              self.eps_estimator)
                             for p in self.parts]
        self.links = mm.build_links(self.owner, self.parts, self._radii(), self.shape, self.v_walls,
                                    self.wall_outflow)
        if self.coupling.startswith("mem"):
            mm.check_link_balance(self.links, len(self.parts))

    # --- sweeps -------------------------------------------------------------
    def _sweep_mem(self):
        gt = fl.collide(self.g, self.collision, self.tau, self.magic, self.fext)
        gn = fl.stream(gt)
        scheme = "cli" if self.coupling == "mem_cli" else "bb"
        Fq, Tq = mm.link_boundary(gt, gn, self.links, scheme, self.g, self.fext)
        P = len(self.parts)
        F = np.zeros((P, 3))
        T = np.zeros((P, 3))
        for p in range(P):
            s = self.links["p"] == p
            F[p] = Fq[s].sum(axis=0)
            T[p] = Tq[s].sum(axis=0)
        self.g = gn
        self._mask_solid()
        return F, T

    def _sweep_psm(self):
        gt, F, T, self._B, self._vB = ps.psm_collide(self.g, self.overlaps, self.parts, self.collision, self.tau,
                                                     self.magic, self.fext, self.msel, self.bsel)
        gn = fl.stream(gt)
        if len(self.links["q"]):
            mm.link_boundary(gt, gn, self.links, "bb", self.g, self.fext)
        self.g = gn
        return F, T

    def _sweep_fluid(self):
        gt = fl.collide(self.g, self.collision, self.tau, self.magic, self.fext)
        gn = fl.stream(gt)
        if len(self.links["q"]):
            mm.link_boundary(gt, gn, self.links, "bb", self.g, self.fext)
        self.g = gn
        self._mask_solid()

    def _rigid(self, dt):
        moved = False
        for p, part in enumerate(self.parts):
            if part["fixed"]:
                continue
            part["X"], part["U"], part["Om"] = rb.euler_step(part["X"], part["U"], part["Om"], self.F[p], self.T[p],
                                                             part["D"], part["rho"], self.gravity, self.fext, dt,
                                                             self.box)
            moved = True
        return moved

    def step(self, n):
        if self.coupling == "none":
            for _ in range(n):
                self._sweep_fluid()
                self.time += 1
            return
        if self.coupling.startswith("mem"):
            assert n % self.n_sub == 0, "MEM steps must be a multiple of n_sub"
            for _ in range(n // self.n_sub):
                P = len(self.parts)
                Fs, Ts = np.zeros((P, 3)), np.zeros((P, 3))
                for _s in range(self.n_sub):
                    F, T = self._sweep_mem()
                    Fs += F
                    Ts += T
                    self.time += 1
                self.F, self.T = Fs / self.n_sub, Ts / self.n_sub
                if self._rigid(float(self.n_sub)):
                    self._remap()
            return
        assert n % self.n_sub == 0, "PSM steps must be a multiple of n_sub"
        for _ in range(n // self.n_sub):
            P = len(self.parts)
            Fs, Ts = np.zeros((P, 3)), np.zeros((P, 3))
            for _s in range(self.n_sub):
                F, T = self._sweep_psm()
                Fs += F
                Ts += T
                self.time += 1
            self.F, self.T = Fs / self.n_sub, Ts / self.n_sub
            if self._rigid(float(self.n_sub)):
                self._remap()

    # --- outputs ------------------------------------------------------------
    def particles(self):
        return dict(F=self.F.copy(), T=self.T.copy(),
                    U=np.array([p["U"] for p in self.parts]).reshape(-1, 3),
                    Om=np.array([p["Om"] for p in self.parts]).reshape(-1, 3),
                    X=np.array([p["X"] for p in self.parts]).reshape(-1, 3))

    def fields(self):
        """Density and macroscopic velocity: Eq. MacVel in fluid cells, zero in
        solid MEM cells, Eq. MacVel_PSM with the current solid fractions for PSM."""
        drho, U = fl.moments(self.g)
        rho = 1.0 + drho
        if self.coupling == "psm":
            # B and sum B_s v_s at the current time level
            _, _, _, B, vB = ps.psm_collide(self.g, self.overlaps, self.parts, self.collision, self.tau, self.magic,
                                            self.fext, self.msel, self.bsel)
            u = ps.psm_velocity(U, self.fext, B, vB)
        else:
            u = fl.macroscopic_velocity(U, self.fext)
        solid = self.owner != mm.FLUID
        rho = np.where(solid, 1.0, rho)
        u[:, solid] = 0.0
        return rho, u
