"""Python binding of the lbmps C-ABI (include/lbmps.h): argument marshalling only.

Every computation runs in the HIP library ``liblbmps.so`` built in this
package directory; torch supplies the device workspace and the stream.  If the
library is missing, importing it raises -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmps.so")

BGK, TRT = 0, 1
NONE, MEM_BB, MEM_CLI, PSM = 0, 1, 2, 3
FP64, FP32, FP16_DEV, BF16_DEV = 0, 1, 2, 3
EPS_FLAT, EPS_RECURSIVE, EPS_LEARNED, EPS_EDGE, EPS_DISTANCE = 0, 1, 2, 3, 4
SWEEP_NT_LOADS, SWEEP_PSM_FUSED, SWEEP_PSM_SEPARATE, SWEEP_OCC6, SWEEP_PSM_STAGED = 1, 2, 4, 8, 16
SWEEP_WG_CAP3, SWEEP_WG_CAP2 = 32, 64  # at most three / two sweep workgroups per CU
SWEEP_CELL_PAIRS = 128  # two x-adjacent cells per sweep thread (even nx)
SWEEP_CELL_QUADS = 256  # four x-adjacent cells per sweep thread (FP16/BF16 storage, nx a multiple of 4)
MLP_NPARAM = 4801
MLP_MAX_BATCH = 65536
COUPLING = {"none": NONE, "mem_bb": MEM_BB, "mem_cli": MEM_CLI, "psm": PSM}
PRECISION = {"fp64": FP64, "fp32": FP32, "fp16": FP16_DEV, "bf16": BF16_DEV}
STORAGE_BYTES = {FP64: 8, FP32: 4, FP16_DEV: 2, BF16_DEV: 2}
REFILL_EXTRAPOLATE, REFILL_EQUILIBRIUM = 0, 1
REFILL = {"extrapolation": REFILL_EXTRAPOLATE, "equilibrium": REFILL_EQUILIBRIUM}


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("coupling", ctypes.c_int32),
        ("psm_m", ctypes.c_int32), ("psm_b", ctypes.c_int32), ("n_sub", ctypes.c_int32),
        ("eps_n", ctypes.c_int32), ("eps_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("max_particles", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("block_threads", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32), ("wall_link_cap", ctypes.c_int32),
        ("sweep_flags", ctypes.c_int32), ("refill", ctypes.c_int32),
        ("max_diameter", ctypes.c_double), ("nu", ctypes.c_double), ("magic", ctypes.c_double),
        ("f_ext", ctypes.c_double * 3), ("gravity", ctypes.c_double * 3),
    ]


class Particle(ctypes.Structure):
    _fields_ = [("X", ctypes.c_double * 3), ("U", ctypes.c_double * 3), ("Omega", ctypes.c_double * 3),
                ("D", ctypes.c_double), ("rho_p", ctypes.c_double), ("fixed", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class ParticleState(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double * 3), ("T", ctypes.c_double * 3), ("U", ctypes.c_double * 3),
                ("Omega", ctypes.c_double * 3), ("X", ctypes.c_double * 3)]


class MlpTrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("mult", ctypes.c_void_p), ("add", ctypes.c_void_p)]


class LbmpsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbmps status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbmps.so is not built: run `python -m paper_1702_04910_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        L.lbmps_workspace_bytes.restype = SZ
        L.lbmps_workspace_bytes.argtypes = [P]
        L.lbmps_batch_workspace_bytes.restype = SZ
        L.lbmps_batch_workspace_bytes.argtypes = [I32, P]
        L.lbmps_batch_create.restype = I32
        L.lbmps_batch_create.argtypes = [I32, P, P, SZ, P, ctypes.POINTER(P)]
        L.lbmps_create.restype = I32
        L.lbmps_create.argtypes = [P, P, SZ, P, ctypes.POINTER(P)]
        L.lbmps_destroy.restype = None
        L.lbmps_destroy.argtypes = [P]
        L.lbmps_init_equilibrium.restype = I32
        L.lbmps_init_equilibrium.argtypes = [P, I32, D, P]
        L.lbmps_set_static_solid.restype = I32
        L.lbmps_set_static_solid.argtypes = [P, I32, P, P]
        L.lbmps_set_outflow.restype = I32
        L.lbmps_set_outflow.argtypes = [P, I32, P, D]
        L.lbmps_set_viscosity.restype = I32
        L.lbmps_set_viscosity.argtypes = [P, I32, D]
        L.lbmps_set_gravity.restype = I32
        L.lbmps_set_gravity.argtypes = [P, I32, P]
        L.lbmps_set_particles.restype = I32
        L.lbmps_set_particles.argtypes = [P, I32, I32, P]
        L.lbmps_step.restype = I32
        L.lbmps_step.argtypes = [P, I32]
        L.lbmps_step_noalloc.restype = I32
        L.lbmps_step_noalloc.argtypes = [P, I32]
        L.lbmps_set_launch.restype = I32
        L.lbmps_set_launch.argtypes = [P, I32, I32, I32]
        L.lbmps_step_graph.restype = I32
        L.lbmps_step_graph.argtypes = [P, I32]
        L.lbmps_sync.restype = I32
        L.lbmps_sync.argtypes = [P]
        L.lbmps_get_particles.restype = I32
        L.lbmps_get_particles.argtypes = [P, I32, I32, P]
        L.lbmps_get_fields.restype = I32
        L.lbmps_get_fields.argtypes = [P, I32, P, P]
        L.lbmps_get_pdfs.restype = I32
        L.lbmps_get_pdfs.argtypes = [P, I32, P]
        L.lbmps_set_pdfs.restype = I32
        L.lbmps_set_pdfs.argtypes = [P, I32, P]
        L.lbmps_get_links.restype = I32
        L.lbmps_get_links.argtypes = [P, I64, P, P, P, P, ctypes.POINTER(I64)]
        L.lbmps_get_overlaps.restype = I32
        L.lbmps_get_overlaps.argtypes = [P, I64, P, P, P, ctypes.POINTER(I64)]
        L.lbmps_particle_base.restype = I32
        L.lbmps_particle_base.argtypes = [P, I32]
        L.lbmps_status_string.restype = ctypes.c_char_p
        L.lbmps_status_string.argtypes = [I32]
        L.lbmps_last_error.restype = ctypes.c_char_p
        L.lbmps_last_error.argtypes = [P]
        L.lbmps_set_timing.restype = I32
        L.lbmps_set_timing.argtypes = [P, I32]
        L.lbmps_get_timing.restype = I32
        L.lbmps_get_timing.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64)]
        L.lbmps_velocities.restype = None
        L.lbmps_velocities.argtypes = [P]
        L.lbmps_set_eps_model.restype = I32
        L.lbmps_set_eps_model.argtypes = [P, P, D, D]
        L.lbmps_rebuild_overlaps.restype = I32
        L.lbmps_rebuild_overlaps.argtypes = [P]
        L.lbmps_eps_judge.restype = I32
        L.lbmps_eps_judge.argtypes = [P, I32, P]
        L.lbmps_mlp_workspace_bytes.restype = SZ
        L.lbmps_mlp_workspace_bytes.argtypes = [I64]
        L.lbmps_mlp_create.restype = I32
        L.lbmps_mlp_create.argtypes = [I64, P, SZ, P, ctypes.POINTER(P)]
        L.lbmps_mlp_destroy.restype = None
        L.lbmps_mlp_destroy.argtypes = [P]
        for name in ("set_params", "get_params", "set_targets", "get_targets", "predict"):
            f = getattr(L, "lbmps_mlp_" + name)
            f.restype = I32
            f.argtypes = [P, P]
        L.lbmps_mlp_set_samples.restype = I32
        L.lbmps_mlp_set_samples.argtypes = [P, I64, P]
        L.lbmps_mlp_set_inputs.restype = I32
        L.lbmps_mlp_set_inputs.argtypes = [P, I32]
        L.lbmps_mlp_label.restype = I32
        L.lbmps_mlp_label.argtypes = [P, I32]
        L.lbmps_mlp_gradient.restype = I32
        L.lbmps_mlp_gradient.argtypes = [P, I64, I32, I64, I64, P]
        L.lbmps_mlp_train.restype = I32
        L.lbmps_mlp_train.argtypes = [P, P]
        L.lbmps_mlp_last_error.restype = ctypes.c_char_p
        L.lbmps_mlp_last_error.argtypes = [P]
        _lib = L
    return _lib


def velocities():
    c = np.zeros((19, 3), dtype=np.int32)
    lib().lbmps_velocities(c.ctypes.data)
    return c


def make_config(nx, ny, nz, nu, collision="trt", coupling="none", psm_m=1, psm_b=1, n_sub=0, eps_n=8,
                eps_mode=EPS_FLAT, precision="fp64", max_particles=0, max_diameter=0.0, magic=3.0 / 16.0,
                f_ext=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0), tile_rows=0, block_threads=0, grid_blocks=0,
                wall_link_cap=0, sweep_flags=0, refill=0):
    c = Config()
    c.nx, c.ny, c.nz = nx, ny, nz
    c.collision = TRT if collision == "trt" else BGK
    c.coupling = COUPLING[coupling] if isinstance(coupling, str) else coupling
    c.psm_m, c.psm_b, c.n_sub = psm_m, psm_b, n_sub
    c.eps_n, c.eps_mode = eps_n, eps_mode
    c.precision = PRECISION[precision] if isinstance(precision, str) else precision
    c.max_particles = max_particles
    c.tile_rows, c.block_threads, c.grid_blocks, c.wall_link_cap = tile_rows, block_threads, grid_blocks, wall_link_cap
    c.sweep_flags = sweep_flags
    c.refill = REFILL[refill] if isinstance(refill, str) else refill
    c.max_diameter, c.nu, c.magic = max_diameter, nu, magic
    for k in range(3):
        c.f_ext[k] = f_ext[k]
        c.gravity[k] = gravity[k]
    return c


def workspace_bytes(cfgs):
    if isinstance(cfgs, Config):
        cfgs = [cfgs]
    arr = (Config * len(cfgs))(*cfgs)
    return int(lib().lbmps_batch_workspace_bytes(len(cfgs), ctypes.addressof(arr)))


class Sim:
    """A context of one or more lattice instances (batched when len(cfgs) > 1)."""

    def __init__(self, cfgs, device="cuda", stream=None):
        import torch

        if isinstance(cfgs, Config):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self._arr = (Config * len(cfgs))(*cfgs)
        nbytes = int(lib().lbmps_batch_workspace_bytes(len(cfgs), ctypes.addressof(self._arr)))
        if nbytes == 0:
            raise LbmpsError(-1, "invalid configuration")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        st = lib().lbmps_batch_create(len(cfgs), ctypes.addressof(self._arr), self.workspace.data_ptr(), nbytes,
                                      self.stream.cuda_stream, ctypes.byref(self._ctx))
        if st != 0:
            msg = lib().lbmps_last_error(self._ctx).decode() if self._ctx.value else ""
            raise LbmpsError(st, msg)
        self.n_particles = [0] * len(cfgs)

    # -- helpers
    def _chk(self, st):
        if st != 0:
            raise LbmpsError(st, lib().lbmps_last_error(self._ctx).decode())

    def close(self):
        if self._ctx.value:
            lib().lbmps_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ncell(self, inst=0):
        c = self.cfgs[inst]
        return c.nx * c.ny * c.nz

    # -- API
    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0), inst=0):
        uu = (ctypes.c_double * 3)(*u)
        self._chk(lib().lbmps_init_equilibrium(self._ctx, inst, float(rho), ctypes.addressof(uu)))

    def set_static_solid(self, mask, v_wall=(0.0, 0.0, 0.0), inst=0):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
        assert m.size == self.ncell(inst)
        v = (ctypes.c_double * 3)(*v_wall)
        self._chk(lib().lbmps_set_static_solid(self._ctx, inst, m.ctypes.data, ctypes.addressof(v)))

    def set_outflow(self, mask, rho_out=1.0, inst=0):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
        assert m.size == self.ncell(inst)
        self._chk(lib().lbmps_set_outflow(self._ctx, inst, m.ctypes.data, float(rho_out)))

    def set_viscosity(self, nu, inst=0):
        self._chk(lib().lbmps_set_viscosity(self._ctx, inst, float(nu)))

    def set_gravity(self, g, inst=0):
        gg = (ctypes.c_double * 3)(*g)
        self._chk(lib().lbmps_set_gravity(self._ctx, inst, ctypes.addressof(gg)))

    def set_particles(self, X, U, Om, D, rho_p, fixed, inst=0):
        n = len(D)
        arr = (Particle * max(n, 1))()
        for i in range(n):
            for k in range(3):
                arr[i].X[k] = float(X[i][k])
                arr[i].U[k] = float(U[i][k])
                arr[i].Omega[k] = float(Om[i][k])
            arr[i].D = float(D[i])
            arr[i].rho_p = float(rho_p[i])
            arr[i].fixed = 1 if fixed[i] else 0
        self._chk(lib().lbmps_set_particles(self._ctx, inst, n, ctypes.addressof(arr)))
        self.n_particles[inst] = n

    def step(self, n):
        self._chk(lib().lbmps_step(self._ctx, int(n)))

    def step_noalloc(self, n):
        self._chk(lib().lbmps_step_noalloc(self._ctx, int(n)))

    def set_launch(self, block_threads=0, grid_blocks=0, sweep_flags=0):
        self._chk(lib().lbmps_set_launch(self._ctx, block_threads, grid_blocks, sweep_flags))

    def step_graph(self, n):
        self._chk(lib().lbmps_step_graph(self._ctx, int(n)))

    def sync(self):
        self._chk(lib().lbmps_sync(self._ctx))

    def particles(self, inst=0):
        n = self.n_particles[inst]
        arr = (ParticleState * max(n, 1))()
        self._chk(lib().lbmps_get_particles(self._ctx, inst, n, ctypes.addressof(arr)))
        out = {k: np.array([[getattr(arr[i], k)[j] for j in range(3)] for i in range(n)]).reshape(-1, 3)
               for k in ("F", "T", "U", "Omega", "X")}
        return out

    def fields(self, inst=0):
        N = self.ncell(inst)
        c = self.cfgs[inst]
        rho = np.empty(N)
        u = np.empty(3 * N)
        self._chk(lib().lbmps_get_fields(self._ctx, inst, rho.ctypes.data, u.ctypes.data))
        return rho.reshape(c.nz, c.ny, c.nx), u.reshape(3, c.nz, c.ny, c.nx)

    def get_pdfs(self, inst=0):
        c = self.cfgs[inst]
        g = np.empty(19 * self.ncell(inst))
        self._chk(lib().lbmps_get_pdfs(self._ctx, inst, g.ctypes.data))
        return g.reshape(19, c.nz, c.ny, c.nx)

    def set_pdfs(self, g, inst=0):
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        assert g.size == 19 * self.ncell(inst)
        self._chk(lib().lbmps_set_pdfs(self._ctx, inst, g.ctypes.data))

    def links(self):
        n = ctypes.c_int64()
        self._chk(lib().lbmps_get_links(self._ctx, 0, None, None, None, None, ctypes.byref(n)))
        cnt = n.value
        cell = np.empty(cnt, np.int32)
        q = np.empty(cnt, np.int32)
        p = np.empty(cnt, np.int32)
        d = np.empty(cnt, np.float64)
        self._chk(lib().lbmps_get_links(self._ctx, cnt, cell.ctypes.data, q.ctypes.data, p.ctypes.data,
                                        d.ctypes.data, ctypes.byref(n)))
        return dict(cell=cell, q=q, p=p, delta=d)

    def overlaps(self):
        n = ctypes.c_int64()
        self._chk(lib().lbmps_get_overlaps(self._ctx, 0, None, None, None, ctypes.byref(n)))
        cnt = n.value
        cell = np.empty(cnt, np.int32)
        p = np.empty(cnt, np.int32)
        e = np.empty(cnt, np.float64)
        self._chk(lib().lbmps_get_overlaps(self._ctx, cnt, cell.ctypes.data, p.ctypes.data, e.ctypes.data,
                                           ctypes.byref(n)))
        return dict(cell=cell, p=p, eps=e)

    def set_timing(self, enable, stride=1):
        """Time every `stride`-th sweep launch from now on (enable False: off)."""
        self._chk(lib().lbmps_set_timing(self._ctx, int(stride) if enable else 0))

    def timing(self):
        """(summed sweep-kernel milliseconds, number of sweep launches) since set_timing."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._chk(lib().lbmps_get_timing(self._ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def particle_base(self, inst):
        return int(lib().lbmps_particle_base(self._ctx, inst))

    # -- learned solid fraction
    def set_eps_model(self, params, r_min, r_max):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        assert p.size == MLP_NPARAM
        self._chk(lib().lbmps_set_eps_model(self._ctx, p.ctypes.data, float(r_min), float(r_max)))

    def rebuild_overlaps(self):
        self._chk(lib().lbmps_rebuild_overlaps(self._ctx))

    def eps_judge(self, stride=1):
        """(mean |error|, max |error|, cells judged) of the learned eps_s of the last rebuild."""
        out = np.zeros(3)
        self._chk(lib().lbmps_eps_judge(self._ctx, int(stride), out.ctypes.data))
        return float(out[0]), float(out[1]), int(out[2])


class Mlp:
    """Trainer of the solid-fraction network on the device."""

    def __init__(self, max_samples, device="cuda", stream=None):
        import torch

        nbytes = int(lib().lbmps_mlp_workspace_bytes(int(max_samples)))
        if nbytes == 0:
            raise LbmpsError(-1, "invalid sample capacity")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._m = ctypes.c_void_p()
        st = lib().lbmps_mlp_create(int(max_samples), self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                                    ctypes.byref(self._m))
        if st != 0:
            raise LbmpsError(st, "lbmps_mlp_create failed")
        self.n = 0

    def _chk(self, st):
        if st != 0:
            raise LbmpsError(st, lib().lbmps_mlp_last_error(self._m).decode())

    def close(self):
        if self._m.value:
            lib().lbmps_mlp_destroy(self._m)
            self._m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        assert p.size == MLP_NPARAM
        self._chk(lib().lbmps_mlp_set_params(self._m, p.ctypes.data))

    def params(self):
        p = np.empty(MLP_NPARAM, np.float32)
        self._chk(lib().lbmps_mlp_get_params(self._m, p.ctypes.data))
        return p

    def set_samples(self, rd):
        rd = np.ascontiguousarray(np.asarray(rd, dtype=np.float64).reshape(-1, 4))
        self._chk(lib().lbmps_mlp_set_samples(self._m, len(rd), rd.ctypes.data))
        self.n = len(rd)

    def set_inputs(self, n_inputs):
        self._chk(lib().lbmps_mlp_set_inputs(self._m, int(n_inputs)))

    def label(self, eps_n):
        self._chk(lib().lbmps_mlp_label(self._m, int(eps_n)))

    def set_targets(self, t):
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32).reshape(-1))
        assert t.size == self.n
        self._chk(lib().lbmps_mlp_set_targets(self._m, t.ctypes.data))

    def targets(self):
        t = np.empty(self.n, np.float32)
        self._chk(lib().lbmps_mlp_get_targets(self._m, t.ctypes.data))
        return t

    def predict(self):
        y = np.empty(self.n, np.float32)
        self._chk(lib().lbmps_mlp_predict(self._m, y.ctypes.data))
        return y

    def gradient(self, b0, batch, mult, add):
        g = np.empty(MLP_NPARAM, np.float32)
        self._chk(lib().lbmps_mlp_gradient(self._m, int(b0), int(batch), int(mult), int(add), g.ctypes.data))
        return g

    def train(self, mult, add, batch, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8):
        mult = np.ascontiguousarray(np.asarray(mult, dtype=np.int64))
        add = np.ascontiguousarray(np.asarray(add, dtype=np.int64))
        assert mult.size == add.size
        cfg = MlpTrainCfg(len(mult), int(batch), lr, beta1, beta2, adam_eps, mult.ctypes.data, add.ctypes.data)
        self._chk(lib().lbmps_mlp_train(self._m, ctypes.byref(cfg)))
