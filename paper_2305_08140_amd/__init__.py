"""MI355X NEP-ZBL energy / force / virial library (HIP, gfx950).

A thin ctypes binding over ``libnep_hip.so``: it marshals arguments into the
C ABI declared in ``include/nep.h`` and nothing else.  Every step of the
computation runs in the library's HIP kernels; PyTorch only provides device
memory and the current stream.  If the library has not been built the
import of the context raises: there is no CPU fallback.

Build:  python -m paper_2305_08140_amd.build
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep_hip.so")

NEP_OK = 0
NEP_E_ARG = -1
NEP_E_HIP = -2
NEP_E_NEIGH_OVERFLOW = -3
NEP_E_OVERLAP = -4
NEP_E_NONFINITE = -5
NEP_E_DT_UNDERFLOW = -6
NEP_E_STATE = -7
NEP_E_UNSUPPORTED = -8
NEP_E_INTERNAL = -9
NEP_E_CAPACITY = -10
NEP_WS_WORK_INTS = 8
NEP_MAX_POPULATION = 1024
NEP_LOSS_TERMS = 6
# loss weights of Sec. III.A
PAPER_LAMBDAS = {"e": 1.0, "f": 1.0, "v": 0.1, "l1": 0.05, "l2": 0.05}

EXPORTED = ("nep_create", "nep_destroy", "nep_set_weights", "nep_build_neighbors", "nep_update_neighbors",
            "nep_compute_efv",
            "nep_step_verlet", "nep_status", "nep_required_neighbors", "nep_mean_neighbors",
            "nep_time_efv", "nep_num_params", "nep_backward", "nep_backward_noalloc", "nep_compute_efv_graph", "nep_autotune",
            "nep_set_precision", "nep_wigner_seitz", "nep_population_reserve", "nep_population_efv",
            "nep_snes_sample", "nep_snes_update", "nep_strerror")


class NepError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class Hparams(C.Structure):
    _fields_ = [("n_rad", C.c_int32), ("n_ang", C.c_int32), ("k_rad", C.c_int32), ("k_ang", C.c_int32),
                ("l_max", C.c_int32), ("n_hidden", C.c_int32), ("Z", C.c_int32), ("pad_", C.c_int32),
                ("rc_rad", C.c_double), ("rc_ang", C.c_double), ("zbl_r1", C.c_double),
                ("zbl_r2", C.c_double)]


class Weights(C.Structure):
    _fields_ = [("c_rad", C.c_void_p), ("c_ang", C.c_void_p), ("q_scale", C.c_void_p), ("w0", C.c_void_p),
                ("b0", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_float), ("pad_", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("max_atoms", C.c_int64), ("max_cells", C.c_int32), ("max_neigh_ang", C.c_int32),
                ("max_neigh_rad", C.c_int32), ("pad_", C.c_int32), ("skin", C.c_double)]


class System(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_cells", C.c_int32), ("pbc", C.c_int32 * 3),
                ("cell_start", C.c_void_p), ("h", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p), ("mass", C.c_double)]


class Efv(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p),
                ("virial", C.c_void_p), ("energy_atom", C.c_void_p)]


class Md(C.Structure):
    _fields_ = [("dt_max", C.c_double), ("max_disp", C.c_double), ("dt_min", C.c_double),
                ("forces_valid", C.c_int32), ("thermo_chain", C.c_int32), ("thermo_T", C.c_double),
                ("thermo_tau", C.c_double), ("thermo_border", C.c_double), ("thermo_axes", C.c_int32),
                ("thermo_reset", C.c_int32), ("time_kernels", C.c_int32), ("pad_", C.c_int32)]


class BccRef(C.Structure):
    _fields_ = [("a", C.c_double), ("n", C.c_int32 * 3), ("pad_", C.c_int32)]


class Defects(C.Structure):
    _fields_ = [("n_vacancies", C.c_int64), ("n_interstitial_sites", C.c_int64), ("n_interstitials", C.c_int64),
                ("n_vacancy_clusters", C.c_int32), ("largest_vacancy_cluster", C.c_int32),
                ("n_interstitial_clusters", C.c_int32), ("largest_interstitial_cluster", C.c_int32)]


class Targets(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p),
                ("virial", C.c_void_p), ("has_virial", C.c_void_p), ("lambda_e", C.c_double),
                ("lambda_f", C.c_double), ("lambda_v", C.c_double), ("lambda_1", C.c_double),
                ("lambda_2", C.c_double)]


class MdStats(C.Structure):
    _fields_ = [("n_rebuilds", C.c_int64), ("dt_last", C.c_double), ("time", C.c_double),
                ("n_border", C.c_int64), ("thermo_energy", C.c_double), ("border_temperature", C.c_double),
                ("ms_descriptor", C.c_double), ("ms_force", C.c_double), ("n_timed_steps", C.c_int64)]


_lib = None


def lib():
    """Load libnep_hip.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2305_08140_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.nep_create.argtypes = [C.POINTER(Hparams), C.POINTER(Config), C.POINTER(P)]
        L.nep_destroy.argtypes = [P]
        L.nep_destroy.restype = None
        L.nep_set_weights.argtypes = [P, C.POINTER(Weights), C.c_int32, P]
        L.nep_build_neighbors.argtypes = [P, C.POINTER(System), P]
        L.nep_update_neighbors.argtypes = [P, C.POINTER(System), P]
        L.nep_compute_efv.argtypes = [P, C.POINTER(System), C.POINTER(Efv), P]
        L.nep_step_verlet.argtypes = [P, C.POINTER(System), C.POINTER(Md), C.c_int32, C.POINTER(Efv),
                                      C.POINTER(MdStats), P]
        L.nep_status.argtypes = [P, P]
        L.nep_required_neighbors.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.nep_mean_neighbors.argtypes = [P, P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nep_time_efv.argtypes = [P, C.POINTER(System), C.POINTER(Efv), C.c_int32, C.POINTER(C.c_double), P]
        L.nep_num_params.argtypes = [P]
        L.nep_set_precision.argtypes = [P, C.c_int32]
        L.nep_compute_efv_graph.argtypes = [P, C.POINTER(System), C.POINTER(Efv), P]
        L.nep_autotune.argtypes = [P, C.POINTER(System), C.POINTER(Efv), C.c_int32, C.POINTER(C.c_int32), P]
        L.nep_backward.argtypes = [P, C.POINTER(System), C.POINTER(Efv), P, P, P, P, P, P, P]
        L.nep_backward_noalloc.argtypes = [P, C.POINTER(System), C.POINTER(Efv), P, P, P, P, P, P, P]
        L.nep_wigner_seitz.argtypes = [C.POINTER(System), C.POINTER(BccRef), P, P, C.c_int32, P, P, P, P, P, P,
                                       C.POINTER(Defects), P]
        L.nep_population_reserve.argtypes = [P, C.c_int32]
        L.nep_population_efv.argtypes = [P, C.POINTER(System), C.c_int32, P, P, P, P, C.POINTER(Targets), P, P]
        L.nep_snes_sample.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P]
        L.nep_snes_update.argtypes = [C.c_int32, C.c_int32, P, C.c_int32, P, P, P, C.c_double, C.c_double, P]
        L.nep_strerror.argtypes = [C.c_int]
        L.nep_strerror.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("nep_destroy", "nep_strerror"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().nep_strerror(int(code)).decode()
    except ImportError:
        return "error %d" % code


def _check(code: int, where: str):
    if code != NEP_OK:
        raise NepError(code, where)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceSystem:
    """Positions / velocities in device memory plus the host-side cell description."""

    def __init__(self, pos, h, cell_start=None, vel=None, pbc=(1, 1, 1), mass=183.84, device="cuda"):
        torch = _torch()
        pos = np.asarray(pos, dtype=np.float64)
        n = pos.shape[0]
        self.h = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(-1, 9))
        self.n_cells = self.h.shape[0]
        if cell_start is None:
            cell_start = np.array([0, n], dtype=np.int64)
        self.cell_start = np.ascontiguousarray(cell_start, dtype=np.int64)
        self.pbc = tuple(int(p) for p in pbc)
        self.mass = float(mass)
        p = torch.from_numpy(np.ascontiguousarray(pos.T)).to(device)
        self.x, self.y, self.z = p[0].contiguous(), p[1].contiguous(), p[2].contiguous()
        if vel is None:
            vel = np.zeros_like(pos)
        v = torch.from_numpy(np.ascontiguousarray(np.asarray(vel, dtype=np.float64).T)).to(device)
        self.vx, self.vy, self.vz = v[0].contiguous(), v[1].contiguous(), v[2].contiguous()
        self.n_atoms = n

    @classmethod
    def from_synth(cls, s, device="cuda"):
        return cls(s.pos, s.h, s.cell_start, s.vel, s.pbc, s.mass, device)

    def positions(self):
        torch = _torch()
        return torch.stack([self.x, self.y, self.z], dim=1)

    def velocities(self):
        torch = _torch()
        return torch.stack([self.vx, self.vy, self.vz], dim=1)

    def c_struct(self) -> System:
        s = System()
        s.n_atoms = self.n_atoms
        s.n_cells = self.n_cells
        for a in range(3):
            s.pbc[a] = self.pbc[a]
        s.cell_start = self.cell_start.ctypes.data
        s.h = self.h.ctypes.data
        s.x, s.y, s.z = self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr()
        s.vx, s.vy, s.vz = self.vx.data_ptr(), self.vy.data_ptr(), self.vz.data_ptr()
        s.mass = self.mass
        return s


class EFV:
    """Output buffers: energy [C] f64, fx/fy/fz [N] f32, virial [C,9] f64, energy_atom [N] f32."""

    def __init__(self, n_atoms, n_cells, device="cuda", energy_atom=True):
        torch = _torch()
        self.energy = torch.zeros(n_cells, dtype=torch.float64, device=device)
        self.fx = torch.zeros(n_atoms, dtype=torch.float32, device=device)
        self.fy = torch.zeros(n_atoms, dtype=torch.float32, device=device)
        self.fz = torch.zeros(n_atoms, dtype=torch.float32, device=device)
        self.virial = torch.zeros(n_cells, 9, dtype=torch.float64, device=device)
        self.energy_atom = torch.zeros(n_atoms, dtype=torch.float32, device=device) if energy_atom else None

    def forces(self):
        torch = _torch()
        return torch.stack([self.fx, self.fy, self.fz], dim=1)

    def c_struct(self) -> Efv:
        e = Efv()
        e.energy = self.energy.data_ptr()
        e.fx, e.fy, e.fz = self.fx.data_ptr(), self.fy.data_ptr(), self.fz.data_ptr()
        e.virial = self.virial.data_ptr()
        e.energy_atom = self.energy_atom.data_ptr() if self.energy_atom is not None else None
        return e


def hparams_from(m) -> Hparams:
    return Hparams(m.n_rad, m.n_ang, m.k_rad, m.k_ang, m.l_max, m.n_hidden, int(m.Z), 0,
                   m.rc_rad, m.rc_ang, m.zbl_r1, m.zbl_r2)


class Context:
    """One nep_ctx: model, capacities and the neighbour-list state."""

    def __init__(self, model, max_atoms, max_cells=1, max_neigh_ang=48, max_neigh_rad=96, skin=1.0,
                 check=True):
        self._ptr = None
        self.check = check
        L = lib()
        hp = hparams_from(model)
        cfg = Config(int(max_atoms), int(max_cells), int(max_neigh_ang), int(max_neigh_rad), 0, float(skin))
        ptr = C.c_void_p()
        _check(L.nep_create(C.byref(hp), C.byref(cfg), C.byref(ptr)), "nep_create")
        self._ptr = ptr
        # sizes of the parameter blocks (c_rad, c_ang, w0, b0, w1, b1) of
        # this context's model, in the flat layout of nep_backward
        dim = model.n_rad + model.n_ang * model.l_max
        self.theta_sizes = (model.n_rad * model.k_rad, model.n_ang * model.k_ang, model.n_hidden * dim,
                            model.n_hidden, model.n_hidden, 1)
        # which forward's weights and neighbour lists the context holds (the
        # differentiable energy restores them before its backward)
        self.state_token = None
        self.nep_set_weights(model)

    def __del__(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.nep_destroy(self._ptr)
            self._ptr = None

    def close(self):
        self.__del__()

    def nep_set_weights(self, model):
        arrs = [np.ascontiguousarray(getattr(model, k), dtype=np.float32)
                for k in ("c_rad", "c_ang", "q_scale", "w0", "b0", "w1")]
        self.state_token = None
        w = Weights(*[a.ctypes.data for a in arrs], float(model.b1), 0)
        _check(lib().nep_set_weights(self._ptr, C.byref(w), 0, None), "nep_set_weights")

    def nep_build_neighbors(self, system: DeviceSystem, stream=None):
        self.state_token = None
        s = system.c_struct()
        _check(lib().nep_build_neighbors(self._ptr, C.byref(s), _stream_ptr(stream)), "nep_build_neighbors")
        if self.check:
            self.nep_status(stream)

    def nep_update_neighbors(self, system: DeviceSystem, stream=None):
        """Rebuild the lists only if an atom moved more than skin/2 since the last build (decided on the device)."""
        self.state_token = None
        s = system.c_struct()
        _check(lib().nep_update_neighbors(self._ptr, C.byref(s), _stream_ptr(stream)), "nep_update_neighbors")
        if self.check:
            self.nep_status(stream)

    def nep_compute_efv(self, system: DeviceSystem, out: EFV, stream=None):
        s = system.c_struct()
        o = out.c_struct()
        _check(lib().nep_compute_efv(self._ptr, C.byref(s), C.byref(o), _stream_ptr(stream)), "nep_compute_efv")
        if self.check:
            self.nep_status(stream)
        return out

    def nep_step_verlet(self, system: DeviceSystem, n_steps, out: EFV, dt_max=1.0, max_disp=0.0, dt_min=1e-6,
                        forces_valid=False, thermostat=None, time_kernels=False, stream=None):
        """thermostat: None, or a dict with keys T (K), tau (fs), border (A),
        axes (tuple of lattice-vector indices), chain (length, default 3) and
        reset (bool) for the Nose-Hoover chain on the border atoms."""
        self.state_token = None
        s = system.c_struct()
        o = out.c_struct()
        md = Md(dt_max=float(dt_max), max_disp=float(max_disp), dt_min=float(dt_min),
                forces_valid=int(bool(forces_valid)), time_kernels=int(bool(time_kernels)))
        if thermostat is not None:
            md.thermo_chain = int(thermostat.get("chain", 3))
            md.thermo_T = float(thermostat["T"])
            md.thermo_tau = float(thermostat["tau"])
            md.thermo_border = float(thermostat["border"])
            md.thermo_axes = sum(1 << int(a) for a in thermostat.get("axes", (0, 1, 2)))
            md.thermo_reset = int(bool(thermostat.get("reset", False)))
        st = MdStats()
        _check(lib().nep_step_verlet(self._ptr, C.byref(s), C.byref(md), int(n_steps), C.byref(o), C.byref(st),
                                     _stream_ptr(stream)), "nep_step_verlet")
        return {"n_rebuilds": int(st.n_rebuilds), "dt_last": float(st.dt_last), "time": float(st.time),
                "n_border": int(st.n_border), "thermo_energy": float(st.thermo_energy),
                "border_temperature": float(st.border_temperature), "ms_descriptor": float(st.ms_descriptor),
                "ms_force": float(st.ms_force), "n_timed_steps": int(st.n_timed_steps)}

    def nep_status(self, stream=None):
        _check(lib().nep_status(self._ptr, _stream_ptr(stream)), "device status")

    def nep_required_neighbors(self):
        a, r = C.c_int32(), C.c_int32()
        _check(lib().nep_required_neighbors(self._ptr, C.byref(a), C.byref(r)), "nep_required_neighbors")
        return int(a.value), int(r.value)

    def nep_time_efv(self, system: DeviceSystem, out: EFV, reps=5, stream=None):
        """Mean per-launch milliseconds of (position refresh, descriptor, force, reductions)."""
        s = system.c_struct()
        o = out.c_struct()
        ms = (C.c_double * 4)()
        _check(lib().nep_time_efv(self._ptr, C.byref(s), C.byref(o), int(reps), ms, _stream_ptr(stream)),
               "nep_time_efv")
        return {"sort": ms[0], "descriptor": ms[1], "force": ms[2], "reduce": ms[3]}

    def nep_compute_efv_graph(self, system: DeviceSystem, out: EFV, stream=None):
        """Graph-replayed evaluation; needs a non-default stream (e.g. torch.cuda.Stream())."""
        s = system.c_struct()
        o = out.c_struct()
        _check(lib().nep_compute_efv_graph(self._ptr, C.byref(s), C.byref(o), _stream_ptr(stream)),
               "nep_compute_efv_graph")
        if self.check:
            self.nep_status(stream)
        return out

    SHAPE_NAMES = ("64/tile", "128/tile", "256/tile", "64/persistent", "128/persistent", "256/persistent")

    def nep_autotune(self, system: DeviceSystem, out: EFV, reps=3, stream=None):
        """Pick the fastest launch shapes for this size; returns (descriptor, force) shape names."""
        s = system.c_struct()
        o = out.c_struct()
        sh = (C.c_int32 * 2)()
        _check(lib().nep_autotune(self._ptr, C.byref(s), C.byref(o), int(reps), sh, _stream_ptr(stream)),
               "nep_autotune")
        return self.SHAPE_NAMES[sh[0]], self.SHAPE_NAMES[sh[1]]

    def nep_set_precision(self, mode):
        """0: FP32 hidden layer (vector ALUs); 1: BF16 and 2: FP32 hidden layer on the matrix cores."""
        _check(lib().nep_set_precision(self._ptr, int(mode)), "nep_set_precision")

    def nep_num_params(self):
        return int(lib().nep_num_params(self._ptr))

    def nep_population_reserve(self, n_pop):
        _check(lib().nep_population_reserve(self._ptr, int(n_pop)), "nep_population_reserve")
        self.pop_cap = int(n_pop)

    def nep_population_efv(self, system: DeviceSystem, theta, targets=None, lambdas=PAPER_LAMBDAS,
                           want_energy=True, want_forces=True, want_virial=True, stream=None):
        """Evaluate every row of theta (device float32 [P, n_params]) on the
        batch; returns device tensors energy [P, C], forces [P, 3, N],
        virial [P, C, 9] (None where not wanted) and, with targets (a dict of
        device tensors energy [C] f64, forces [3, N] f32, virial [C, 9] f64 or
        None, has_virial [C] uint8 or None), loss [P, 6]."""
        torch = _torch()
        theta = theta.contiguous()
        P_ = int(theta.shape[0])
        dev = theta.device
        N, Cc = system.n_atoms, system.n_cells
        E = torch.empty(P_, Cc, dtype=torch.float64, device=dev) if want_energy else None
        F = torch.empty(P_, 3, N, dtype=torch.float32, device=dev) if want_forces else None
        W = torch.empty(P_, Cc, 9, dtype=torch.float64, device=dev) if want_virial else None
        loss = None
        tg = None
        if targets is not None:
            loss = torch.empty(P_, NEP_LOSS_TERMS, dtype=torch.float64, device=dev)
            tf = targets["forces"]
            tv = targets.get("virial")
            hv = targets.get("has_virial")
            tg = Targets(targets["energy"].data_ptr(), tf[0].data_ptr(), tf[1].data_ptr(), tf[2].data_ptr(),
                         tv.data_ptr() if tv is not None else None, hv.data_ptr() if hv is not None else None,
                         float(lambdas["e"]), float(lambdas["f"]), float(lambdas["v"]), float(lambdas["l1"]),
                         float(lambdas["l2"]))
        s = system.c_struct()
        ptr = (lambda t: t.data_ptr() if t is not None else None)
        _check(lib().nep_population_efv(self._ptr, C.byref(s), P_, theta.data_ptr(), ptr(E), ptr(F), ptr(W),
                                        C.byref(tg) if tg is not None else None, ptr(loss), _stream_ptr(stream)),
               "nep_population_efv")
        if self.check:
            self.nep_status(stream)
        return {"energy": E, "forces": F, "virial": W, "loss": loss}

    def nep_backward(self, system: DeviceSystem, out: EFV, gE, grad_pos=True, grad_cell=True, stream=None):
        """dL/dtheta [P], dL/dx [N,3] and dL/dh [C,3,3] for L = sum_c gE[c] E_c (device FP64 tensors)."""
        return self._backward("nep_backward", system, out, gE, grad_pos, grad_cell, stream, None)

    def nep_backward_noalloc(self, system: DeviceSystem, out: EFV, gE, grad_pos=True, grad_cell=True,
                             stream=None, outputs=None):
        """nep_backward through the library's allocation-free entry point.  `outputs`, if given, is a
        dict of preallocated device FP64 tensors {"params": [P], "x", "y", "z": [N], "h": [C, 9]}
        (so that the call allocates nothing at all); otherwise they are allocated here."""
        return self._backward("nep_backward_noalloc", system, out, gE, grad_pos, grad_cell, stream, outputs)

    def _backward(self, name, system, out, gE, grad_pos, grad_cell, stream, outputs):
        torch = _torch()
        dev = out.fx.device
        gE = gE.to(device=dev, dtype=torch.float64).contiguous()
        outputs = outputs or {}
        gp = outputs.get("params")
        if gp is None:
            gp = torch.empty(self.nep_num_params(), dtype=torch.float64, device=dev)
        gx = gy = gz = gh = None
        if grad_pos:
            gx, gy, gz = (outputs.get(k) for k in ("x", "y", "z"))
            if gx is None or gy is None or gz is None:
                gx, gy, gz = (torch.empty(system.n_atoms, dtype=torch.float64, device=dev) for _ in range(3))
        if grad_cell:
            gh = outputs.get("h")
            if gh is None:
                gh = torch.empty(system.n_cells, 9, dtype=torch.float64, device=dev)
        s = system.c_struct()
        o = out.c_struct()
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        _check(getattr(lib(), name)(self._ptr, C.byref(s), C.byref(o), ptr(gE), ptr(gp), ptr(gx), ptr(gy),
                                    ptr(gz), ptr(gh), _stream_ptr(stream)), name)
        if self.check:
            self.nep_status(stream)
        gpos = torch.stack([gx, gy, gz], dim=1) if grad_pos else None
        return gp, gpos, (gh.view(-1, 3, 3) if grad_cell else None)

    def nep_mean_neighbors(self, stream=None):
        r, a = C.c_double(), C.c_double()
        _check(lib().nep_mean_neighbors(self._ptr, _stream_ptr(stream), C.byref(r), C.byref(a)),
               "nep_mean_neighbors")
        return float(r.value), float(a.value)


def efv(model, system: DeviceSystem, ctx: Context | None = None, max_neigh_ang=48, max_neigh_rad=96, skin=1.0):
    """Convenience: build lists and evaluate once; returns (EFV, Context)."""
    if ctx is None:
        ctx = Context(model, system.n_atoms, system.n_cells, max_neigh_ang, max_neigh_rad, skin)
    out = EFV(system.n_atoms, system.n_cells)
    ctx.nep_build_neighbors(system)
    ctx.nep_compute_efv(system, out)
    return out, ctx


def snes_sample(mu, sigma, draws, stream=None):
    """theta = mu + sigma * draws on the device (float32 tensors; draws [P, n])."""
    torch = _torch()
    P_, n = (int(v) for v in draws.shape)
    theta = torch.empty(P_, n, dtype=torch.float32, device=draws.device)
    _check(lib().nep_snes_sample(P_, n, mu.data_ptr(), sigma.data_ptr(), draws.contiguous().data_ptr(),
                                 theta.data_ptr(), _stream_ptr(stream)), "nep_snes_sample")
    return theta


def snes_update(mu, sigma, draws, loss, eta_mu=0.0, eta_sigma=0.0, stream=None):
    """In-place SNES update of mu and sigma (device float32) from the members'
    losses (device float64 [P] or [P, k], the first column is used)."""
    P_, n = (int(v) for v in draws.shape)
    stride = 1 if loss.dim() == 1 else int(loss.stride(0))
    _check(lib().nep_snes_update(P_, n, loss.data_ptr(), stride, draws.contiguous().data_ptr(), mu.data_ptr(),
                                 sigma.data_ptr(), float(eta_mu), float(eta_sigma), _stream_ptr(stream)),
           "nep_snes_update")


def snes_generation(ctx: "Context", system: "DeviceSystem", mu, sigma, draws, targets, lambdas=PAPER_LAMBDAS,
                    stream=None):
    """One SNES generation on the device: sample the population from (mu,
    sigma) with the given standard-normal draws, evaluate every member's loss
    on the batch, update mu and sigma in place.  Returns the loss terms [P, 6]."""
    theta = snes_sample(mu, sigma, draws, stream)
    res = ctx.nep_population_efv(system, theta, targets, lambdas, want_energy=False, want_forces=False,
                                 want_virial=False, stream=stream)
    snes_update(mu, sigma, draws, res["loss"], stream=stream)
    return res["loss"]


def wigner_seitz(system: "DeviceSystem", a: float, n_cells, capacity: int = 65536, site_of_atom: bool = False,
                 stream=None):
    """nep_wigner_seitz on a one-cell system against the perfect bcc lattice of
    n_cells conventional cells of constant a.  Returns the summary and device
    tensors: occupancy, sorted vacancy / interstitial sites, interstitial
    multiplicities, cluster labels (and the site of every atom if asked)."""
    torch = _torch()
    n0, n1, n2 = (int(v) for v in n_cells)
    dev = system.x.device
    i32 = dict(dtype=torch.int32, device=dev)
    occ = torch.empty(2 * n0 * n1 * n2, **i32)
    site = torch.empty(system.n_atoms, **i32) if site_of_atom else None
    arr = [torch.empty(max(capacity, 1), **i32) for _ in range(5)]
    work = torch.empty(NEP_WS_WORK_INTS, **i32)
    ref = BccRef(float(a), (C.c_int32 * 3)(n0, n1, n2), 0)
    out = Defects()
    s = system.c_struct()
    code = lib().nep_wigner_seitz(C.byref(s), C.byref(ref), occ.data_ptr(), site.data_ptr() if site is not None
                                  else None, int(capacity), arr[0].data_ptr(), arr[1].data_ptr(),
                                  arr[2].data_ptr(), arr[3].data_ptr(), arr[4].data_ptr(), work.data_ptr(),
                                  C.byref(out), _stream_ptr(stream))
    _check(code, "nep_wigner_seitz")
    nv, ni = int(out.n_vacancies), int(out.n_interstitial_sites)
    res = {k: getattr(out, k) for k, _ in Defects._fields_}
    res.update(occupancy=occ, vacancy_sites=arr[0][:nv], vacancy_cluster=arr[1][:nv],
               interstitial_sites=arr[2][:ni], interstitial_mult=arr[3][:ni], interstitial_cluster=arr[4][:ni],
               site_of_atom=site)
    return res
