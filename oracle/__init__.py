"""FP64 CPU oracle for NEP-ZBL (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
shares no code with the GPU library: the arithmetic lives in
``nep_oracle.c`` (plain C, double precision), this file only marshals numpy
arrays through ctypes and adds a plain velocity-Verlet loop.

Paper passages followed: Sec. II.A, Eqs. 1-4 (site energy, ZBL repulsion,
W-W screening function, screening length, Tersoff switch); the NEP descriptor
and network of the NEP framework cited in Sec. II.A / Sec. III.A; the
adaptive time step of Sec. II.B.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nep_oracle.c")
_LIB = os.path.join(_HERE, "libnep_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (portable flags: the library may run on another host)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("n_rad", C.c_int32), ("n_ang", C.c_int32), ("k_rad", C.c_int32),
                ("k_ang", C.c_int32), ("l_max", C.c_int32), ("n_hidden", C.c_int32),
                ("rc_rad", C.c_double), ("rc_ang", C.c_double), ("zbl_r1", C.c_double),
                ("zbl_r2", C.c_double), ("Z", C.c_double),
                ("c_rad", C.POINTER(C.c_double)), ("c_ang", C.POINTER(C.c_double)),
                ("q_scale", C.POINTER(C.c_double)), ("w0", C.POINTER(C.c_double)),
                ("b0", C.POINTER(C.c_double)), ("w1", C.POINTER(C.c_double)),
                ("b1", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        L.orc_efv.restype = C.c_int
        L.orc_efv.argtypes = [C.POINTER(_Model), C.c_int64, dp, dp, i32p, C.c_int64, i64p,
                              dp, dp, dp, dp, C.c_int]
        L.orc_pairs.restype = C.c_int
        L.orc_pairs.argtypes = [C.c_int64, dp, dp, i32p, C.c_double, C.c_int, C.c_int, i64p,
                                i64p, i64p, i32p, dp]
        L.orc_chebyshev.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_basis.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_legendre.argtypes = [C.c_double, dp, dp]
        L.orc_tersoff_fc.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_zbl.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_params.restype = C.c_int
        L.orc_num_params.argtypes = [C.POINTER(_Model)]
        L.orc_param_grad.restype = C.c_int
        L.orc_param_grad.argtypes = [C.POINTER(_Model), C.c_int64, dp, dp, i32p, C.c_int, dp]
        L.orc_coulomb.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _ModelRef:
    """Holds the ctypes struct together with the arrays it points into."""

    def __init__(self, m):
        self.arrays = [_c64(m.c_rad), _c64(m.c_ang), _c64(m.q_scale), _c64(m.w0), _c64(m.b0),
                       _c64(m.w1)]
        ca, cb, qs, w0, b0, w1 = self.arrays
        self.s = _Model(m.n_rad, m.n_ang, m.k_rad, m.k_ang, m.l_max, m.n_hidden,
                        m.rc_rad, m.rc_ang, m.zbl_r1, m.zbl_r2, float(m.Z),
                        _dp(ca), _dp(cb), _dp(qs), _dp(w0), _dp(b0), _dp(w1), float(m.b1))


def efv_cell(model, pos, h, pbc=(1, 1, 1), targets=None, virial=True, desc=False, method=-1):
    """Energy per atom, forces, virial (and optionally descriptors) of one cell.

    Returns a dict with ``energy_atom`` [T], ``forces`` [T,3], ``energy`` (sum, only
    when all atoms are targets), ``virial`` [3,3] (only when all atoms are targets),
    ``desc`` [T,D]."""
    L = lib()
    mr = _ModelRef(model)
    pos = _c64(pos)
    h = _c64(np.asarray(h).reshape(9))
    pbc_a = np.ascontiguousarray(pbc, dtype=np.int32)
    N = pos.shape[0]
    if targets is None:
        T = N
        tptr = None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        T = targets.shape[0]
        tptr = targets.ctypes.data_as(C.POINTER(C.c_int64))
        virial = False
    e = np.zeros(T)
    f = np.zeros((T, 3))
    w = np.zeros(9) if virial else None
    D = model.dim
    q = np.zeros((T, D)) if desc else None
    rc = L.orc_efv(C.byref(mr.s), N, _dp(pos), _dp(h), pbc_a.ctypes.data_as(C.POINTER(C.c_int32)),
                   T, tptr, _dp(e), _dp(f), _dp(w) if w is not None else None,
                   _dp(q) if q is not None else None, method)
    if rc != 0:
        raise ValueError("orc_efv rejected its arguments (rc=%d)" % rc)
    out = {"energy_atom": e, "forces": f}
    if targets is None:
        out["energy"] = float(np.sum(e))
    if w is not None:
        out["virial"] = w.reshape(3, 3)
    if q is not None:
        out["desc"] = q
    return out


def efv_system(model, system, virial=True):
    """Evaluate every cell of a ``nep_synth.System``; per-cell energy [C], forces [N,3], virial [C,3,3]."""
    E = np.zeros(system.n_cells)
    W = np.zeros((system.n_cells, 3, 3))
    F = np.zeros((system.n_atoms, 3))
    U = np.zeros(system.n_atoms)
    for c in range(system.n_cells):
        s, t = int(system.cell_start[c]), int(system.cell_start[c + 1])
        r = efv_cell(model, system.pos[s:t], system.h[c], system.pbc, virial=virial)
        E[c] = r["energy"]
        F[s:t] = r["forces"]
        U[s:t] = r["energy_atom"]
        if virial:
            W[c] = r["virial"]
    return {"energy": E, "forces": F, "virial": W, "energy_atom": U}


def param_grad_cell(model, pos, h, pbc=(1, 1, 1), method=-1):
    """dE/dtheta of one cell, theta = (c_rad, c_ang, w0, b0, w1, b1) flattened (see Model.param_vector)."""
    L = lib()
    mr = _ModelRef(model)
    pos = _c64(pos)
    h = _c64(np.asarray(h).reshape(9))
    pbc_a = np.ascontiguousarray(pbc, dtype=np.int32)
    P = L.orc_num_params(C.byref(mr.s))
    g = np.zeros(P)
    rc = L.orc_param_grad(C.byref(mr.s), pos.shape[0], _dp(pos), _dp(h), pbc_a.ctypes.data_as(C.POINTER(C.c_int32)),
                          method, _dp(g))
    if rc != 0:
        raise ValueError("orc_param_grad rejected its arguments")
    return g


def pairs(pos, h, pbc, rc, method=0):
    """All (i, j, n) with |x_j + n.h - x_i| < rc.  Returns (start[N+1], j[P], n[P,3], r[P])."""
    L = lib()
    pos = _c64(pos)
    h = _c64(np.asarray(h).reshape(9))
    pbc_a = np.ascontiguousarray(pbc, dtype=np.int32)
    N = pos.shape[0]
    counts = np.zeros(N, dtype=np.int64)
    i64 = C.POINTER(C.c_int64)
    i32 = C.POINTER(C.c_int32)
    rc_ = L.orc_pairs(N, _dp(pos), _dp(h), pbc_a.ctypes.data_as(i32), rc, method, 0,
                      counts.ctypes.data_as(i64), None, None, None, None)
    if rc_ != 0:
        raise ValueError("orc_pairs rejected its arguments")
    start = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    P = int(start[-1])
    j = np.zeros(P, dtype=np.int64)
    n = np.zeros((P, 3), dtype=np.int32)
    r = np.zeros(P)
    L.orc_pairs(N, _dp(pos), _dp(h), pbc_a.ctypes.data_as(i32), rc, method, 1,
                counts.ctypes.data_as(i64), start.ctypes.data_as(i64), j.ctypes.data_as(i64),
                n.ctypes.data_as(i32), _dp(r))
    return start, j, n, r


# ---- scalar building blocks, exposed for the pin tests -------------------

def chebyshev(K, x):
    T = np.zeros(K); dT = np.zeros(K)
    lib().orc_chebyshev(K, float(x), _dp(T), _dp(dT))
    return T, dT


def basis(K, r, rc):
    f = np.zeros(K); df = np.zeros(K)
    lib().orc_basis(K, float(r), float(rc), _dp(f), _dp(df))
    return f, df


def legendre(c):
    P = np.zeros(5); dP = np.zeros(5)
    lib().orc_legendre(float(c), _dp(P), _dp(dP))
    return P, dP


def tersoff_fc(r, r1=1.0, r2=2.0):
    f = np.zeros(1); df = np.zeros(1)
    lib().orc_tersoff_fc(float(r), r1, r2, _dp(f), _dp(df))
    return float(f[0]), float(df[0])


def zbl(r, Z=74.0, r1=1.0, r2=2.0):
    U = np.zeros(1); dU = np.zeros(1)
    lib().orc_zbl(float(r), float(Z), float(Z), r1, r2, _dp(U), _dp(dU))
    return float(U[0]), float(dU[0])


def coulomb():
    return float(lib().orc_coulomb())


def num_threads():
    return int(lib().orc_num_threads())


from .md import (velocity_verlet, velocity_verlet_nhc, kinetic_energy, border_mask,  # noqa: E402,F401
                 NoseHooverChain, EV_PER_U_TO_A2_PER_FS2, K_B_EV)
