"""Plausible mistakes planted in a copy of the oracle must fail at least one pin.

Each mutation edits the C source text, builds it into a temporary library,
and runs a set of fast pin checks (the same kinds as test_oracle_pins.py)
against it.  The real oracle is untouched.
"""
import ctypes as C
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special as sp

import nep_synth
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "nep_oracle.c")

MUTATIONS = {
    "drop_j_eq_k": ("            if (b == a) c = 1.0;\n            double P[5], dP[5];",
                    "            if (b == a) continue;\n            double P[5], dP[5];"),
    "angular_factor_2_dropped": ("double t1 = 2.0 * w * dgA", "double t1 = 1.0 * w * dgA"),
    "angular_sign": ("acc[k] += t1 * ua[k] + t2 * (ub[k] - c * ua[k]);", "acc[k] += t1 * ua[k] - t2 * (ub[k] - c * ua[k]);"),
    "w0_transposed": ("z += m->w0[mu * D + nu] * m->q_scale[nu] * q[nu];", "z += m->w0[nu * H % (H * D) + mu] * m->q_scale[nu] * q[nu];"),
    "zbl_not_halved": ("            e += 0.5 * uz;", "            e += uz;"),
    "zbl_screening_length": ("double a = 0.46848 / (pow(Zi, 0.23) + pow(Zj, 0.23));", "double a = 0.46848 / pow(Zi * Zj, 0.23);"),
    "cutoff_sign": ("*f = 0.5 * (1.0 + cos(ORC_PI * r / rc));", "*f = 0.5 * (1.0 - cos(ORC_PI * r / rc));"),
    "chebyshev_recurrence": ("T[k] = 2.0 * x * T[k - 1] - T[k - 2];", "T[k] = 2.0 * x * T[k - 1] + T[k - 2];"),
    "legendre_p3": ("P[3] = 0.5 * (5.0 * c * c * c - 3.0 * c);", "P[3] = 0.5 * (5.0 * c * c * c - 2.0 * c);"),
    "image_range_short": ("lo[a] = -ds - rc / wid[a];", "lo[a] = -ds - 0.5 * rc / wid[a];"),
    "virial_transposed": ("virial[3 * al + be] -= Dp[a][3 * p + al] * PL[a].p[p].d[be];",
                          "virial[3 * be + al] -= Dp[a][3 * p + al] * PL[a].p[p].d[be] * (al == be ? 1.0 : 1.1);"),
    "reverse_force_missing": ("                F[3 * b + k] -= Dp[a][3 * p + k];", "                F[3 * b + k] -= 0.0 * Dp[a][3 * p + k];"),
    "descriptor_scale_ignored": ("z += m->w0[mu * D + nu] * m->q_scale[nu] * q[nu];", "z += m->w0[mu * D + nu] * q[nu];"),
}


def _build(mutation, tmpdir):
    src = open(SRC).read()
    old, new = MUTATIONS[mutation]
    assert old in src, mutation
    path = os.path.join(tmpdir, f"orc_{mutation}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new, 1))
    lib = os.path.join(tmpdir, f"liborc_{mutation}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", lib, path, "-lm"])
    return lib


def _with_lib(path):
    """Point the oracle module at another build (argtypes copied from the real one)."""
    real = oracle.lib()
    L = C.CDLL(path)
    for name in ("orc_efv", "orc_pairs", "orc_chebyshev", "orc_basis", "orc_legendre", "orc_tersoff_fc", "orc_zbl",
                 "orc_num_threads", "orc_num_params", "orc_param_grad", "orc_coulomb"):
        f, g = getattr(L, name), getattr(real, name)
        f.argtypes, f.restype = g.argtypes, g.restype
    return L


# ---- fast pin checks (each returns True when the pin holds) -------------------


def _pin_zbl_dimer(m):
    mm = m.copy()
    mm.w1[:] = 0.0
    for r in (0.6, 1.3):
        s = nep_synth.dimer(r)
        out = oracle.efv_cell(mm, s.pos, s.h[0])
        ke = 14.3996454784
        a = 0.46848 / (2 * 74 ** 0.23)
        phi = 0.32825 * math.exp(-2.54931 * r / a) + 0.09219 * math.exp(-0.29182 * r / a) + \
            0.58110 * math.exp(-0.59231 * r / a)
        ft = 1.0 if r < 1 else 0.5 * (1 + math.cos(math.pi * (r - 1)))
        if abs(out["energy"] - ke * 74 * 74 / r * phi * ft) > 1e-6 * out["energy"]:
            return False
    return True


def _pin_trimer(m):
    mm = m.copy()
    mm.c_rad, mm.c_ang = np.eye(9), np.eye(5, 9)
    r = 2.9
    pos = np.array([[10.0, 10, 10], [10 + r, 10, 10], [10 + r / 2, 10 + r * math.sqrt(3) / 2, 10]])
    q = oracle.efv_cell(mm, pos, np.eye(3) * 40, desc=True)["desc"]
    x = 2 * (r / 4 - 1) ** 2 - 1
    fc = 0.5 * (1 + math.cos(math.pi * r / 4))
    g = np.array([0.5 * (math.cos(k * math.acos(x)) + 1) * fc for k in range(5)])
    ok = True
    for l in range(1, 5):
        ok &= np.allclose(q[0, 9 + 5 * (l - 1):9 + 5 * l], 2 * g * g * (1 + sp.eval_legendre(l, 0.5)), atol=1e-12)
    return bool(ok)


def _pin_fd_forces(m):
    s = nep_synth.tiny(n_cells=4)
    F = oracle.efv_cell(m, s.pos, s.h[0])["forces"]
    h = 1e-4
    for i in (0, 7):
        for a in range(3):
            p = s.pos.copy(); p[i, a] += h
            ep = oracle.efv_cell(m, p, s.h[0], virial=False)["energy"]
            p[i, a] -= 2 * h
            em = oracle.efv_cell(m, p, s.h[0], virial=False)["energy"]
            if abs(F[i, a] + (ep - em) / (2 * h)) > 1e-6 * max(1, abs(F[i, a])):
                return False
    return True


def _pin_fd_virial(m):
    pos, hc = nep_synth.bcc_lattice(3, 3, 3)
    pos = pos + np.random.default_rng(2).normal(0, 0.08, pos.shape)
    W = oracle.efv_cell(m, pos, hc)["virial"]
    h = 1e-5
    for a, b in ((0, 0), (0, 1), (2, 1)):
        eps = np.zeros((3, 3)); eps[b, a] = h
        ep = oracle.efv_cell(m, pos @ (np.eye(3) + eps), hc @ (np.eye(3) + eps), virial=False)["energy"]
        em = oracle.efv_cell(m, pos @ (np.eye(3) - eps), hc @ (np.eye(3) - eps), virial=False)["energy"]
        if abs(W[a, b] + (ep - em) / (2 * h)) > 2e-6 * max(1, np.abs(W).max()):
            return False
    return True


def _pin_network_torch(m):
    import torch
    s = nep_synth.tiny(n_cells=4)
    out = oracle.efv_cell(m, s.pos, s.h[0], desc=True)
    q = torch.tensor(out["desc"] * m.q_scale)
    hid = torch.nn.functional.linear(q, torch.tensor(m.w0), -torch.tensor(m.b0)).tanh()
    U = (hid @ torch.tensor(m.w1)).numpy() - m.b1
    mask = np.ones(s.n_atoms, bool)
    for i, j, _ in s.meta["pulled_pairs"]:
        mask[i] = mask[j] = False
    return bool(np.allclose(out["energy_atom"][mask], U[mask], atol=1e-10))


def _pin_supercell(m):
    pos, h = nep_synth.bcc_lattice(1, 2, 2)
    pos = pos + np.random.default_rng(5).normal(0, 0.1, pos.shape)
    small = oracle.efv_cell(m, pos, h, method=0)
    R = (6, 3, 3)
    big = np.concatenate([pos + (a * h[0] + b * h[1] + c * h[2]) for c in range(3) for b in range(3)
                          for a in range(6)])
    sup = oracle.efv_cell(m, big, h * np.array(R)[:, None])
    return bool(np.allclose(sup["energy_atom"][:pos.shape[0]], small["energy_atom"], atol=1e-9))


def _pin_addition_theorem(m):
    # one atom's angular descriptor vs a library (scipy) factorised evaluation
    s = nep_synth.diffbatch(n_cells=4)
    pos, h = s.cell(1)
    q = oracle.efv_cell(m, pos, h, desc=True)["desc"][0]
    start, j, n, r = oracle.pairs(pos, h, (1, 1, 1), 4.0, method=0)
    sacc = np.zeros((5, 5, 9), dtype=complex)
    for jj, nn, rr in zip(j[start[0]:start[1]], n[start[0]:start[1]], r[start[0]:start[1]]):
        d = pos[jj] + nn @ h - pos[0]
        x = 2 * (rr / 4 - 1) ** 2 - 1
        fc = 0.5 * (1 + math.cos(math.pi * rr / 4))
        f = np.array([0.5 * (np.polynomial.chebyshev.chebval(x, np.eye(9)[k]) + 1) * fc for k in range(9)])
        g = m.c_ang @ f
        th, ph = math.acos(d[2] / rr), math.atan2(d[1], d[0])
        for l in range(1, 5):
            for mm in range(-l, l + 1):
                sacc[:, l, mm + l] += g * sp.sph_harm_y(l, mm, th, ph)
    for l in range(1, 5):
        ref = 4 * math.pi / (2 * l + 1) * np.sum(np.abs(sacc[:, l, :2 * l + 1]) ** 2, axis=1)
        if not np.allclose(q[9 + 5 * (l - 1):9 + 5 * l], ref, rtol=1e-9, atol=1e-10):
            return False
    return True


def _pin_chebyshev(m):
    T, _ = oracle.chebyshev(9, math.cos(0.7))
    return bool(np.allclose(T, np.cos(np.arange(9) * 0.7), atol=1e-12))


def _pin_legendre(m):
    P, _ = oracle.legendre(0.3)
    return bool(np.allclose(P, [sp.eval_legendre(l, 0.3) for l in range(5)], atol=1e-14))


PINS = [_pin_zbl_dimer, _pin_trimer, _pin_fd_forces, _pin_fd_virial, _pin_network_torch, _pin_supercell,
        _pin_addition_theorem, _pin_chebyshev, _pin_legendre]


def test_pins_hold_on_the_real_oracle():
    m = nep_synth.random_model()
    for pin in PINS:
        assert pin(m), pin.__name__


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_planted_mistake_is_caught(mutation):
    m = nep_synth.random_model()
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    saved = oracle._lib
    try:
        oracle._lib = _with_lib(_build(mutation, tmp))
        failed = [p.__name__ for p in PINS if not p(m)]
    finally:
        oracle._lib = saved
        shutil.rmtree(tmp, ignore_errors=True)
    assert failed, f"no pin caught the mutation {mutation}"
