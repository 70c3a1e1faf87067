"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these tests compares the oracle with itself: each one checks it
against a library routine (numpy / scipy / torch), a closed form, a
constant printed in the paper (tests/golden/), a finite difference or an
invariant that the definition implies.
"""
import math
import os

import numpy as np
import pytest
import scipy.constants as sc
import scipy.special as sp

import nep_synth
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _zbl_constants():
    rows, kv = [], {}
    with open(os.path.join(GOLDEN, "zbl_ww_constants.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            a, b = line.split()
            try:
                rows.append((float(a), float(b)))
            except ValueError:
                kv[a] = float(b)
    return np.array(rows), kv


def _model(**kw):
    m = nep_synth.random_model()
    for k, v in kw.items():
        setattr(m, k, v)
    return m


# ------------------------------------------------------------------ ZBL, Eqs. 2-4


def test_coulomb_constant_matches_alpha_hbar_c():
    # e^2/(4 pi eps0) = alpha * hbar * c, a different route than e and eps0
    ref = sc.fine_structure * sc.hbar * sc.c / sc.e * 1e10
    assert abs(oracle.coulomb() - ref) / ref < 1e-9


def test_tersoff_switch_is_tersoffs_sine_form():
    # Tersoff's cutoff with R = (r1 + r2)/2, D = (r2 - r1)/2: 1/2 - 1/2 sin(pi/2 (r - R)/D)
    R, D = 1.5, 0.5
    for r in np.linspace(0.0, 2.5, 251):
        f, df = oracle.tersoff_fc(r)
        if r < R - D:
            ref = 1.0
        elif r > R + D:
            ref = 0.0
        else:
            ref = 0.5 - 0.5 * math.sin(0.5 * math.pi * (r - R) / D)
        assert abs(f - ref) < 1e-14
    for r in [1.1, 1.37, 1.5, 1.81, 1.95]:
        h = 1e-6
        fd = (oracle.tersoff_fc(r + h)[0] - oracle.tersoff_fc(r - h)[0]) / (2 * h)
        assert abs(oracle.tersoff_fc(r)[1] - fd) < 1e-8


def test_zbl_matches_printed_screening_function():
    rows, kv = _zbl_constants()
    Z = kv["Z"]
    a = kv["A"] / (2.0 * Z ** kv["exponent"])
    ke = sc.fine_structure * sc.hbar * sc.c / sc.e * 1e10
    for r in [0.05, 0.3, 0.5, 0.8, 0.99, 1.2, 1.5, 1.9]:
        phi = float(np.sum(rows[:, 0] * np.exp(-rows[:, 1] * r / a)))
        ft = 1.0 if r < kv["r1"] else 0.5 * (1 + math.cos(math.pi * (r - kv["r1"]) / (kv["r2"] - kv["r1"])))
        ref = ke * Z * Z / r * phi * ft
        U, _ = oracle.zbl(r)
        assert abs(U - ref) / ref < 1e-9, r
    assert oracle.zbl(2.0)[0] == 0.0 and oracle.zbl(2.5) == (0.0, 0.0)


def test_zbl_coulomb_limit():
    # r -> 0: U r / (k_e Z^2) -> phi(0) = sum of the printed c_q (1.00154)
    rows, kv = _zbl_constants()
    ke = sc.fine_structure * sc.hbar * sc.c / sc.e * 1e10
    r = 1e-7
    U, _ = oracle.zbl(r)
    assert abs(U * r / (ke * kv["Z"] ** 2) - rows[:, 0].sum()) < 1e-5
    assert abs(rows[:, 0].sum() - 1.00154) < 1e-12


def test_zbl_screening_length_near_universal_value():
    # universal ZBL: a_U = 0.8854 a_0 / (Z1^0.23 + Z2^0.23); the paper's 0.46848 A is within 2e-4
    _, kv = _zbl_constants()
    a0 = sc.physical_constants["Bohr radius"][0] * 1e10
    assert abs(kv["A"] - 0.8854 * a0) / kv["A"] < 2e-4


@pytest.mark.parametrize("r", [0.3, 0.5, 0.8, 0.95, 1.05, 1.3, 1.5, 1.7, 1.95])
def test_zbl_force_is_minus_gradient(r):
    h = 1e-6
    U, dU = oracle.zbl(r)
    fd = (oracle.zbl(r + h)[0] - oracle.zbl(r - h)[0]) / (2 * h)
    assert abs(dU - fd) <= 1e-7 * max(1.0, abs(dU))


def test_dimer_with_network_off_is_pure_zbl():
    # Eq. 1: each atom carries half of U_ZBL; with the network output switched off
    # (w1 = 0, b1 = 0) the dimer energy is U_ZBL(r), the force +-dU/dr along the bond
    m = _model()
    m.w1 = np.zeros_like(m.w1)
    m.b1 = 0.0
    for r in [0.5, 0.8, 1.2, 1.6, 1.9, 2.3]:
        s = nep_synth.dimer(r)
        out = oracle.efv_cell(m, s.pos, s.h[0])
        U, dU = oracle.zbl(r)
        assert abs(out["energy"] - U) <= 1e-10 * max(1.0, U)
        assert np.allclose(out["forces"][0], [dU, 0, 0], rtol=1e-12, atol=1e-12)
        assert np.allclose(out["forces"][1], [-dU, 0, 0], rtol=1e-12, atol=1e-12)
        # virial of an isolated pair: W_xx = -dU/dr * r
        assert abs(out["virial"][0, 0] + dU * r) <= 1e-9 * max(1.0, abs(dU * r))
        assert np.allclose(out["energy_atom"], 0.5 * U)


# ------------------------------------------------------------------ descriptor pieces


def test_chebyshev_recurrence_matches_cos_k_t_and_numpy():
    for t in np.linspace(0.0, math.pi, 17):
        T, dT = oracle.chebyshev(12, math.cos(t))
        assert np.allclose(T, np.cos(np.arange(12) * t), atol=1e-13)
    for x in np.linspace(-1, 1, 9):
        T, dT = oracle.chebyshev(12, x)
        for k in range(12):
            e = np.zeros(k + 1)
            e[k] = 1.0
            assert abs(T[k] - np.polynomial.chebyshev.chebval(x, e)) < 1e-12
            assert abs(dT[k] - np.polynomial.chebyshev.chebval(x, np.polynomial.chebyshev.chebder(e))) < 1e-10


def test_legendre_matches_scipy():
    for c in np.linspace(-1, 1, 21):
        P, dP = oracle.legendre(c)
        for l in range(5):
            assert abs(P[l] - sp.eval_legendre(l, c)) < 1e-14
            h = 1e-6
            fd = (sp.eval_legendre(l, c + h) - sp.eval_legendre(l, c - h)) / (2 * h)
            assert abs(dP[l] - fd) < 1e-7


def _fc(r, rc):
    return 0.5 * (1 + np.cos(np.pi * r / rc)) if r < rc else 0.0


def _basis_np(K, r, rc):
    x = 2 * (r / rc - 1) ** 2 - 1
    return np.array([0.5 * (np.polynomial.chebyshev.chebval(x, np.eye(K)[k]) + 1) * _fc(r, rc)
                     for k in range(K)])


def test_basis_matches_numpy_chebyshev_and_fd():
    for rc in (4.0, 6.0):
        for r in np.linspace(0.2, rc - 1e-3, 23):
            f, df = oracle.basis(9, r, rc)
            assert np.allclose(f, _basis_np(9, r, rc), atol=1e-13)
            h = 1e-6
            fd = (oracle.basis(9, r + h, rc)[0] - oracle.basis(9, r - h, rc)[0]) / (2 * h)
            assert np.allclose(df, fd, atol=1e-7)
        f, _ = oracle.basis(9, rc + 0.1, rc)
        assert np.all(f == 0.0)


def test_dimer_descriptor_with_identity_coefficients():
    # with c = I the radial functions are the basis itself (the NEP1 special case):
    # q_n = f_n(r); a single angular neighbour gives q_nl = f_n(r)^2 P_l(1) = f_n(r)^2
    m = _model(c_rad=np.eye(9), c_ang=np.eye(5, 9))
    for r in [2.2, 2.741, 3.5, 3.9, 4.5, 5.9]:
        s = nep_synth.dimer(r)
        q = oracle.efv_cell(m, s.pos, s.h[0], desc=True)["desc"]
        fR = _basis_np(9, r, 6.0)
        fA = _basis_np(9, r, 4.0)[:5]
        for i in range(2):
            assert np.allclose(q[i, :9], fR, atol=1e-13)
            for l in range(1, 5):
                assert np.allclose(q[i, 9 + 5 * (l - 1):9 + 5 * l], fA ** 2, atol=1e-13)


def test_equilateral_trimer_angular_descriptor():
    # two neighbours at equal distance and 60 degrees: q_nl = 2 g^2 (1 + P_l(1/2))
    m = _model(c_rad=np.eye(9), c_ang=np.eye(5, 9))
    r = 2.9
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0],
                    [10.0 + r / 2, 10.0 + r * math.sqrt(3) / 2, 10.0]])
    q = oracle.efv_cell(m, pos, np.eye(3) * 40.0, desc=True)["desc"]
    g = _basis_np(9, r, 4.0)[:5]
    for l in range(1, 5):
        ref = 2 * g * g * (1 + sp.eval_legendre(l, 0.5))
        assert np.allclose(q[0, 9 + 5 * (l - 1):9 + 5 * l], ref, atol=1e-13)
    assert [sp.eval_legendre(l, 0.5) for l in range(1, 5)] == pytest.approx([0.5, -0.125, -0.4375, -0.2890625])


def _factorised_descriptor(m, pos, h, i):
    """Descriptor of atom i from the addition theorem with scipy's complex
    spherical harmonics and numpy's Chebyshev series (library route)."""
    start, j, n, r = oracle.pairs(pos, h, (1, 1, 1), m.rc_rad, method=0)
    q = np.zeros(m.dim)
    sl = slice(start[i], start[i + 1])
    for jj, nn, rr in zip(j[sl], n[sl], r[sl]):
        fR = _basis_np(m.k_rad, rr, m.rc_rad)
        q[:m.n_rad] += m.c_rad @ fR
    s = np.zeros((m.n_ang, m.l_max + 1, 2 * m.l_max + 1), dtype=complex)
    for jj, nn, rr in zip(j[sl], n[sl], r[sl]):
        if rr >= m.rc_ang:
            continue
        d = pos[jj] + nn @ h - pos[i]
        g = m.c_ang @ _basis_np(m.k_ang, rr, m.rc_ang)
        theta = math.acos(d[2] / rr)
        phi = math.atan2(d[1], d[0])
        for l in range(1, m.l_max + 1):
            for mm in range(-l, l + 1):
                s[:, l, mm + l] += g * sp.sph_harm_y(l, mm, theta, phi)
    for l in range(1, m.l_max + 1):
        q[m.n_rad + m.n_ang * (l - 1): m.n_rad + m.n_ang * l] = \
            4 * math.pi / (2 * l + 1) * np.sum(np.abs(s[:, l, :2 * l + 1]) ** 2, axis=1)
    return q


def test_descriptor_matches_addition_theorem_route():
    m = nep_synth.random_model()
    s = nep_synth.diffbatch()
    for c in [0, 7, 100]:
        pos, h = s.cell(c)
        q = oracle.efv_cell(m, pos, h, desc=True)["desc"]
        for i in [0, pos.shape[0] // 2, pos.shape[0] - 1]:
            ref = _factorised_descriptor(m, pos, h, i)
            assert np.allclose(q[i], ref, rtol=1e-10, atol=1e-11), (c, i)


def test_network_matches_torch():
    torch = pytest.importorskip("torch")
    m = nep_synth.random_model()
    s = nep_synth.tiny()
    out = oracle.efv_cell(m, s.pos, s.h[0], desc=True)
    q = torch.tensor(out["desc"] * m.q_scale)
    hid = torch.nn.functional.linear(q, torch.tensor(m.w0), -torch.tensor(m.b0)).tanh()
    U = torch.nn.functional.linear(hid, torch.tensor(m.w1)[None],
                                   torch.tensor([-m.b1], dtype=torch.float64))[:, 0].numpy()
    # atoms in a ZBL pair carry half of it on top of the network energy
    mask = np.ones(s.n_atoms, bool)
    for i, j, _ in s.meta["pulled_pairs"]:
        mask[i] = mask[j] = False
    assert np.allclose(out["energy_atom"][mask], U[mask], rtol=1e-12, atol=1e-12)
    for i, j, d in s.meta["pulled_pairs"]:
        Uz, _ = oracle.zbl(np.linalg.norm(s.pos[j] - s.pos[i]))
        assert abs(out["energy_atom"][i] - U[i] - 0.5 * Uz) < 1e-9 * max(1, Uz)


# ------------------------------------------------------------------ forces, virial


def _energy(m, pos, h):
    return oracle.efv_cell(m, pos, h, virial=False)["energy"]


def test_forces_are_minus_gradient_fd():
    m = nep_synth.random_model()
    s = nep_synth.tiny()
    out = oracle.efv_cell(m, s.pos, s.h[0])
    F = out["forces"]
    zbl_atoms = [p[0] for p in s.meta["pulled_pairs"]]
    h = 1e-4
    for i in [0, 1, 777] + zbl_atoms:
        for a in range(3):
            p = s.pos.copy()
            p[i, a] += h
            ep = _energy(m, p, s.h[0])
            p[i, a] -= 2 * h
            em = _energy(m, p, s.h[0])
            fd = -(ep - em) / (2 * h)
            assert abs(F[i, a] - fd) <= 1e-6 * max(1.0, abs(F[i, a])), (i, a, F[i, a], fd)


def test_virial_is_minus_strain_derivative():
    m = nep_synth.random_model()
    s = nep_synth.diffbatch()
    pos, hc = s.cell(3)
    W = oracle.efv_cell(m, pos, hc)["virial"]
    h = 1e-5
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3))
            eps[b, a] = h          # W_ab = -dE/d eps_ba for x -> x (I + eps)
            Fp, Fm = np.eye(3) + eps, np.eye(3) - eps
            ep = _energy(m, pos @ Fp, hc @ Fp)
            em = _energy(m, pos @ Fm, hc @ Fm)
            fd = -(ep - em) / (2 * h)
            assert abs(W[a, b] - fd) <= 2e-6 * max(1.0, np.abs(W).max()), (a, b, W[a, b], fd)


def test_cluster_virial_is_sum_r_outer_f():
    m = nep_synth.random_model()
    rng = np.random.default_rng(0)
    pos, _ = nep_synth.bcc_lattice(2, 2, 2)
    pos = pos + rng.normal(0, 0.1, pos.shape) + 20.0
    out = oracle.efv_cell(m, pos, np.eye(3) * 60.0, pbc=(0, 0, 0))
    F = out["forces"]
    W = np.einsum("ia,ib->ab", F, pos)
    assert np.allclose(out["virial"], W, rtol=1e-10, atol=1e-10)
    assert np.allclose(F.sum(0), 0.0, atol=1e-11)


# ------------------------------------------------------------------ invariants


def test_perfect_bcc_symmetry():
    m = nep_synth.random_model()
    pos, h = nep_synth.bcc_lattice(4, 4, 4)
    out = oracle.efv_cell(m, pos, h)
    assert np.abs(out["forces"]).max() < 1e-12
    assert np.ptp(out["energy_atom"]) < 1e-12
    W = out["virial"]
    assert np.abs(W - np.diag(np.diag(W))).max() < 1e-10
    assert np.ptp(np.diag(W)) < 1e-10


def test_translation_rotation_permutation():
    m = nep_synth.random_model()
    s = nep_synth.tiny()
    pos, h = s.pos, s.h[0]
    ref = oracle.efv_cell(m, pos, h)
    assert np.allclose(ref["forces"].sum(0), 0.0, atol=1e-9)
    # translation
    t = oracle.efv_cell(m, pos + np.array([0.37, -1.1, 2.9]), h)
    assert abs(t["energy"] - ref["energy"]) < 1e-9
    assert np.allclose(t["forces"], ref["forces"], atol=1e-9)
    # rotation of the whole periodic system (cell and atoms together)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    r = oracle.efv_cell(m, pos @ Q, h @ Q)
    assert abs(r["energy"] - ref["energy"]) < 1e-8
    assert np.allclose(r["forces"], ref["forces"] @ Q, atol=1e-8)
    assert np.allclose(r["virial"], Q.T @ ref["virial"] @ Q, atol=1e-7)
    # permutation
    p = rng.permutation(pos.shape[0])
    pr = oracle.efv_cell(m, pos[p], h)
    assert abs(pr["energy"] - ref["energy"]) < 1e-9
    assert np.allclose(pr["forces"], ref["forces"][p], atol=1e-9)


def test_small_cell_images_equal_supercell():
    # every periodic image counts: an 8-atom strained cell and its 4x4x4 replica
    # (large enough for the binned search) give the same energy per atom
    m = nep_synth.random_model()
    rng = np.random.default_rng(5)
    pos, h = nep_synth.bcc_lattice(1, 2, 2)
    pos = pos + rng.normal(0, 0.1, pos.shape)
    eps = np.array([[0.02, 0.01, -0.015], [0.01, -0.01, 0.02], [-0.015, 0.02, 0.03]])
    pos, h = pos @ (np.eye(3) + eps), h @ (np.eye(3) + eps)
    small = oracle.efv_cell(m, pos, h, method=0)
    R = (6, 3, 3)
    reps = [pos + (a * h[0] + b * h[1] + c * h[2]) for c in range(R[2]) for b in range(R[1])
            for a in range(R[0])]
    big = np.concatenate(reps)
    H = h * np.array(R)[:, None]
    sup = oracle.efv_cell(m, big, H)
    n = pos.shape[0]
    assert np.allclose(sup["energy_atom"][:n], small["energy_atom"], atol=1e-10)
    assert np.allclose(sup["forces"][:n], small["forces"], atol=1e-9)
    assert np.allclose(sup["virial"], small["virial"] * np.prod(R), rtol=1e-9, atol=1e-8)


def test_neighbour_sets_brute_force_vs_binned():
    s = nep_synth.tiny()
    a = oracle.pairs(s.pos, s.h[0], (1, 1, 1), 7.0, method=0)
    b = oracle.pairs(s.pos, s.h[0], (1, 1, 1), 7.0, method=1)
    assert np.array_equal(a[0], b[0])
    for i in [0, 1, 999, 1999]:
        sa = {(int(j), tuple(n)) for j, n in zip(a[1][a[0][i]:a[0][i + 1]], a[2][a[0][i]:a[0][i + 1]])}
        sb = {(int(j), tuple(n)) for j, n in zip(b[1][b[0][i]:b[0][i + 1]], b[2][b[0][i]:b[0][i + 1]])}
        assert sa == sb
    # perfect bcc shell counts below 6 A and 4 A: 8+6+12+24+8 = 58 and 8+6 = 14
    pos, h = nep_synth.bcc_lattice(6, 6, 6)
    st, _, _, _ = oracle.pairs(pos, h, (1, 1, 1), 6.0, method=1)
    assert np.all(np.diff(st) == 58)
    st, _, _, _ = oracle.pairs(pos, h, (1, 1, 1), 4.0, method=1)
    assert np.all(np.diff(st) == 14)


# ------------------------------------------------------------------ dynamics


def test_nve_energy_conservation_and_second_order():
    m = nep_synth.random_model()
    s = nep_synth.mid(n_cells=4)
    errs = []
    for dt in (2.0, 1.0):
        n = int(round(100 / dt))
        _, _, _, log = oracle.velocity_verlet(m, s.pos, s.vel, s.h[0], s.mass, n, dt_max=dt, record=True)
        et = np.array([x["epot"] + x["ekin"] for x in log])
        errs.append(np.abs(et - et[0]).max() / s.n_atoms)
    assert errs[1] < 1e-4
    # velocity Verlet is second order: halving dt cuts the energy error about 4x
    assert 2.5 < errs[0] / errs[1] < 6.0


def test_adaptive_time_step_caps_displacement():
    m = nep_synth.random_model()
    s = nep_synth.mid(n_cells=4)
    vel = s.vel.copy()
    vel[5] = nep_synth.speed_for_energy(1000.0) * np.array([0.6, 0.8, 0.0])
    _, _, _, log = oracle.velocity_verlet(m, s.pos, vel, s.h[0], s.mass, 5, dt_max=1.0, d_max=0.015,
                                          record=True)
    for x in log:
        assert x["dt"] <= 1.0
    assert abs(log[0]["dt"] - 0.015 / nep_synth.speed_for_energy(1000.0)) < 1e-12


# ------------------------------------------------------------------ parameter gradients


def test_parameter_gradient_matches_finite_differences():
    # dE/dtheta (analytic, FP64) against central differences of the energy,
    # on every parameter group; h scaled to each parameter's size
    m = nep_synth.random_model()
    s = nep_synth.diffbatch()
    pos, hc = s.cell(11)
    g = oracle.param_grad_cell(m, pos, hc)
    theta = m.param_vector()
    assert g.shape == theta.shape == (81 + 45 + 870 + 30 + 30 + 1,)
    rng = np.random.default_rng(4)
    groups = {"c_rad": (0, 81), "c_ang": (81, 126), "w0": (126, 996), "b0": (996, 1026),
              "w1": (1026, 1056), "b1": (1056, 1057)}
    for name, (a, b) in groups.items():
        for p in rng.choice(np.arange(a, b), size=min(6, b - a), replace=False):
            h = 1e-5 * max(1.0, abs(theta[p]))
            tp, tm = theta.copy(), theta.copy()
            tp[p] += h
            tm[p] -= h
            ep = oracle.efv_cell(m.with_param_vector(tp), pos, hc, virial=False)["energy"]
            em = oracle.efv_cell(m.with_param_vector(tm), pos, hc, virial=False)["energy"]
            fd = (ep - em) / (2 * h)
            assert abs(g[p] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, p, g[p], fd)
    assert g[1056] == -pos.shape[0]      # dE/db1 = -N


def test_parameter_gradient_linear_in_output_weights():
    # E is linear in w1 and b1: E(theta) = w1 . dE/dw1 + b1 dE/db1 + (ZBL part)
    m = nep_synth.random_model()
    pos, h = nep_synth.bcc_lattice(3, 3, 3)
    pos = pos + np.random.default_rng(1).normal(0, 0.05, pos.shape)
    g = oracle.param_grad_cell(m, pos, h)
    E = oracle.efv_cell(m, pos, h)["energy"]
    assert abs(E - (m.w1 @ g[1026:1056] + m.b1 * g[1056])) < 1e-9 * max(1.0, abs(E))


def test_paper_size_model_forces_virial_and_identity_dimer():
    # the paper's hyperparameters (16 radial and 11 angular functions on as
    # many Chebyshev terms, 100 neurons): forces and virial by finite
    # differences, and the NEP1 special case c = I on a dimer
    m = nep_synth.random_model(size="paper")
    assert m.dim == 60 and m.w0.shape == (100, 60)
    pos, hc = nep_synth.bcc_lattice(3, 3, 3)
    pos = pos + np.random.default_rng(12).normal(0.0, 0.08, pos.shape)
    out = oracle.efv_cell(m, pos, hc)
    h = 1e-4
    for i in (0, 13, 40):
        for a in range(3):
            p = pos.copy(); p[i, a] += h
            ep = _energy(m, p, hc)
            p[i, a] -= 2 * h
            em = _energy(m, p, hc)
            assert abs(out["forces"][i, a] + (ep - em) / (2 * h)) <= 1e-6 * max(1.0, abs(out["forces"][i, a]))
    hs = 1e-5
    for a, b in ((0, 0), (1, 2)):
        eps = np.zeros((3, 3)); eps[b, a] = hs
        ep = _energy(m, pos @ (np.eye(3) + eps), hc @ (np.eye(3) + eps))
        em = _energy(m, pos @ (np.eye(3) - eps), hc @ (np.eye(3) - eps))
        assert abs(out["virial"][a, b] + (ep - em) / (2 * hs)) <= 2e-6 * max(1.0, np.abs(out["virial"]).max())
    mi = m.copy()
    mi.c_rad, mi.c_ang = np.eye(16), np.eye(11)
    for r in (2.3, 3.7, 5.5):
        s = nep_synth.dimer(r)
        q = oracle.efv_cell(mi, s.pos, s.h[0], desc=True)["desc"]
        assert np.allclose(q[0, :16], _basis_np(16, r, 6.0), atol=1e-13)
        fA = _basis_np(11, r, 4.0)
        for l in range(1, 5):
            assert np.allclose(q[0, 16 + 11 * (l - 1):16 + 11 * l], fA ** 2, atol=1e-13)


def test_paper_size_model_parameter_gradient_matches_finite_differences():
    # dE/dtheta of the paper-size model (16 x 16 radial and 11 x 11 angular
    # coefficients, 100 x 60 input weights) against central differences of
    # the energy on sampled parameters of every group, and dE/db1 = -N
    m = nep_synth.random_model(size="paper")
    pos, hc = nep_synth.bcc_lattice(3, 3, 3)
    pos = pos + np.random.default_rng(6).normal(0.0, 0.06, pos.shape)
    g = oracle.param_grad_cell(m, pos, hc)
    theta = m.param_vector()
    sizes = (256, 121, 6000, 100, 100, 1)
    assert g.shape == theta.shape == (sum(sizes),)
    o = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(8)
    for name, a, b in zip(("c_rad", "c_ang", "w0", "b0", "w1", "b1"), o[:-1], o[1:]):
        for p in rng.choice(np.arange(a, b), size=min(5, b - a), replace=False):
            h = 1e-5 * max(1.0, abs(theta[p]))
            tp, tm = theta.copy(), theta.copy()
            tp[p] += h
            tm[p] -= h
            ep = oracle.efv_cell(m.with_param_vector(tp), pos, hc, virial=False)["energy"]
            em = oracle.efv_cell(m.with_param_vector(tm), pos, hc, virial=False)["energy"]
            fd = (ep - em) / (2 * h)
            assert abs(g[p] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, p, g[p], fd)
    assert g[-1] == -pos.shape[0]
    # E is linear in w1 and b1 apart from the ZBL part (none at these spacings)
    E = oracle.efv_cell(m, pos, hc)["energy"]
    assert abs(E - (m.w1 @ g[o[4]:o[5]] + m.b1 * g[-1])) < 1e-9 * max(1.0, abs(E))
