"""Border thermostat (Nose-Hoover chain on the face layers, Sec. II.B) and foil
boundaries (open z, Table I foil rows) on the GPU, against the FP64 oracle."""
import numpy as np
import pytest

import nep_synth
import oracle
from gpu_common import E_ATOM_TOL, F_REL_TOL, force_errors, gpu_available, model

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

A = nep_synth.A_W


def _heat_up_system(n_cells=20, t0=100.0):
    # bcc W on lattice sites with Maxwell-Boltzmann velocities at t0
    s = nep_synth.mid(n_cells=n_cells)
    s.vel = s.vel * np.sqrt(t0 / 300.0)
    return s


def _kinetic(sysd, mass):
    v = sysd.velocities().double()
    return 0.5 * mass * float((v * v).sum()) / oracle.EV_PER_U_TO_A2_PER_FS2


def _compare(s, sysd, out, ref, pos_tol=1e-7, vel_tol=1e-8):
    pos_ref, vel_ref, F_ref, log = ref[:4]
    dp = np.abs(sysd.positions().cpu().numpy() - pos_ref).max()
    dv = np.abs(sysd.velocities().cpu().numpy() - vel_ref).max()
    e_all, _ = force_errors(out.forces().cpu().numpy().astype(np.float64), F_ref)
    de = abs(out.energy.item() - log[-1]["epot"]) / s.n_atoms
    print(f"[{s.name}] max |dx| {dp:.2e} A, max |dv| {dv:.2e} A/fs, force rel err {e_all:.2e}, "
          f"energy err {de:.2e} eV/atom", flush=True)
    assert dp < pos_tol and dv < vel_tol
    assert e_all <= F_REL_TOL
    assert de <= E_ATOM_TOL


def test_border_thermostat_trajectory():
    # 16,000 atoms at 100 K; the 3 a0 layers at all six faces held at 900 K by a
    # chain of 3 (tau 20 fs); 10 steps in two calls of 5 (the chain persists)
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    s = _heat_up_system()
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    th = dict(T=900.0, tau=20.0, border=3 * A, axes=(0, 1, 2), chain=3)
    st1 = ctx.nep_step_verlet(sysd, 5, out, dt_max=1.0, thermostat=th)
    st2 = ctx.nep_step_verlet(sysd, 5, out, dt_max=1.0, forces_valid=True, thermostat=th)
    torch.cuda.synchronize()
    ref = oracle.velocity_verlet_nhc(m, s.pos, s.vel, s.h[0], s.mass, 10, dt_max=1.0, temperature=900.0, tau=20.0,
                                     chain=3, thickness=3 * A, axes=(0, 1, 2), record=True)
    mask, ch = ref[4], ref[5]
    # 20^3 cells, 40 layers per axis of which 6 + 6 in the layer: 16000 (1 - (28/40)^3)
    assert st1["n_border"] == st2["n_border"] == int(mask.sum()) == 10512
    _compare(s, sysd, out, ref)
    log = ref[3]
    assert abs(st2["thermo_energy"] - ch.energy()) <= 1e-7 * abs(ch.energy()) + 1e-9 * s.n_atoms
    assert abs(st2["border_temperature"] - log[-1]["T_border"]) <= 1e-6 * log[-1]["T_border"]
    assert ch.v[0] < 0.0   # the chain is heating the layer (2K below N_f kT)


def test_empty_border_leaves_the_trajectory_unchanged():
    # a layer of zero thickness selects no atom: bit for bit the plain integrator
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    s = _heat_up_system(n_cells=12)
    res = []
    for th in (None, dict(T=900.0, tau=20.0, border=0.0, axes=(0, 1, 2), chain=3)):
        sysd = nep.DeviceSystem.from_synth(s)
        ctx = nep.Context(m, s.n_atoms, 1)
        out = nep.EFV(s.n_atoms, 1)
        st = ctx.nep_step_verlet(sysd, 8, out, dt_max=1.0, max_disp=0.01, thermostat=th)
        torch.cuda.synchronize()
        res.append((sysd.positions().cpu().numpy(), sysd.velocities().cpu().numpy(), st))
    assert res[1][2]["n_border"] == 0
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2]["dt_last"] == res[1][2]["dt_last"]


def test_extended_energy_is_conserved():
    # 300 steps from lattice sites at 300 K (equipartition halves the
    # temperature; the 3 a0 layers are held at 300 K, tau 100 fs): total +
    # kinetic energy changes by several meV/atom, the extended energy (plus the
    # chain's) stays put.  (A single chain substep per half step, as here, is
    # accurate when the layer is near its target; a 9x temperature jump with
    # tau = 20 fs makes the chain stiff and the oracle itself drifts.)
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    s = nep_synth.mid(n_cells=20)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    th = dict(T=300.0, tau=100.0, border=3 * A, axes=(0, 1, 2), chain=3)
    h, et = [], []
    first = True
    for _ in range(6):
        st = ctx.nep_step_verlet(sysd, 50, out, dt_max=1.0, forces_valid=not first, thermostat=th)
        first = False
        torch.cuda.synchronize()
        e = out.energy.item() + _kinetic(sysd, s.mass)
        et.append(e)
        h.append(e + st["thermo_energy"])
    et, h = np.array(et), np.array(h)
    work = np.abs(et - et[0]).max() / s.n_atoms
    drift = np.abs(h - h[0]).max() / s.n_atoms
    print(f"[heat] E+K change {work:.3e} eV/atom, extended-energy drift {drift:.3e} eV/atom", flush=True)
    assert work > 2e-3
    assert drift < 2e-3 * work


def test_foil_with_pka_trajectory():
    # foil of 20 x 20 x 24 cells (19,200 atoms), open along z, thermostat on the
    # x and y faces only (Sec. II.B), 1 keV PKA along <135> into the foil near
    # the top surface; adaptive step (0.01 A); 12 steps against the oracle
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    s = nep_synth.cascade((20, 20, 24), foil=True, pka_ev=1000.0)
    assert s.pbc == (1, 1, 0)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    th = dict(T=300.0, tau=100.0, border=3 * A, axes=(0, 1), chain=3)
    st = ctx.nep_step_verlet(sysd, 12, out, dt_max=1.0, max_disp=0.01, thermostat=th)
    torch.cuda.synchronize()
    ref = oracle.velocity_verlet_nhc(m, s.pos, s.vel, s.h[0], s.mass, 12, dt_max=1.0, d_max=0.01, pbc=s.pbc,
                                     temperature=300.0, tau=100.0, chain=3, thickness=3 * A, axes=(0, 1),
                                     record=True)
    assert st["n_border"] == int(ref[4].sum())
    assert abs(st["time"] - sum(x["dt"] for x in ref[3])) <= 1e-12
    _compare(s, sysd, out, ref)
    # the free surfaces: the top and bottom layers feel opposite net normal forces
    # (mirror images of each other on the ideal lattice; thermal noise averages out)
    lattice_z, _ = nep_synth.bcc_lattice(20, 20, 24)
    z = lattice_z[:, 2]
    F = out.forces().cpu().numpy().astype(np.float64)
    top, bottom = z > z.max() - 0.1, z < z.min() + 0.1
    pka = s.meta["pka"]
    top[pka] = bottom[pka] = False
    assert F[top, 2].mean() * F[bottom, 2].mean() < 0.0


def test_thermostat_argument_checks():
    import paper_2305_08140_amd as nep
    m = model()
    s = _heat_up_system(n_cells=8)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    good = dict(T=300.0, tau=100.0, border=3 * A, axes=(0, 1, 2), chain=3)
    for bad in (dict(chain=9), dict(tau=0.0), dict(T=-1.0), dict(border=-1.0), dict(axes=())):
        with pytest.raises(nep.NepError) as e:
            ctx.nep_step_verlet(sysd, 1, out, thermostat={**good, **bad})
        assert e.value.code == nep.NEP_E_ARG
    # a sheared cell is refused
    h = s.h[0].copy()
    h[1, 0] = 0.5
    sheared = nep_synth.System(pos=s.pos, vel=s.vel, cell_start=s.cell_start, h=h[None])
    sysd2 = nep.DeviceSystem.from_synth(sheared)
    with pytest.raises(nep.NepError) as e:
        ctx.nep_step_verlet(sysd2, 1, out, thermostat=good)
    assert e.value.code == nep.NEP_E_UNSUPPORTED
