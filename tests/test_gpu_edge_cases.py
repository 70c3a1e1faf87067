"""Edge cases of the HIP path through the C ABI: the device-side errors
(list capacity, overlapping atoms, non-finite positions, step underflow),
empty and over-capacity inputs, isolated atoms and clusters in open cells
against the oracle, and the largest system one context takes (2^26 atoms)."""
import numpy as np
import pytest

import nep_synth
import oracle
from gpu_common import E_ATOM_TOL, F_REL_TOL, force_errors, gpu_available, model

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _sys(pos, h, pbc=(1, 1, 1), vel=None):
    s = nep_synth._single(np.asarray(pos, dtype=np.float64), np.asarray(h, dtype=np.float64), vel)
    s.pbc = tuple(pbc)
    return s


def test_list_capacity_overflow_is_reported_then_recovered():
    import paper_2305_08140_amd as nep
    m = model()
    s = nep_synth.tiny()
    sysd = nep.DeviceSystem.from_synth(s)
    small = nep.Context(m, s.n_atoms, 1, max_neigh_ang=8, max_neigh_rad=16)
    with pytest.raises(nep.NepError) as e:
        small.nep_build_neighbors(sysd)
    assert e.value.code == nep.NEP_E_NEIGH_OVERFLOW
    # the error was reported (and cleared); the truncated lists stay unusable:
    # an evaluation on them reports an error instead of returning numbers
    out_small = nep.EFV(s.n_atoms, 1)
    for _ in range(2):
        with pytest.raises(nep.NepError) as e:
            small.nep_compute_efv(sysd, out_small)
        assert e.value.code == nep.NEP_E_STATE
    # and an MD chunk on them rebuilds first (overflowing again)
    with pytest.raises(nep.NepError) as e:
        small.nep_step_verlet(sysd, 1, out_small, dt_max=1.0, forces_valid=True)
    assert e.value.code == nep.NEP_E_NEIGH_OVERFLOW
    need_a, need_r = small.nep_required_neighbors()
    # bcc within 5 A and between 5 and 7 A, plus thermal spread
    assert 26 <= need_a <= 40 and 55 <= need_r <= 80
    ok = nep.Context(m, s.n_atoms, 1, max_neigh_ang=need_a, max_neigh_rad=need_r)
    out = nep.EFV(s.n_atoms, 1)
    ok.nep_build_neighbors(sysd)
    ok.nep_compute_efv(sysd, out)
    ref = oracle.efv_cell(m, s.pos, s.h[0])
    e_all, _ = force_errors(out.forces().cpu().numpy().astype(np.float64), ref["forces"])
    assert e_all <= F_REL_TOL


def test_overlapping_atoms_are_reported():
    import paper_2305_08140_amd as nep
    m = model()
    pos, h = nep_synth.bcc_lattice(6, 6, 6)
    pos[1] = pos[0] + np.array([1e-4, 0.0, 0.0])
    s = _sys(pos, h)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_build_neighbors(sysd)
    with pytest.raises(nep.NepError) as e:
        ctx.nep_compute_efv(sysd, out)
    assert e.value.code == nep.NEP_E_OVERLAP


def test_non_finite_position_is_reported():
    import paper_2305_08140_amd as nep
    m = model()
    pos, h = nep_synth.bcc_lattice(6, 6, 6)
    pos[7, 1] = np.nan
    s = _sys(pos, h)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    with pytest.raises(nep.NepError) as e:
        ctx.nep_build_neighbors(sysd)
    assert e.value.code == nep.NEP_E_NONFINITE


def test_step_underflow_is_reported():
    import paper_2305_08140_amd as nep
    m = model()
    s = nep_synth.mid(n_cells=8)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    # 300 K atoms move ~0.01 A/fs: a 1e-6 A cap asks for ~1e-4 fs, below dt_min
    with pytest.raises(nep.NepError) as e:
        ctx.nep_step_verlet(sysd, 3, out, dt_max=1.0, max_disp=1e-6, dt_min=0.5)
    assert e.value.code == nep.NEP_E_DT_UNDERFLOW
    # positions untouched by the refused steps
    assert np.array_equal(sysd.positions().cpu().numpy(), s.pos)


def test_empty_and_over_capacity_inputs_are_refused():
    import ctypes as C
    import paper_2305_08140_amd as nep
    m = model()
    pos, h = nep_synth.bcc_lattice(4, 4, 4)
    s = _sys(pos, h)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, 64, 1)          # holds 64 of the 128 atoms
    with pytest.raises(nep.NepError) as e:
        ctx.nep_build_neighbors(sysd)
    assert e.value.code == nep.NEP_E_ARG
    cs = sysd.c_struct()
    cs.n_atoms = 0
    assert nep.lib().nep_build_neighbors(ctx._ptr, C.byref(cs), None) == nep.NEP_E_ARG


@pytest.mark.parametrize("kind", ["single", "dimer_zbl", "trimer"])
def test_isolated_atoms_in_open_cells(kind):
    # open boundaries on every axis: a lone atom (U of the zero descriptor, no
    # force), a dimer inside the ZBL range, an equilateral trimer
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    c = np.array([15.0, 15.0, 15.0])
    if kind == "single":
        pos = c[None, :]
    elif kind == "dimer_zbl":
        pos = np.stack([c, c + np.array([1.3, 0.4, -0.2])])
    else:
        a = 2.6
        pos = np.stack([c, c + np.array([a, 0.0, 0.0]), c + np.array([0.5 * a, 0.5 * a * np.sqrt(3.0), 0.0])])
    h = np.eye(3) * 30.0
    s = _sys(pos, h, pbc=(0, 0, 0))
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    ref = oracle.efv_cell(m, pos, h, pbc=(0, 0, 0))
    F = out.forces().cpu().numpy().astype(np.float64)
    assert abs(out.energy.item() - ref["energy"]) / s.n_atoms <= E_ATOM_TOL
    if kind == "single":
        assert np.all(F == 0.0)
        assert np.all(out.virial.cpu().numpy() == 0.0)
    else:
        assert np.linalg.norm(F - ref["forces"]) <= F_REL_TOL * np.linalg.norm(ref["forces"])
        W = out.virial.cpu().numpy().reshape(3, 3)
        assert np.linalg.norm(W - ref["virial"]) <= 1e-5 * np.linalg.norm(ref["virial"]) + 1e-6 * s.n_atoms


def test_largest_system_of_one_context():
    # 2^26 atoms (256 x 256 x 512 bcc cells, the local-index limit of a list
    # entry), sigma = 0.05 A: sampled atoms against the oracle, net force and
    # virial symmetry over everything
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    pos, h = nep_synth.bcc_lattice(256, 256, 512)
    n = pos.shape[0]
    assert n == 1 << 26
    pos += np.random.default_rng(13).normal(0.0, 0.05, pos.shape)
    s = _sys(pos, h)
    sysd = nep.DeviceSystem.from_synth(s)
    print(f"[2^26] {n} atoms on the device", flush=True)
    ctx = nep.Context(m, n, 1)
    out = nep.EFV(n, 1, energy_atom=False)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    print("[2^26] evaluated, oracle next", flush=True)
    F = out.forces().double()
    assert float(F.sum(0).abs().max()) <= 1e-6 * float(F.abs().sum())
    W = out.virial.cpu().numpy().reshape(3, 3)
    assert np.abs(W - W.T).max() <= 1e-5 * np.abs(W).max()
    idx = np.sort(np.random.default_rng(14).choice(n, size=128, replace=False))
    idx[-1] = n - 1
    ref = oracle.efv_cell(m, pos, h, targets=idx, virial=False)
    Fs = F.cpu().numpy()[idx]
    err = np.linalg.norm(Fs - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[2^26] sampled force rel err {err:.2e}", flush=True)
    assert err <= F_REL_TOL


def test_update_neighbors_keeps_valid_lists_and_rebuilds_stale_ones():
    # nep_update_neighbors: after moves below skin/2 the lists built before
    # still hold every pair within the cutoffs; after a few atoms jumped by
    # 1.6 A they do not (an evaluation on them misses pairs, and differs from
    # the FP64 oracle), and the update must rebuild them (device decision)
    import torch
    import paper_2305_08140_amd as nep
    m = model()
    s = nep_synth.mid(n_cells=20)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    rng = np.random.default_rng(31)

    def set_pos(p):
        t = torch.tensor(p, device="cuda")
        sysd.x.copy_(t[:, 0])
        sysd.y.copy_(t[:, 1])
        sysd.z.copy_(t[:, 2])

    def check(label, idx, expect_ok):
        torch.cuda.synchronize()
        pos = sysd.positions().cpu().numpy()
        F = out.forces().cpu().numpy().astype(np.float64)[idx]
        ref = oracle.efv_cell(m, pos, s.h[0], targets=idx, virial=False)["forces"]
        err = np.linalg.norm(F - ref) / np.linalg.norm(ref)
        print(f"[update neighbors] {label}: sampled force rel err {err:.3e}", flush=True)
        assert (err <= F_REL_TOL) == expect_ok, (label, err)

    # small moves (0.15 A per component at most): the kept lists are complete
    p0 = s.pos + rng.uniform(-0.15, 0.15, s.pos.shape)
    set_pos(p0)
    ctx.nep_update_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    idx = np.sort(rng.choice(s.n_atoms, 128, replace=False))
    check("moves below skin/2", idx, True)
    # 16 atoms jump 1.6 A along x: the old lists miss pairs around them
    movers = np.sort(rng.choice(s.n_atoms, 16, replace=False))
    p1 = p0.copy()
    p1[movers, 0] += 1.6
    set_pos(p1)
    ctx.nep_compute_efv(sysd, out)        # on the stale lists
    check("stale lists", movers, False)
    ctx.nep_update_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    check("after the update", movers, True)
