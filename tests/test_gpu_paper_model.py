"""The paper-size model (16/11 radial/angular functions, 100 neurons;
Sec. III.A) on the GPU through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

import nep_synth
import oracle
from gpu_common import (E_ATOM_TOL, F_REL_TOL, W_ATOM_TOL, W_REL_TOL, force_errors, gpu_available, run_gpu,
                        zbl_atoms)

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def pmodel():
    return nep_synth.random_model(size="paper")


def _compare(s, ref, res, zbl, label):
    for c in range(s.n_cells):
        n_c = int(s.cell_start[c + 1] - s.cell_start[c])
        assert abs(res["energy"][c] - ref["energy"][c]) / n_c <= E_ATOM_TOL, (label, c)
        dW = np.linalg.norm(res["virial"][c] - ref["virial"][c])
        assert dW <= W_REL_TOL * np.linalg.norm(ref["virial"][c]) + W_ATOM_TOL * n_c, (label, c, dW)
    e_all, e_rest = force_errors(res["forces"], ref["forces"], zbl)
    print(f"[paper model {label}] force rel err all={e_all:.3e} non-ZBL={e_rest:.3e}", flush=True)
    assert e_all <= F_REL_TOL and e_rest <= F_REL_TOL


def test_tiny_matches_oracle():
    m = pmodel()
    s = nep_synth.tiny()
    ref = oracle.efv_system(m, s)
    res, *_ = run_gpu(m, s)
    _compare(s, ref, res, zbl_atoms(s.pos, s.h[0]), "tiny")
    assert np.abs(res["energy_atom"] - ref["energy_atom"]).max() <= 1e-5


def test_small_strained_cells_with_images():
    m = pmodel()
    full = nep_synth.batch()
    sizes = np.diff(full.cell_start)
    pick = [int(c) for c in np.argsort(sizes)[:24]] + list(range(100, 4096, 400))
    pos = np.concatenate([full.cell(c)[0] for c in pick])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in pick])]).astype(np.int64)
    s = nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[pick].copy())
    ref = oracle.efv_system(m, s)
    res, *_ = run_gpu(m, s)
    _compare(s, ref, res, None, "small cells")


def test_near_lattice_forces():
    m = pmodel()
    pos, h = nep_synth.bcc_lattice(12, 12, 12)
    pos = pos + np.random.default_rng(13).normal(0.0, 0.004, pos.shape)
    s = nep_synth._single(pos, h)
    ref = oracle.efv_system(m, s)
    res, *_ = run_gpu(m, s)
    _compare(s, ref, res, None, "near lattice")


def test_md_steps_then_sampled():
    # 128,000 atoms at 300 K, 20 steps of 1 fs, sampled atoms against FP64
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    s = nep_synth.mid()
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_step_verlet(sysd, 20, out, dt_max=1.0)
    torch.cuda.synchronize()
    pos = sysd.positions().cpu().numpy()
    F = out.forces().cpu().numpy().astype(np.float64)
    idx = np.sort(np.random.default_rng(7).choice(s.n_atoms, 256, replace=False))
    ref = oracle.efv_cell(m, pos, s.h[0], targets=idx, virial=False)
    err = np.linalg.norm(F[idx] - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[paper model mid] sampled force rel err {err:.3e}", flush=True)
    assert err <= F_REL_TOL


def test_unsupported_calls_are_refused():
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    s = nep_synth.tiny(n_cells=4)
    res, ctx, sysd, out = run_gpu(m, s)
    assert ctx.nep_num_params() == 16 * 16 + 11 * 11 + 100 * 60 + 100 + 100 + 1
    with pytest.raises(nep.NepError) as e:
        ctx.nep_set_precision(1)
    assert e.value.code == nep.NEP_E_UNSUPPORTED
    with pytest.raises(nep.NepError) as e:
        ctx.nep_backward(sysd, out, torch.ones(1, dtype=torch.float64, device="cuda"))
    assert e.value.code == nep.NEP_E_UNSUPPORTED


def test_md_candidate_walk_matches_full_walk():
    # the radial walk over the last full walk's candidates (as in the default
    # model): the last MD evaluation equals a fresh full evaluation bit for bit
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    s = nep_synth.mid(n_cells=24)
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_step_verlet(sysd, 30, out, dt_max=1.0, max_disp=0.0)
    torch.cuda.synchronize()
    F_md = out.forces().cpu().numpy().copy()
    E_md = out.energy.cpu().numpy().copy()
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    assert np.array_equal(F_md, out.forces().cpu().numpy())
    assert np.array_equal(E_md, out.energy.cpu().numpy())
