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


def test_autotune_keeps_results():
    # the phase kernels in 64/128/256-thread blocks: whichever shapes the
    # autotuner keeps, every atom's arithmetic is the same, so the results
    # are bitwise those of the default shapes
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    full = nep_synth.batch()
    sizes = np.diff(full.cell_start)
    pick = list(range(0, 4096, 97))
    pos = np.concatenate([full.cell(c)[0] for c in pick])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in pick])]).astype(np.int64)
    s = nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[pick].copy())
    res, ctx, sysd, out = run_gpu(m, s)
    assert ctx.nep_num_params() == 16 * 16 + 11 * 11 + 100 * 60 + 100 + 100 + 1
    shapes = ctx.nep_autotune(sysd, out, reps=2)
    print(f"[paper model] autotuned shapes {shapes}", flush=True)
    assert all(sh in ctx.SHAPE_NAMES[:3] for sh in shapes)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.forces().cpu().numpy().astype(np.float64), res["forces"])
    assert np.array_equal(out.energy.cpu().numpy(), res["energy"])
    assert np.array_equal(out.virial.cpu().numpy().reshape(-1, 3, 3), res["virial"])


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


# parameter gradients: FP32 products summed per 64-atom tile, FP64 across
# tiles (the default model's bar)
P_REL_TOL = 1e-5
P_SIZES = (256, 121, 6000, 100, 100, 1)
P_NAMES = ("c_rad", "c_ang", "w0", "b0", "w1", "b1")


def _subset(full, picks):
    sizes = np.diff(full.cell_start)
    pos = np.concatenate([full.cell(c)[0] for c in picks])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in picks])]).astype(np.int64)
    return nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[list(picks)].copy())


def test_backward_matches_oracle_gradients():
    # dE/dtheta, dE/dpos through the differentiable energy on strained cells
    # with images (several tiles, a ragged tail), against the FP64 oracle
    import torch
    import paper_2305_08140_amd as nep
    from paper_2305_08140_amd.autograd import nep_energy
    m = pmodel()
    full = nep_synth.diffbatch()
    s = _subset(full, range(0, 512, 32))
    ctx = nep.Context(m, s.n_atoms, s.n_cells)
    pos = torch.tensor(s.pos, device="cuda", requires_grad=True)
    cell = torch.tensor(s.h, device="cuda", requires_grad=True)
    theta = torch.tensor(m.param_vector(), device="cuda", dtype=torch.float32, requires_grad=True)
    q_scale = torch.tensor(m.q_scale, device="cuda", dtype=torch.float32)
    E = nep_energy(ctx, pos, cell, theta, q_scale, cell_start=s.cell_start)
    gE = torch.tensor(np.random.default_rng(3).normal(size=s.n_cells), device="cuda")
    (E * gE).sum().backward()
    g_np = gE.cpu().numpy()
    ref_gp = np.zeros(theta.numel())
    ref_gx = np.zeros((s.n_atoms, 3))
    for c in range(s.n_cells):
        a, b = int(s.cell_start[c]), int(s.cell_start[c + 1])
        ref_gx[a:b] = -g_np[c] * oracle.efv_cell(m, s.pos[a:b], s.h[c], virial=False)["forces"]
        ref_gp += g_np[c] * oracle.param_grad_cell(m, s.pos[a:b], s.h[c])
    gx = pos.grad.cpu().numpy()
    assert np.linalg.norm(gx - ref_gx) / np.linalg.norm(ref_gx) <= F_REL_TOL
    gp = theta.grad.double().cpu().numpy()
    o = np.concatenate([[0], np.cumsum(P_SIZES)])
    for name, a, b in zip(P_NAMES, o[:-1], o[1:]):
        err = np.linalg.norm(gp[a:b] - ref_gp[a:b]) / np.linalg.norm(ref_gp[a:b])
        print(f"[paper model param grad] {name}: rel err {err:.2e}", flush=True)
        assert err <= P_REL_TOL, name


def test_parameter_gradient_over_many_tiles():
    # more 64-atom tiles than blocks: two calls agree bit for bit, and the
    # whole batch's gradient is the sum of its halves' to FP32 rounding
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    full = nep_synth.diffbatch()
    assert (full.n_atoms + 63) // 64 > 1024
    g_all = np.random.default_rng(21).uniform(0.5, 1.5, size=full.n_cells)

    def grad(s, g):
        sysd = nep.DeviceSystem.from_synth(s)
        ctx = nep.Context(m, s.n_atoms, s.n_cells)
        o = nep.EFV(s.n_atoms, s.n_cells)
        ctx.nep_build_neighbors(sysd)
        ctx.nep_compute_efv(sysd, o)
        gE = torch.tensor(g, device="cuda", dtype=torch.float64)
        a = ctx.nep_backward(sysd, o, gE, grad_pos=False, grad_cell=False)[0].clone()
        b = ctx.nep_backward(sysd, o, gE, grad_pos=False, grad_cell=False)[0]
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        return a.cpu().numpy()

    gp = grad(full, g_all)
    parts = grad(_subset(full, range(0, 256)), g_all[:256]) + grad(_subset(full, range(256, 512)), g_all[256:])
    o = np.concatenate([[0], np.cumsum(P_SIZES)])
    for name, a, b in zip(P_NAMES, o[:-1], o[1:]):
        err = np.linalg.norm(gp[a:b] - parts[a:b]) / np.linalg.norm(parts[a:b])
        print(f"[paper model param grad, 1111 tiles] {name}: whole vs halves rel diff {err:.2e}", flush=True)
        assert err <= 1e-6, name


def test_matrix_core_network_matches_oracle_and_vector_path():
    # precision mode 2: the 60 -> 100 -> 1 network on the matrix cores (FP32
    # operands and accumulation) against the FP64 oracle at the same bars,
    # and against the vector-ALU network to FP32 summation-order rounding;
    # strained cells with images and a ragged last tile (several tiles, so
    # the persistent grid strides)
    import torch
    m = pmodel()
    full = nep_synth.batch()
    sizes = np.diff(full.cell_start)
    pick = [int(c) for c in np.argsort(sizes)[:24]] + list(range(100, 4096, 400))
    pos = np.concatenate([full.cell(c)[0] for c in pick])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in pick])]).astype(np.int64)
    s = nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[pick].copy())
    assert s.n_atoms % 64 != 0
    ref = oracle.efv_system(m, s)
    res0, ctx, sysd, out = run_gpu(m, s)
    ctx.nep_set_precision(2)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    res2 = {"energy": out.energy.cpu().numpy(), "forces": out.forces().cpu().numpy().astype(np.float64),
            "virial": out.virial.cpu().numpy().reshape(-1, 3, 3), "energy_atom": out.energy_atom.cpu().numpy()}
    _compare(s, ref, res2, None, "matrix-core network")
    d = np.linalg.norm(res2["forces"] - res0["forces"]) / np.linalg.norm(res0["forces"])
    du = np.abs(res2["energy_atom"] - res0["energy_atom"]).max()
    print(f"[paper model] matrix-core vs vector network: force rel diff {d:.2e}, site energy {du:.2e} eV", flush=True)
    assert d <= 1e-6 and du <= 1e-5
    # mode 1 (BF16 operands): the scaled descriptors and dU/dz rounded to 8
    # significant bits (2^-9 relative), ~2^-9 sqrt(60) ~ 1.5e-2 relative in
    # the forces; bound 4e-2, and visibly worse than FP32 (the BF16 products ran)
    ctx.nep_set_precision(1)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    Fb = out.forces().cpu().numpy().astype(np.float64)
    eb = np.linalg.norm(Fb - ref["forces"]) / np.linalg.norm(ref["forces"])
    e2 = np.linalg.norm(res2["forces"] - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[paper model] BF16 matrix-core network: force rel err {eb:.2e} (FP32 {e2:.2e})", flush=True)
    assert e2 < eb <= 4e-2


def test_matrix_core_network_md_sampled():
    # 128,000 atoms, 20 MD steps with the matrix-core network, sampled atoms
    # against FP64
    import torch
    import paper_2305_08140_amd as nep
    m = pmodel()
    s = nep_synth.mid()
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, 1)
    ctx.nep_set_precision(2)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_step_verlet(sysd, 20, out, dt_max=1.0)
    torch.cuda.synchronize()
    pos = sysd.positions().cpu().numpy()
    F = out.forces().cpu().numpy().astype(np.float64)
    idx = np.sort(np.random.default_rng(8).choice(s.n_atoms, 256, replace=False))
    ref = oracle.efv_cell(m, pos, s.h[0], targets=idx, virial=False)
    err = np.linalg.norm(F[idx] - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[paper model mid, matrix-core network] sampled force rel err {err:.3e}", flush=True)
    assert err <= F_REL_TOL
