"""SNES population evaluation on the GPU (Sec. III.A: population 50, loss
weights of the paper) against the single-model path and the FP64 oracle."""
import numpy as np
import pytest

import nep_synth
from oracle import snes as S
from gpu_common import E_ATOM_TOL, F_REL_TOL, W_ATOM_TOL, W_REL_TOL, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _population(model, n_pop, spread, seed):
    rng = np.random.default_rng(seed)
    th0 = model.param_vector()
    th = th0[None, :] + spread * rng.standard_normal((n_pop, th0.size)) * np.maximum(np.abs(th0), 0.1)[None, :]
    th[0] = th0
    return th.astype(np.float32)


def _targets_device(tg, torch):
    dev = "cuda"
    return {"energy": torch.tensor(tg["energy"], dtype=torch.float64, device=dev),
            "forces": torch.tensor(np.ascontiguousarray(tg["forces"].T), dtype=torch.float32, device=dev),
            "virial": torch.tensor(tg["virial"].reshape(-1, 9), dtype=torch.float64, device=dev),
            "has_virial": torch.tensor(tg["has_virial"].astype(np.uint8), device=dev)}


def _setup(s, model, n_pop):
    import paper_2305_08140_amd as nep
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(model, s.n_atoms, s.n_cells)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_population_reserve(n_pop)
    return sysd, ctx


def test_members_equal_the_single_model_path():
    # 40 cells of 16-256 atoms; 7 members (tiles x members not a multiple of
    # 8): every member's energies, forces and virials are those of
    # nep_compute_efv with that member's parameters, bit for bit
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    s = nep_synth.diffbatch(n_cells=40)
    th = _population(m, 7, 0.05, 1)
    sysd, ctx = _setup(s, m, 7)
    res = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"))
    torch.cuda.synchronize()
    single = nep.Context(m, s.n_atoms, s.n_cells)
    out = nep.EFV(s.n_atoms, s.n_cells)
    single.nep_build_neighbors(sysd)
    for k in range(th.shape[0]):
        single.nep_set_weights(m.with_param_vector(th[k].astype(np.float64)))
        single.nep_compute_efv(sysd, out)
        torch.cuda.synchronize()
        assert torch.equal(res["energy"][k], out.energy), k
        assert torch.equal(res["virial"][k], out.virial.reshape(-1, 9)), k
        assert torch.equal(res["forces"][k, 0], out.fx) and torch.equal(res["forces"][k, 1], out.fy), k
        assert torch.equal(res["forces"][k, 2], out.fz), k


def test_population_and_loss_against_the_oracle():
    # 12 cells; targets from another random model (the oracle); 5 members;
    # half of the cells carry a virial target
    import torch
    m = nep_synth.random_model()
    teacher = nep_synth.random_model(seed=77)
    s = nep_synth.diffbatch(n_cells=12)
    E_t, F_t, W_t = S.evaluate_cells(teacher, s)
    tg = {"energy": E_t, "forces": F_t, "virial": W_t, "has_virial": np.arange(s.n_cells) % 2 == 0}
    th = _population(m, 5, 0.05, 2)
    sysd, ctx = _setup(s, m, 5)
    res = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"), _targets_device(tg, torch))
    torch.cuda.synchronize()
    na = np.diff(s.cell_start).astype(np.float64)
    loss_gpu = res["loss"].cpu().numpy()
    for k in range(th.shape[0]):
        E, F, W = S.evaluate_cells(m, s, th[k].astype(np.float64))
        Eg = res["energy"][k].cpu().numpy()
        Fg = res["forces"][k].cpu().numpy().T.astype(np.float64)
        Wg = res["virial"][k].cpu().numpy().reshape(-1, 3, 3)
        assert np.max(np.abs(Eg - E) / na) <= E_ATOM_TOL
        assert np.linalg.norm(Fg - F) <= F_REL_TOL * np.linalg.norm(F)
        for c in range(s.n_cells):
            assert np.linalg.norm(Wg[c] - W[c]) <= W_REL_TOL * np.linalg.norm(W[c]) + W_ATOM_TOL * na[c]
        ref = S.loss_terms(th[k].astype(np.float64), E, F, W, tg, na)
        lg = loss_gpu[k]
        print(f"[member {k}] loss gpu {lg[0]:.9f} oracle {ref[0]:.9f}", flush=True)
        # bounds from the evaluation tolerances: an energy error <= 1e-6 eV/atom
        # moves the energy RMSE by at most that; a force error of relative norm
        # <= 1e-5 moves the force RMSE by at most 1e-5 rms(F); the virial
        # likewise per atom
        assert abs(lg[1] - ref[1]) <= E_ATOM_TOL
        assert abs(lg[2] - ref[2]) <= F_REL_TOL * np.sqrt(np.mean(F ** 2))
        assert abs(lg[3] - ref[3]) <= W_REL_TOL * np.sqrt(np.mean((W / na[:, None, None]) ** 2)) + W_ATOM_TOL
        assert abs(lg[4] - ref[4]) <= 1e-12 * ref[4] and abs(lg[5] - ref[5]) <= 1e-12 * ref[5]
        w = S.LAMBDAS
        bound = (w["e"] * E_ATOM_TOL + w["f"] * F_REL_TOL * np.sqrt(np.mean(F ** 2))
                 + w["v"] * (W_REL_TOL * np.sqrt(np.mean((W / na[:, None, None]) ** 2)) + W_ATOM_TOL) + 1e-12)
        assert abs(lg[0] - ref[0]) <= bound
    # member 0 is the model itself; a member equal to the teacher has no error
    th_t = teacher.param_vector().astype(np.float32)[None, :]
    res_t = ctx.nep_population_efv(sysd, torch.tensor(th_t, device="cuda"), _targets_device(tg, torch))
    lt = res_t["loss"].cpu().numpy()[0]
    assert lt[1] < 1e-5 and lt[2] < 1e-4 * np.sqrt(np.mean(F_t ** 2)) and lt[3] < 1e-5


def test_loss_without_virial_targets():
    import torch
    m = nep_synth.random_model()
    s = nep_synth.diffbatch(n_cells=6)
    E_t, F_t, W_t = S.evaluate_cells(nep_synth.random_model(seed=77), s)
    tg = {"energy": E_t, "forces": F_t, "virial": W_t, "has_virial": np.zeros(s.n_cells, bool)}
    th = _population(m, 3, 0.05, 3)
    sysd, ctx = _setup(s, m, 3)
    td = _targets_device(tg, torch)
    a = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"), dict(td, virial=None, has_virial=None))
    b = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"), td)
    torch.cuda.synchronize()
    assert torch.all(a["loss"][:, 3] == 0) and torch.all(b["loss"][:, 3] == 0)
    assert torch.equal(a["loss"], b["loss"])


def test_snes_sample_and_update_against_the_oracle():
    import torch
    import paper_2305_08140_amd as nep
    rng = np.random.default_rng(5)
    P_, n = 50, 1057
    mu = rng.normal(size=n).astype(np.float32)
    sigma = rng.uniform(0.05, 0.2, size=n).astype(np.float32)
    s = rng.standard_normal((P_, n)).astype(np.float32)
    loss = rng.uniform(1.0, 2.0, size=P_)
    loss[7] = loss[3]          # a tie: member order decides
    loss[11] = np.nan          # worst
    mu_d, sg_d, s_d = (torch.tensor(a, device="cuda") for a in (mu, sigma, s))
    th = nep.snes_sample(mu_d, sg_d, s_d)
    th_ref = S.sample(mu, sigma, s)
    assert np.max(np.abs(th.cpu().numpy() - th_ref) / np.maximum(np.abs(th_ref), 1e-30)) <= 2 ** -23
    loss_d = torch.tensor(np.stack([loss, np.zeros(P_)], axis=1), device="cuda")   # stride 2
    nep.snes_update(mu_d, sg_d, s_d, loss_d)
    torch.cuda.synchronize()
    mu_ref, sg_ref = S.update(mu, sigma, s, loss)
    assert np.max(np.abs(mu_d.cpu().numpy() - mu_ref) / np.maximum(np.abs(mu_ref), 1e-3)) <= 2e-6
    assert np.max(np.abs(sg_d.cpu().numpy() - sg_ref) / sg_ref) <= 2e-6
    with pytest.raises(nep.NepError):
        nep.snes_update(mu_d, sg_d, s_d[:1], loss_d[:1])


def test_snes_training_lowers_the_loss():
    # 60 generations of 24 members on 16 cells against a teacher's targets,
    # all on the device; the loss of the mean falls
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    s = nep_synth.diffbatch(n_cells=16)
    E_t, F_t, W_t = S.evaluate_cells(nep_synth.random_model(seed=77), s)
    tg = {"energy": E_t, "forces": F_t, "virial": W_t, "has_virial": np.ones(s.n_cells, bool)}
    P_ = 24
    sysd, ctx = _setup(s, m, P_)
    td = _targets_device(tg, torch)
    mu = torch.tensor(m.param_vector().astype(np.float32), device="cuda")
    sigma = torch.full_like(mu, 0.1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)

    def mean_loss():
        return float(ctx.nep_population_efv(sysd, mu[None, :].clone(), td, want_energy=False, want_forces=False,
                                            want_virial=False)["loss"][0, 0])
    l0 = mean_loss()
    for _ in range(60):
        draws = torch.randn(P_, mu.numel(), device="cuda", generator=gen)
        nep.snes_generation(ctx, sysd, mu, sigma, draws, td)
    l1 = mean_loss()
    print(f"[snes] loss of the mean {l0:.4f} -> {l1:.4f}", flush=True)
    assert l1 < 0.8 * l0


def test_population_limits():
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    s = nep_synth.diffbatch(n_cells=4)
    sysd, ctx = _setup(s, m, 2)
    th = _population(m, 3, 0.05, 4)
    with pytest.raises(nep.NepError) as e:
        ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"))
    assert e.value.code == nep.NEP_E_ARG
    one = ctx.nep_population_efv(sysd, torch.tensor(th[:1], device="cuda"))
    assert one["energy"].shape == (1, s.n_cells)
    # the paper-size model's members: the same limits
    sysw, wide = _setup(s, nep_synth.random_model(size="paper"), 2)
    thw = _population(nep_synth.random_model(size="paper"), 3, 0.05, 4)
    with pytest.raises(nep.NepError) as e:
        wide.nep_population_efv(sysw, torch.tensor(thw, device="cuda"))
    assert e.value.code == nep.NEP_E_ARG
    assert wide.nep_population_efv(sysw, torch.tensor(thw[:2], device="cuda"))["energy"].shape == (2, s.n_cells)


def test_paper_size_members_equal_the_single_model_path():
    # the paper-size model (Sec. III.A: the model the paper trains with SNES)
    # evaluates its members one after another through its staged phases:
    # each member's results are bitwise those of nep_compute_efv with that
    # member's parameters
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model(size="paper")
    s = nep_synth.diffbatch(n_cells=24)
    th = _population(m, 4, 0.05, 11)
    sysd, ctx = _setup(s, m, 4)
    res = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"))
    torch.cuda.synchronize()
    single = nep.Context(m, s.n_atoms, s.n_cells)
    out = nep.EFV(s.n_atoms, s.n_cells)
    single.nep_build_neighbors(sysd)
    for k in range(th.shape[0]):
        single.nep_set_weights(m.with_param_vector(th[k].astype(np.float64)))
        single.nep_compute_efv(sysd, out)
        torch.cuda.synchronize()
        assert torch.equal(res["energy"][k], out.energy), k
        assert torch.equal(res["virial"][k], out.virial.reshape(-1, 9)), k
        assert torch.equal(res["forces"][k, 0], out.fx) and torch.equal(res["forces"][k, 1], out.fy), k
        assert torch.equal(res["forces"][k, 2], out.fz), k
    # the context's own weights are untouched by the population call
    ctx_out = nep.EFV(s.n_atoms, s.n_cells)
    ctx.nep_compute_efv(sysd, ctx_out)
    single.nep_set_weights(m)
    single.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    assert torch.equal(ctx_out.energy, out.energy)


def test_paper_size_population_loss_against_the_oracle():
    import torch
    m = nep_synth.random_model(size="paper")
    teacher = nep_synth.random_model(size="paper", seed=78)
    s = nep_synth.diffbatch(n_cells=6)
    E_t, F_t, W_t = S.evaluate_cells(teacher, s)
    tg = {"energy": E_t, "forces": F_t, "virial": W_t, "has_virial": np.arange(s.n_cells) % 2 == 0}
    th = _population(m, 3, 0.05, 12)
    sysd, ctx = _setup(s, m, 3)
    res = ctx.nep_population_efv(sysd, torch.tensor(th, device="cuda"), _targets_device(tg, torch))
    torch.cuda.synchronize()
    na = np.diff(s.cell_start).astype(np.float64)
    loss_gpu = res["loss"].cpu().numpy()
    for k in range(th.shape[0]):
        E, F, W = S.evaluate_cells(m, s, th[k].astype(np.float64))
        ref = S.loss_terms(th[k].astype(np.float64), E, F, W, tg, na)
        lg = loss_gpu[k]
        print(f"[paper-size member {k}] loss gpu {lg[0]:.9f} oracle {ref[0]:.9f}", flush=True)
        assert abs(lg[1] - ref[1]) <= E_ATOM_TOL
        assert abs(lg[2] - ref[2]) <= F_REL_TOL * np.sqrt(np.mean(F ** 2))
        assert abs(lg[3] - ref[3]) <= W_REL_TOL * np.sqrt(np.mean((W / na[:, None, None]) ** 2)) + W_ATOM_TOL
        assert abs(lg[4] - ref[4]) <= 1e-12 * ref[4] and abs(lg[5] - ref[5]) <= 1e-12 * ref[5]
