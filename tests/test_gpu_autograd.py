"""Differentiable energy: the library's backward against the FP64 oracle's
analytic gradients (parameters, forces) and finite differences (cell)."""
import numpy as np
import pytest

import nep_synth
import oracle
from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# Parameter gradients are sums over atoms of FP32 products (relative rounding
# ~1e-7 per term, FP64 sums across blocks); the network-weight components of
# a small batch reach ~1e-6 relative, so the bar is 1e-5 per parameter group.
P_REL_TOL = 1e-5


def _subset(full, picks):
    sizes = np.diff(full.cell_start)
    pos = np.concatenate([full.cell(c)[0] for c in picks])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in picks])]).astype(np.int64)
    return nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[list(picks)].copy())


def _energy_fn(m, s):
    import torch
    import paper_2305_08140_amd as nep
    from paper_2305_08140_amd.autograd import nep_energy
    ctx = nep.Context(m, s.n_atoms, s.n_cells)
    pos = torch.tensor(s.pos, device="cuda", requires_grad=True)
    cell = torch.tensor(s.h, device="cuda", requires_grad=True)
    theta = torch.tensor(m.param_vector(), device="cuda", dtype=torch.float32, requires_grad=True)
    q_scale = torch.tensor(m.q_scale, device="cuda", dtype=torch.float32)
    E = nep_energy(ctx, pos, cell, theta, q_scale, cell_start=s.cell_start)
    return E, pos, cell, theta, ctx


def test_backward_matches_oracle_gradients():
    import torch
    m = nep_synth.random_model()
    full = nep_synth.diffbatch()
    s = _subset(full, range(0, 512, 32))
    E, pos, cell, theta, _ = _energy_fn(m, s)
    rng = np.random.default_rng(3)
    gE = torch.tensor(rng.normal(size=s.n_cells), device="cuda")
    (E * gE).sum().backward()
    g_np = gE.cpu().numpy()
    ref_E = np.zeros(s.n_cells)
    ref_gp = np.zeros(theta.numel())
    ref_gx = np.zeros((s.n_atoms, 3))
    for c in range(s.n_cells):
        a, b = int(s.cell_start[c]), int(s.cell_start[c + 1])
        r = oracle.efv_cell(m, s.pos[a:b], s.h[c])
        ref_E[c] = r["energy"]
        ref_gx[a:b] = -g_np[c] * r["forces"]
        ref_gp += g_np[c] * oracle.param_grad_cell(m, s.pos[a:b], s.h[c])
    counts = np.diff(s.cell_start)
    assert np.all(np.abs(E.detach().cpu().numpy() - ref_E) / counts <= 1e-6)
    gx = pos.grad.cpu().numpy()
    assert np.linalg.norm(gx - ref_gx) / np.linalg.norm(ref_gx) <= 1e-5
    gp = theta.grad.double().cpu().numpy()
    groups = {"c_rad": (0, 81), "c_ang": (81, 126), "w0": (126, 996), "b0": (996, 1026), "w1": (1026, 1056),
              "b1": (1056, 1057)}
    for name, (a, b) in groups.items():
        err = np.linalg.norm(gp[a:b] - ref_gp[a:b]) / np.linalg.norm(ref_gp[a:b])
        print(f"[param grad] {name}: rel err {err:.2e}", flush=True)
        assert err <= P_REL_TOL, name


def test_cell_gradient_matches_finite_differences():
    import torch
    m = nep_synth.random_model()
    full = nep_synth.diffbatch()
    s = _subset(full, [5, 40])
    E, pos, cell, theta, _ = _energy_fn(m, s)
    E.sum().backward()
    gh = cell.grad.cpu().numpy()
    for c in range(s.n_cells):
        a, b = int(s.cell_start[c]), int(s.cell_start[c + 1])
        p = s.pos[a:b]
        fd = np.zeros((3, 3))
        h = 1e-5
        for i in range(3):
            for j in range(3):
                hp, hm = s.h[c].copy(), s.h[c].copy()
                hp[i, j] += h
                hm[i, j] -= h
                fd[i, j] = (oracle.efv_cell(m, p, hp, virial=False)["energy"] -
                            oracle.efv_cell(m, p, hm, virial=False)["energy"]) / (2 * h)
        err = np.linalg.norm(gh[c] - fd) / np.linalg.norm(fd)
        print(f"[cell grad] cell {c}: rel err {err:.2e}", flush=True)
        assert err <= 1e-4


def test_parameter_gradient_over_many_tiles():
    # the 512-cell batch has more 64-atom tiles than the 1024 blocks of the
    # parameter-gradient launch, so blocks add several tiles into their
    # partial rows: two calls agree bit for bit, and the gradient of the whole
    # batch is the sum of the gradients of its two halves (each under 1024
    # tiles) to FP32 rounding
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    full = nep_synth.diffbatch()
    assert (full.n_atoms + 63) // 64 > 1024
    rng = np.random.default_rng(21)
    g_all = rng.uniform(0.5, 1.5, size=full.n_cells)

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
    lo, hi = range(0, 256), range(256, 512)
    parts = grad(_subset(full, lo), g_all[:256]) + grad(_subset(full, hi), g_all[256:])
    groups = {"c_rad": (0, 81), "c_ang": (81, 126), "w0": (126, 996), "b0": (996, 1026), "w1": (1026, 1056),
              "b1": (1056, 1057)}
    for name, (a, b) in groups.items():
        err = np.linalg.norm(gp[a:b] - parts[a:b]) / np.linalg.norm(parts[a:b])
        print(f"[param grad, 1111 tiles] {name}: whole vs halves rel diff {err:.2e}", flush=True)
        assert err <= 1e-6, name


def test_two_forwards_on_one_context_keep_their_own_gradients():
    # E(theta1, x1) and E(theta2, x2) on one context, then one backward: each
    # forward's gradients must be those of a context that saw only it (the
    # parameter-gradient pass reads the weights and lists from the context,
    # so the second forward's state must not leak into the first's gradient)
    import torch
    import paper_2305_08140_amd as nep
    from paper_2305_08140_amd.autograd import nep_energy
    m = nep_synth.random_model()
    full = nep_synth.diffbatch()
    s = _subset(full, [3, 17, 60])
    rng = np.random.default_rng(5)
    theta1 = m.param_vector().astype(np.float32)
    theta2 = (theta1 * (1.0 + 0.05 * rng.standard_normal(theta1.size))).astype(np.float32)
    pos1 = s.pos
    pos2 = s.pos + rng.normal(scale=0.4, size=s.pos.shape)   # moved beyond skin / 2
    q_scale = torch.tensor(m.q_scale, device="cuda", dtype=torch.float32)
    cell0 = torch.tensor(s.h, device="cuda")
    gE1 = torch.tensor(rng.uniform(0.5, 1.5, size=s.n_cells), device="cuda")
    gE2 = torch.tensor(rng.uniform(0.5, 1.5, size=s.n_cells), device="cuda")

    def leaves(p, th):
        return (torch.tensor(p, device="cuda", requires_grad=True), cell0.clone().requires_grad_(True),
                torch.tensor(th, device="cuda", requires_grad=True))

    shared = nep.Context(m, s.n_atoms, s.n_cells)
    a = leaves(pos1, theta1)
    b = leaves(pos2, theta2)
    E1 = nep_energy(shared, *a, q_scale, cell_start=s.cell_start)
    E2 = nep_energy(shared, *b, q_scale, cell_start=s.cell_start)
    ((E1 * gE1).sum() + (E2 * gE2).sum()).backward()
    for (p, th, g), got in (((pos1, theta1, gE1), a), ((pos2, theta2, gE2), b)):
        own = nep.Context(m, s.n_atoms, s.n_cells)
        ref = leaves(p, th)
        E = nep_energy(own, *ref, q_scale, cell_start=s.cell_start)
        (E * g).sum().backward()
        for x, y, name in zip(got, ref, ("pos", "cell", "theta")):
            err = (torch.linalg.norm(x.grad - y.grad) / torch.linalg.norm(y.grad)).item()
            print(f"[two forwards] {name} grad rel diff {err:.2e}", flush=True)
            assert err <= 1e-12, name
