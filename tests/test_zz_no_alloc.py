"""The allocation-free backward (nep_backward_noalloc, block partials in the
library's file-scope device array) against nep_backward through the C ABI:
two calls in a row, the second on a smaller system, each compared with
nep_backward on the same forward (same kernels and launch width, so the
results must agree bit for bit, which is stricter than the FP32 bar)."""
import numpy as np
import pytest

import nep_synth
from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _subset(full, picks):
    sizes = np.diff(full.cell_start)
    pos = np.concatenate([full.cell(c)[0] for c in picks])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in picks])]).astype(np.int64)
    return nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[list(picks)].copy())


def _compare(ctx, s, seed):
    import torch
    import paper_2305_08140_amd as nep
    sysd = nep.DeviceSystem.from_synth(s)
    out = nep.EFV(s.n_atoms, s.n_cells)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    gE = torch.tensor(np.random.default_rng(seed).normal(size=s.n_cells), device="cuda")
    dev = out.fx.device
    pre = {"params": torch.full((ctx.nep_num_params(),), np.nan, dtype=torch.float64, device=dev),
           "x": torch.full((s.n_atoms,), np.nan, dtype=torch.float64, device=dev),
           "y": torch.full((s.n_atoms,), np.nan, dtype=torch.float64, device=dev),
           "z": torch.full((s.n_atoms,), np.nan, dtype=torch.float64, device=dev),
           "h": torch.full((s.n_cells, 9), np.nan, dtype=torch.float64, device=dev)}
    print(f"[no-alloc] {s.n_cells} cells, {s.n_atoms} atoms, {(s.n_atoms + 63) // 64} tiles", flush=True)
    gp_s, gx_s, gh_s = ctx.nep_backward_noalloc(sysd, out, gE, outputs=pre)
    gp, gx, gh = ctx.nep_backward(sysd, out, gE)
    torch.cuda.synchronize()
    assert gp_s.data_ptr() == pre["params"].data_ptr()
    for a, b in ((gp_s, gp), (gx_s, gx), (gh_s, gh)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.isfinite(a))
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert rel <= 1e-12, rel
        assert np.array_equal(a, b)
    return gp_s.cpu().numpy()


def test_noalloc_backward_matches_backward_twice_then_smaller():
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    full = nep_synth.diffbatch()
    ctx = nep.Context(m, full.n_atoms, full.n_cells)
    # 1111 tiles: all 1024 rows of the device array in use
    big = _compare(ctx, full, 1)
    # smaller: 16 cells, a few tiles; rows beyond them still hold the first call's partials
    small_sys = _subset(full, range(0, 512, 32))
    small = _compare(ctx, small_sys, 2)
    assert not np.array_equal(big, small)
    # a second context on the same GPU shares the array
    ctx2 = nep.Context(m, small_sys.n_atoms, small_sys.n_cells)
    again = _compare(ctx2, small_sys, 2)
    assert np.array_equal(again, small)


def test_noalloc_backward_argument_checks():
    import torch
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model()
    s = nep_synth.tiny()
    ctx = nep.Context(m, s.n_atoms, 1)
    sysd = nep.DeviceSystem.from_synth(s)
    out = nep.EFV(s.n_atoms, 1)
    gE = torch.ones(1, dtype=torch.float64, device="cuda")
    # before any build: the call-order error, as nep_backward
    with pytest.raises(nep.NepError) as e:
        ctx.nep_backward_noalloc(sysd, out, gE)
    assert e.value.code == nep.NEP_E_STATE
    with pytest.raises(nep.NepError) as e2:
        ctx.nep_backward(sysd, out, gE)
    assert e2.value.code == nep.NEP_E_STATE
    # the paper-size model's backward: checked before any build as well
    mw = nep_synth.random_model(size="paper")
    ctxw = nep.Context(mw, s.n_atoms, 1)
    with pytest.raises(nep.NepError) as e3:
        ctxw.nep_backward_noalloc(sysd, out, gE)
    assert e3.value.code == nep.NEP_E_STATE


def test_noalloc_backward_paper_model_twice_then_smaller():
    # the paper-size model (6,578 parameters per partial row): all 1024 rows
    # of the device array in use, then a smaller system on the same context
    import paper_2305_08140_amd as nep
    m = nep_synth.random_model(size="paper")
    full = nep_synth.diffbatch()
    ctx = nep.Context(m, full.n_atoms, full.n_cells)
    big = _compare(ctx, full, 3)
    small = _compare(ctx, _subset(full, range(5, 512, 40)), 4)
    assert big.shape == small.shape == (6578,)
    assert not np.array_equal(big, small)
