"""Batched small cells: graph replay, autotuned launch shapes, BF16 hidden layer."""
import numpy as np
import pytest

import nep_synth
import oracle
from gpu_common import E_ATOM_TOL, F_REL_TOL, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _subset(full, picks):
    sizes = np.diff(full.cell_start)
    pos = np.concatenate([full.cell(c)[0] for c in picks])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in picks])]).astype(np.int64)
    return nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[list(picks)].copy())


def _setup(s, m):
    import paper_2305_08140_amd as nep
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(m, s.n_atoms, s.n_cells)
    out = nep.EFV(s.n_atoms, s.n_cells)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    return sysd, ctx, out


def _snap(out):
    return (out.energy.cpu().numpy().copy(), out.forces().cpu().numpy().copy(), out.virial.cpu().numpy().copy())


def test_batch_matches_oracle():
    m = nep_synth.random_model()
    full = nep_synth.batch()
    s = _subset(full, range(0, 4096, 64))
    sysd, ctx, out = _setup(s, m)
    E, F, W = _snap(out)
    ref = oracle.efv_system(m, s)
    counts = np.diff(s.cell_start)
    assert np.all(np.abs(E - ref["energy"]) / counts <= E_ATOM_TOL)
    err = np.linalg.norm(F - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[batch] force rel err {err:.2e}", flush=True)
    assert err <= F_REL_TOL


def test_graph_replay_equals_eager():
    import torch
    m = nep_synth.random_model()
    full = nep_synth.batch()
    s = _subset(full, range(0, 4096, 16))
    sysd, ctx, out = _setup(s, m)
    torch.cuda.synchronize()
    ref = _snap(out)
    st = torch.cuda.Stream()
    for rep in range(4):
        with torch.cuda.stream(st):
            out.fx.zero_()
            out.energy.zero_()
            ctx.nep_compute_efv_graph(sysd, out, stream=st)
        st.synchronize()
        got = _snap(out)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
        # eager work of the program between replays
        ctx.nep_compute_efv(sysd, out)
        torch.cuda.synchronize()
        assert np.array_equal(_snap(out)[1], ref[1])


def test_autotuned_shapes_give_identical_results():
    import torch
    m = nep_synth.random_model()
    full = nep_synth.batch()
    s = _subset(full, range(0, 4096, 8))
    sysd, ctx, out = _setup(s, m)
    torch.cuda.synchronize()
    ref = _snap(out)
    shapes = ctx.nep_autotune(sysd, out, reps=2)
    print("[autotune]", shapes, flush=True)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    for a, b in zip(_snap(out), ref):
        assert np.array_equal(a, b)


def test_bf16_hidden_layer_error_vs_fp64():
    # BF16 rounds the scaled descriptors and dU/dz to 8 significant bits
    # (relative 2^-9); that error enters the network output and dU/dq linearly,
    # ~2^-9 sqrt(29) ~ 1e-2 relative in the forces.  Bound: 3e-2.
    import torch
    m = nep_synth.random_model()
    full = nep_synth.batch()
    s = _subset(full, range(3, 4096, 64))
    sysd, ctx, out = _setup(s, m)
    torch.cuda.synchronize()
    F32 = out.forces().cpu().numpy().astype(np.float64)
    ctx.nep_set_precision(1)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    Fb = out.forces().cpu().numpy().astype(np.float64)
    Eb = out.energy.cpu().numpy()
    ref = oracle.efv_system(m, s)
    e32 = np.linalg.norm(F32 - ref["forces"]) / np.linalg.norm(ref["forces"])
    eb = np.linalg.norm(Fb - ref["forces"]) / np.linalg.norm(ref["forces"])
    de = np.max(np.abs(Eb - ref["energy"]) / np.diff(s.cell_start))
    print(f"[precision] force rel err FP32 {e32:.2e}  BF16-MFMA {eb:.2e}; BF16 energy err {de:.2e} eV/atom",
          flush=True)
    assert e32 <= F_REL_TOL
    assert eb <= 3e-2
    assert eb > e32        # the reduced precision is visible, i.e. the MFMA path really ran
    ctx.nep_set_precision(0)


def test_fp32_matrix_core_hidden_layer_matches_oracle():
    # mode 2 keeps FP32 operands (exact products, FP32 sums in another
    # order), so it meets the same bars as the vector-ALU path
    import torch
    m = nep_synth.random_model()
    full = nep_synth.batch()
    s = _subset(full, range(5, 4096, 64))
    sysd, ctx, out = _setup(s, m)
    ctx.nep_set_precision(2)
    ctx.nep_compute_efv(sysd, out)
    torch.cuda.synchronize()
    E, F, W = _snap(out)
    ctx.nep_set_precision(0)
    ref = oracle.efv_system(m, s)
    counts = np.diff(s.cell_start)
    assert np.all(np.abs(E - ref["energy"]) / counts <= E_ATOM_TOL)
    err = np.linalg.norm(F - ref["forces"]) / np.linalg.norm(ref["forces"])
    print(f"[precision] force rel err FP32-MFMA {err:.2e}", flush=True)
    assert err <= F_REL_TOL
