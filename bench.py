"""Benchmark: NEP-ZBL molecular dynamics of 8,192,000-atom bcc tungsten on one MI355X.

Workload (synthetic): 160x160x160 conventional bcc W cells (a = 3.165 A),
Maxwell-Boltzmann velocities at 300 K and one 1 keV primary knock-on atom
near the box centre moving along a seeded random direction; velocity-Verlet
with the adaptive step of the paper (fastest atom moves at most 0.015 A per
step, at most 1 fs); neighbour lists with a 1 A skin rebuilt on the device
when an atom moved more than 0.5 A.  A "step" is one full MD step: half
kick, drift, conditional rebuild, energy + forces + virial, half kick, step
length update.  Random NEP weights (the trained model is not available).

Prints one JSON line:  python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (256 CUs x 2.4 GHz x 256 flop/clk)
PEAK_HBM_GBS = 8000.0


def flops_per_atom(n_rad: float, n_ang: float, kr: int = 9, nr: int = 9, ka: int = 9, na: int = 5, nh: int = 30):
    """Algorithmic flops per atom of the evaluation, split into its descriptor
    side and its force kernel, counted on the minimal formulation: FMA = 2, any
    other arithmetic operation and each sqrt / reciprocal / cos / sin / tanh = 1.
    n_rad, n_ang: neighbours inside the radial (6 A) and angular (4 A) cutoffs;
    kr, ka: Chebyshev basis sizes; nr radial descriptors; na angular channels
    (l = 1..4, 24 harmonics); nh hidden neurons.  The defaults are the 8.2M-atom
    workload's model (9 + 5 x 4 descriptors, k = 0..8, 30 neurons); the
    paper-size model of Sec. III.A is kr = nr = 16, ka = na = 11, nh = 100.

    descriptor side: descriptor, network forward + backward, adjoints, and
      the gradient of U_i with respect to every angular pair vector;
    force kernel: radial + ZBL pair forces of both ends, the assembly of the
      angular pair gradients, and the virial."""
    dim = nr + 4 * na
    geom = 9                                                     # r_ij (3), r^2 (5), sqrt (1)
    rad_fwd = geom + 9 + 2 * (kr - 2) + 2 * kr                   # t, fc, x, T_2.., sum fc T_k
    ang_fwd = 9 + 2 * (ka - 2) + na * (2 * ka + 2) + 4 + 60 + 48 * na   # basis, g_n, u, Y_lm, s += g Y
    per_atom = (2 * nr * kr + 2 * nr) + 48 * na + (nh * (2 * dim + 5) + 10) + nh * (2 * dim + 3) \
        + 2 * nr * kr + 48 * na                                  # q_n, q_nl, network fwd (+ output), bwd, a_k, B
    ang_grad = geom + 1 + (14 + 6 * (ka - 2)) + na * (4 * ka + 6) + 60 + 96 * na + 48 + 150 + 20 + 3 + 18
    desc = rad_fwd * n_rad + ang_fwd * n_ang + per_atom + ang_grad * n_ang
    rad_pair = 54 + 6 * (kr - 2) + 6 * kr
    force = rad_pair * n_rad + 3 * n_ang + 20
    return desc, force


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("nep_kernels.hip", "nep_device.h", "nep_pairs.h"):
        with open(os.path.join(ROOT, "paper_2305_08140_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, n_launch_atoms: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration);
    None when the summary is missing or was taken on another kernel source."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("source_hash") != _kernel_source_hash() or d.get("n_atoms") != n_launch_atoms:
        return None
    return float(k["bytes_per_launch"])


def cpu_baseline(model, s, seconds_target=5.0):
    """FP64 oracle (untuned, all host threads) on a bounded sample of the same
    workload: energies and forces of a contiguous block of atoms.  The sample
    is sized for ~seconds_target per run; one warm-up run, then the median of
    three timed runs."""
    import oracle
    n_thr = oracle.num_threads()
    # probe with a small sample, then size the sample for ~seconds_target
    sample = 2000
    t0 = time.time()
    oracle.efv_cell(model, s.pos, s.h[0], targets=np.arange(sample), virial=False)
    per_atom = (time.time() - t0) / sample
    # the probe includes the fixed cost of binning all atoms, so resize once
    # more from the first sized run (which is also the warm-up)
    for _ in range(2):
        sample = int(min(s.n_atoms, 2_000_000, max(2000, seconds_target / max(per_atom, 1e-9))))
        t0 = time.time()
        oracle.efv_cell(model, s.pos, s.h[0], targets=np.arange(sample), virial=False)
        dt = time.time() - t0
        per_atom = dt / sample
        if dt > 0.5 * seconds_target or sample >= min(s.n_atoms, 2_000_000):
            break
    runs = []
    for _ in range(3):
        t0 = time.time()
        oracle.efv_cell(model, s.pos, s.h[0], targets=np.arange(sample), virial=False)
        runs.append(time.time() - t0)
    dt = float(np.median(runs))
    return {"value": sample / dt, "unit": "atom-steps/s", "cores": n_thr, "kind": "oracle",
            "sample": f"FP64 energies+forces of {sample} atoms of the 8,192,000-atom configuration "
                      f"(one evaluation, neighbours found afresh; the integrator update is negligible), "
                      f"median of 3 runs after a warm-up: {dt:.2f} s on {n_thr} threads"}


def oracle_rates(model, nve_system, cell_samples):
    """The oracle timed beside the GPU figures of the other workloads (median
    of 3 after a warm-up, all host threads): one energy + forces + virial
    evaluation of the whole 128,000-atom cell (atom-steps/s; the integrator
    update is negligible), and the sampled cells of each batch (cells/s; with
    dE/dtheta for the differentiable batch)."""
    import oracle

    def med(fn):
        fn()
        runs = []
        for _ in range(3):
            t0 = time.time()
            fn()
            runs.append(time.time() - t0)
        return float(np.median(runs))
    out = {"threads": oracle.num_threads()}
    if nve_system is not None:
        t = med(lambda: oracle.efv_cell(model, nve_system.pos, nve_system.h[0]))
        out["mid_128000"] = {"atom_steps_per_s": nve_system.n_atoms / t, "seconds": t}
    for name, (cells, with_grad) in cell_samples.items():
        def run():
            for pos, h in cells:
                oracle.efv_cell(model, pos, h)
                if with_grad:
                    oracle.param_grad_cell(model, pos, h)
        t = med(run)
        out[name] = {"cells_per_s": len(cells) / t, "n_cells": len(cells), "with_param_grad": with_grad,
                     "seconds": t}
    return out


def fp64_checks(checks):
    """FP64 oracle references for the GPU results that the other sections
    sampled (part of the CPU leg: the only place the bench runs the oracle).
    A check is either sampled atoms of one cell (model, pos, h, pbc, idx, F,
    optional site energies e and an atom to leave out) or a list of whole
    cells (model, cells: [(pos, h, F)])."""
    import oracle
    res = {}
    for name, c in checks.items():
        if "cells" in c:
            num = den = 0.0
            for pos, h, F in c["cells"]:
                r = oracle.efv_cell(c["model"], pos, h, virial=False)
                num += float(np.sum((F - r["forces"]) ** 2))
                den += float(np.sum(r["forces"] ** 2))
            res[name] = {"force_rel_err": (num / den) ** 0.5}
            continue
        ref = oracle.efv_cell(c["model"], c["pos"], c["h"], c["pbc"], targets=c["idx"], virial=False)
        F, Fr = c["F"], ref["forces"]
        out = {"force_rel_err": float(np.linalg.norm(F - Fr) / np.linalg.norm(Fr))}
        ex = c.get("exclude")
        if ex is not None:
            keep = c["idx"] != ex
            out["force_rel_err_without_excluded"] = float(np.linalg.norm(F[keep] - Fr[keep]) /
                                                          np.linalg.norm(Fr[keep]))
        if c.get("e") is not None:
            out["site_energy_max_abs_err"] = float(np.max(np.abs(c["e"] - ref["energy_atom"])))
        res[name] = out
    return res


def summarize_rocprof(kt_dir, fetch_dir, write_dir, n_atoms, command, out_dir):
    """Write profiles/ summaries from rocprofv3 output: kernel-trace statistics
    and the HBM bytes per launch from FETCH_SIZE / WRITE_SIZE, scaled by what
    the counters read for the plain 1 GiB device copy (__amd_rocclr_copyBuffer)."""
    import csv
    import glob

    def one(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        if not f:
            raise FileNotFoundError(os.path.join(d, pat))
        return f[0]

    rows = list(csv.DictReader(open(one(kt_dir, "*kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel time, NEP-ZBL MD of %d-atom bcc W" % n_atoms, "", "Command:", "",
             "    " + command["kt"], "", "| kernel | calls | avg ms | total % |", "|---|---|---|---|"]
    for r in rows[:16]:
        name = r["Name"].split("(")[0]
        lines.append("| %s | %s | %.3f | %.1f |" % (name, r["Calls"], float(r["AverageNs"]) / 1e6,
                                                    float(r["Percentage"])))
    # the list-build kernels are launched every step and return at once
    # unless an atom moved more than skin/2: their cost per actual rebuild
    trace = glob.glob(os.path.join(kt_dir, "**", "*kernel_trace.csv"), recursive=True)
    if trace:
        dur = {}
        for r in csv.DictReader(open(trace[0])):
            name = r["Kernel_Name"].split("(")[0]
            if "build" in name:
                dur.setdefault(name, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
        lines += ["", "List build per rebuild (launches longer than 0.5 ms; the others found no rebuild due):", "",
                  "| kernel | rebuilds | avg ms per rebuild |", "|---|---|---|"]
        for name, d in sorted(dur.items()):
            big = [x for x in d if x > 0.5]
            if big:
                lines.append("| %s | %d | %.3f |" % (name, len(big), float(np.mean(big))))
    with open(os.path.join(out_dir, "nep_md_%d_kernel_stats.md" % n_atoms), "w") as f:
        f.write("\n".join(lines) + "\n")

    def counters(d, cname):
        acc = {}
        for r in csv.DictReader(open(one(d, "*counter_collection.csv"))):
            if r["Counter_Name"] != cname:
                continue
            name = r["Kernel_Name"].split("(")[0]
            name = (name[5:] if name.startswith("void ") else name).split("<")[0]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
        return acc
    fe = counters(fetch_dir, "FETCH_SIZE")
    wr = counters(write_dir, "WRITE_SIZE")
    gib_kib = 1 << 20
    f_fac = gib_kib / max(fe["__amd_rocclr_copyBuffer"])       # 1 GiB read by the calibration copy
    w_fac = gib_kib / max(wr["__amd_rocclr_copyBuffer"])       # 1 GiB written
    out = {"source_hash": _kernel_source_hash(), "n_atoms": n_atoms, "fetch_factor": f_fac,
           "write_factor": w_fac, "kernels": {}, "commands": command}
    lines = ["# HBM traffic per launch, NEP-ZBL MD of %d-atom bcc W" % n_atoms, "",
             "Commands (FETCH_SIZE and WRITE_SIZE in separate runs):", "",
             "    " + command["fetch"], "    " + command["write"], "",
             "Calibration: a plain 1 GiB device copy reads FETCH_SIZE x %.3f and WRITE_SIZE x %.3f of "
             "its true bytes; all values below are scaled by those factors." % (1 / f_fac, 1 / w_fac), "",
             "| kernel | launches | GB read | GB written | bytes/atom |", "|---|---|---|---|---|"]
    for k in ("nep::k_descriptor", "nep::k_force", "nep::k_sort_positions", "nep::k_kick_drift",
              "nep::k_kick", "nep::k_reduce_chunks", "nep::k_build_lists_blocks", "nep::k_build_lists",
              "nep::k_build_reverse"):
        if k not in fe or k not in wr:
            continue
        rd = float(np.median(fe[k])) * 1024 * f_fac
        wb = float(np.median(wr[k])) * 1024 * w_fac
        if k in ("nep::k_build_lists_blocks", "nep::k_build_lists", "nep::k_build_reverse"):
            rd = max(fe[k]) * 1024 * f_fac
            wb = max(wr[k]) * 1024 * w_fac
        out["kernels"][k.split("::")[1]] = {"read_bytes": rd, "write_bytes": wb, "bytes_per_launch": rd + wb}
        lines.append("| %s | %d | %.2f | %.2f | %.0f |" % (k.split("::")[1], len(fe[k]), rd / 1e9, wb / 1e9,
                                                           (rd + wb) / n_atoms))
    with open(os.path.join(out_dir, "nep_md_%d_hbm_counters.md" % n_atoms), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, "hbm_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)


def _subset_system(full, picks):
    import nep_synth
    sizes = np.diff(full.cell_start)
    pos = np.concatenate([full.cell(c)[0] for c in picks])
    starts = np.concatenate([[0], np.cumsum([sizes[c] for c in picks])]).astype(np.int64)
    return nep_synth.System(pos=pos, vel=np.zeros_like(pos), cell_start=starts, h=full.h[list(picks)].copy())


def _timed(fn, reps, torch, stream=None):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_paper_model(args, s, N):
    """MD of the same 8,192,000-atom workload with the paper-size model
    (n_max^R = 15, n_max^A = 10, l_max = 4, 100 neurons; random weights): the
    model size of the paper's own speed figure (Table IV: 1.3e7 atom-steps/s
    on one A100, quoted as context)."""
    import torch
    import nep_synth
    import paper_2305_08140_amd as nep
    pm = nep_synth.random_model(size="paper")
    idx = np.sort(np.random.default_rng(0).choice(N, size=256, replace=False))

    def run(mode):
        # the same start for both network units: a fresh copy of the workload
        sysd = nep.DeviceSystem.from_synth(s)
        ctx = nep.Context(pm, N, 1, max_neigh_ang=48, max_neigh_rad=96, skin=1.0)
        ctx.nep_set_precision(mode)
        out = nep.EFV(N, 1)
        md = dict(dt_max=1.0, max_disp=0.015)
        ctx.nep_step_verlet(sysd, 5, out, forces_valid=False, **md)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.nep_step_verlet(sysd, args.paper_steps, out, forces_valid=True, **md)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = ctx.nep_time_efv(sysd, out, reps=3)
        n_rad, n_ang = ctx.nep_mean_neighbors()
        check = {"model": pm, "pos": sysd.positions().cpu().numpy(), "h": s.h[0], "pbc": (1, 1, 1), "idx": idx,
                 "F": out.forces().cpu().numpy().astype(np.float64)[idx]}
        del ctx, out, sysd
        torch.cuda.empty_cache()
        return wall, kt, (n_rad, n_ang), check

    wall, kt, (n_rad, n_ang), check = run(0)
    f_desc, f_force = flops_per_atom(n_rad, n_ang, kr=16, nr=16, ka=11, na=11, nh=100)
    roof = {}
    for part, f, ms in (("descriptor_phases", f_desc, kt["descriptor"]), ("force", f_force, kt["force"])):
        ach = f * N / (ms * 1e-3) / 1e12
        roof[part] = {"bound": "alu", "flop_per_atom": f, "ms": ms, "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                      "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS}
    res = {"atom_steps_per_s": N * args.paper_steps / wall, "ms_per_step": wall / args.paper_steps * 1e3,
           "steps": args.paper_steps, "kernels_ms": kt, "roofline": roof, "network": "fp32_vector",
           "force_rel_err_vs_fp64_thermal_atoms": None,
           "paper_a100_atom_steps_per_s": 1.3e7}
    # the hidden layer on the matrix cores (precision mode 2: FP32 operands)
    wall2, kt2, _, check2 = run(2)
    res["matrix_core_network"] = {"atom_steps_per_s": N * args.paper_steps / wall2,
                                  "ms_per_step": wall2 / args.paper_steps * 1e3, "kernels_ms": kt2,
                                  "network": "fp32_mfma", "force_rel_err_vs_fp64_thermal_atoms": None}
    return res, {"paper_model": check, "paper_model_mfma": check2}


def bench_nve(args, model):
    """NVE of the 128,000-atom cell (40^3 bcc W cells, Maxwell-Boltzmann
    300 K on lattice sites): args.nve_steps velocity-Verlet steps of 1 fs in
    chunks of 50; the total energy after every chunk gives its drift (slope of
    a linear fit, eV/atom/ps) and its largest excursion."""
    import torch
    import nep_synth
    import paper_2305_08140_amd as nep
    ev_per_u = 1.602176634e-19 / 1.66053906660e-27 * 1e-10   # (eV/u) -> (A/fs)^2, CODATA 2018
    s = nep_synth.mid()
    N = s.n_atoms
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(model, N, 1, max_neigh_ang=48, max_neigh_rad=96, skin=1.0, check=False)
    out = nep.EFV(N, 1)
    chunk = 50
    n_chunks = max(1, args.nve_steps // chunk)
    etot = []

    def total_energy():
        v = sysd.velocities().double()
        return out.energy.item() + 0.5 * s.mass * float((v * v).sum()) / ev_per_u

    ctx.nep_step_verlet(sysd, 0, out, dt_max=1.0)
    torch.cuda.synchronize()
    etot.append(total_energy())
    wall = 0.0
    for k in range(n_chunks):
        t0 = time.perf_counter()
        ctx.nep_step_verlet(sysd, chunk, out, dt_max=1.0, forces_valid=True)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        etot.append(total_energy())
    ctx.nep_status()
    e = np.array(etot) / N
    t_ps = np.arange(len(e)) * chunk * 1e-3
    slope = float(np.polyfit(t_ps, e, 1)[0])
    res = {"n_atoms": N, "steps": n_chunks * chunk, "dt_fs": 1.0, "atom_steps_per_s": N * n_chunks * chunk / wall,
           "drift_eV_per_atom_per_ps": slope, "max_abs_excursion_eV_per_atom": float(np.max(np.abs(e - e[0])))}
    del ctx, out, sysd
    torch.cuda.empty_cache()
    return res


def bench_foil(args, model):
    """The paper's production cascade set-up (Sec. II.B, Table I foil row):
    a 150 x 150 x 180-cell W foil (8,100,000 atoms), open along z, 300 K, the
    3 a0 layers at the x and y faces held at 300 K by a Nose-Hoover chain of 3
    (tau = 100 fs, not stated in the paper), one 200 keV PKA along <135> into
    the foil 4 cells below the top surface, adaptive step (0.01 A, <= 1 fs)."""
    import torch
    import nep_synth
    import paper_2305_08140_amd as nep
    f = nep_synth.cascade((150, 150, 180), foil=True, pka_ev=200e3)
    N = f.n_atoms
    sysd = nep.DeviceSystem.from_synth(f)
    ctx = nep.Context(model, N, 1, max_neigh_ang=48, max_neigh_rad=96, skin=1.0)
    out = nep.EFV(N, 1)
    th = dict(T=300.0, tau=100.0, border=3 * nep_synth.A_W, axes=(0, 1), chain=3)
    md = dict(dt_max=1.0, max_disp=0.01, dt_min=1e-7)
    ctx.nep_step_verlet(sysd, 5, out, forces_valid=False, thermostat=th, **md)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.nep_step_verlet(sysd, args.foil_steps, out, forces_valid=True, thermostat=th, **md)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pka = f.meta["pka"]
    idx = np.sort(np.random.default_rng(1).choice(N, size=256, replace=False))
    check = {"model": model, "pos": sysd.positions().cpu().numpy(), "h": f.h[0], "pbc": f.pbc, "idx": idx,
             "F": out.forces().cpu().numpy().astype(np.float64)[idx]}
    res = {"atom_steps_per_s": N * args.foil_steps / wall, "ms_per_step": wall / args.foil_steps * 1e3,
           "steps": args.foil_steps, "n_atoms": N, "n_border": st["n_border"],
           "border_temperature_K": st["border_temperature"], "dt_last_fs": st["dt_last"],
           "time_fs": st["time"], "n_rebuilds": st["n_rebuilds"],
           "pka_speed_A_per_fs": float(np.linalg.norm(sysd.velocities()[pka].cpu().numpy())),
           "force_rel_err_vs_fp64_sampled": None}
    del ctx, out, sysd
    torch.cuda.empty_cache()
    return res, check


def bench_snes(args, model, n_pop=50):
    """SNES training generations (Sec. III.A: population 50, the paper's loss
    weights) on the 4,096-cell batch standing in for the training set
    (energies, forces and virials of every cell; targets from another random
    model evaluated by the same library).  Timed: sampling, the population's
    energies/forces/virials and loss terms, and the update, all on the device
    (draws generated beforehand).  Compared with evaluating the members one at
    a time (nep_set_weights + nep_compute_efv per member, no loss)."""
    import torch
    import nep_synth
    import paper_2305_08140_amd as nep
    s = nep_synth.batch()
    N, C_ = s.n_atoms, s.n_cells
    sysd = nep.DeviceSystem.from_synth(s)
    teacher = nep_synth.random_model(seed=77)
    ct = nep.Context(teacher, N, C_, check=False)
    o = nep.EFV(N, C_)
    ct.nep_build_neighbors(sysd)
    ct.nep_compute_efv(sysd, o)
    ct.nep_status()
    targets = {"energy": o.energy.clone(), "forces": torch.stack([o.fx, o.fy, o.fz]).clone(),
               "virial": o.virial.clone(), "has_virial": None}
    del ct
    ctx = nep.Context(model, N, C_, check=False)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_population_reserve(n_pop)
    n_par = ctx.nep_num_params()
    mu = torch.tensor(model.param_vector().astype(np.float32), device="cuda")
    sigma = torch.full_like(mu, 0.1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    draws = torch.randn(args.snes_gens + 2, n_pop, n_par, device="cuda", generator=gen)
    loss0 = nep.snes_generation(ctx, sysd, mu, sigma, draws[0], targets)[:, 0].min().item()
    nep.snes_generation(ctx, sysd, mu, sigma, draws[1], targets)
    ctx.nep_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(args.snes_gens):
        loss = nep.snes_generation(ctx, sysd, mu, sigma, draws[2 + g], targets)
    torch.cuda.synchronize()
    t_gen = (time.perf_counter() - t0) / args.snes_gens
    ctx.nep_status()
    best = loss[:, 0].min().item()
    # members one at a time through the single-model path
    thetas = nep.snes_sample(mu, sigma, draws[-1]).cpu().numpy().astype(np.float64)
    single = nep.Context(model, N, C_, check=False)
    single.nep_build_neighbors(sysd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_pop):
        single.nep_set_weights(model.with_param_vector(thetas[k]))
        single.nep_compute_efv(sysd, o)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    res = {"n_pop": n_pop, "n_cells": C_, "n_atoms": N, "n_params": n_par, "generations": args.snes_gens,
           "ms_per_generation": t_gen * 1e3, "member_cell_evaluations_per_s": n_pop * C_ / t_gen,
           "member_atom_evaluations_per_s": n_pop * N / t_gen,
           "one_member_at_a_time_ms": t_seq * 1e3, "speedup_vs_one_member_at_a_time": t_seq / t_gen,
           "best_loss_first_generation": loss0, "best_loss_last_generation": best}
    del ctx, single, sysd, o, targets, draws
    torch.cuda.empty_cache()
    return res


def bench_batches(model, reps=20, n_percell=128):
    """Batched evaluation of many small cells against per-cell launches.

    batch:     4,096 cells of 8-512 atoms (log-uniform), vacancies, half strained
               -> energy + forces + virial of all cells per evaluation
    diffbatch: 512 cells of 16-256 atoms, +-3 % strain
               -> energy, forces, virial and dE/dtheta (backward) per evaluation
    The per-cell path evaluates a sample of n_percell cells one by one (each
    with its own context, lists prebuilt, launches back to back, one sync)."""
    import torch
    import nep_synth
    import paper_2305_08140_amd as nep
    out, checks = {}, {}
    rng = np.random.default_rng(0)
    for name in ("batch", "diffbatch"):
        s = nep_synth.WORKLOADS[name]()
        C_ = s.n_cells
        sysd = nep.DeviceSystem.from_synth(s)
        ctx = nep.Context(model, s.n_atoms, C_, check=False)
        o = nep.EFV(s.n_atoms, C_)
        ctx.nep_build_neighbors(sysd)
        ctx.nep_compute_efv(sysd, o)
        ctx.nep_status()
        shapes = ctx.nep_autotune(sysd, o, reps=3)
        gE = torch.ones(C_, dtype=torch.float64, device="cuda")
        diff = name == "diffbatch"

        def batched():
            ctx.nep_compute_efv(sysd, o)
            if diff:
                ctx.nep_backward(sysd, o, gE, grad_pos=False, grad_cell=False)
        t_b = _timed(batched, reps, torch)
        res = {"n_cells": C_, "n_atoms": s.n_atoms, "launch_shapes": shapes,
               "batched_cells_per_s": C_ / t_b, "batched_ms": t_b * 1e3}
        if not diff:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                t_g = _timed(lambda: ctx.nep_compute_efv_graph(sysd, o, stream=st), reps, torch)
            res["graph_cells_per_s"] = C_ / t_g
            res["graph_ms"] = t_g * 1e3
        ctx.nep_status()
        # sampled cells for the FP64 check of the CPU leg
        picks16 = rng.choice(C_, size=16, replace=False)

        def sampled_cells():
            F = o.forces().cpu().numpy().astype(np.float64)
            cells = []
            for c in picks16:
                a, b = int(s.cell_start[c]), int(s.cell_start[c + 1])
                cells.append((s.pos[a:b].copy(), s.h[c].copy(), F[a:b].copy()))
            return cells
        ctx.nep_compute_efv(sysd, o)
        checks["batch_" + name] = {"model": model, "cells": sampled_cells()}
        res["force_rel_err_vs_fp64"] = None
        if not diff:
            # hidden layer on the matrix cores: BF16 (mode 1) and FP32 (mode 2)
            res["precision_variants"] = {}
            for mode, label in ((1, "bf16_mfma"), (2, "fp32_mfma")):
                ctx.nep_set_precision(mode)
                t_m = _timed(lambda: ctx.nep_compute_efv(sysd, o), reps, torch)
                ctx.nep_status()
                checks[f"batch_{name}_{label}"] = {"model": model, "cells": sampled_cells()}
                res["precision_variants"][label] = {"cells_per_s": C_ / t_m, "ms": t_m * 1e3,
                                                    "force_rel_err_vs_fp64": None}
            ctx.nep_set_precision(0)
        # per-cell path on a sample of cells
        picks = rng.choice(C_, size=min(n_percell, C_), replace=False)
        per = []
        for c in picks:
            sc = _subset_system(s, [int(c)])
            d = nep.DeviceSystem.from_synth(sc)
            cx = nep.Context(model, sc.n_atoms, 1, check=False)
            oc = nep.EFV(sc.n_atoms, 1)
            cx.nep_build_neighbors(d)
            per.append((cx, d, oc))
        g1 = torch.ones(1, dtype=torch.float64, device="cuda")

        def percell():
            for cx, d, oc in per:
                cx.nep_compute_efv(d, oc)
                if diff:
                    cx.nep_backward(d, oc, g1, grad_pos=False, grad_cell=False)
        t_p = _timed(percell, max(2, reps // 4), torch)
        res["per_cell_cells_per_s"] = len(per) / t_p
        res["speedup_vs_per_cell"] = res["batched_cells_per_s"] / res["per_cell_cells_per_s"]
        out[name] = res
        del per, ctx, sysd, o
        torch.cuda.empty_cache()
    return out, checks


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cells", type=int, default=160, help="conventional cells per edge")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batches", action="store_true", help="skip the batched small-cell workloads")
    ap.add_argument("--paper-steps", type=int, default=50,
                    help="MD steps of the paper-size model on the same workload (0 skips it)")
    ap.add_argument("--foil-steps", type=int, default=50,
                    help="MD steps of the 8,100,000-atom foil cascade with the border thermostat (0 skips it)")
    ap.add_argument("--nve-steps", type=int, default=1000,
                    help="NVE steps of 1 fs on the 128,000-atom cell for the energy drift (0 skips it)")
    ap.add_argument("--snes-gens", type=int, default=10,
                    help="timed SNES generations (population 50) on the 4,096-cell batch (0 skips it)")
    ap.add_argument("--timing-reps", type=int, default=5)
    ap.add_argument("--rebuild-probe-steps", type=int, default=300,
                    help="MD steps after the timed region that measure the rebuild rate (0 skips it)")
    ap.add_argument("--summarize-rocprof", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 output directories and exit")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        n = 2 * args.cells ** 3
        kt_dir, fetch_dir, write_dir = args.summarize_rocprof
        cmd = {"kt": "rocprofv3 --kernel-trace --stats -d %s -o kt --output-format csv -- "
                     "python3 bench.py --steps 500 --warmup 10 --no-cpu-baseline --no-batches --foil-steps 0 --snes-gens 0 "
                     "--nve-steps 0 --paper-steps 0" % kt_dir,
               "fetch": "rocprofv3 --pmc FETCH_SIZE -d %s -o f --output-format csv -- "
                        "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-batches --foil-steps 0 "
                        "--snes-gens 0 --nve-steps 0 --paper-steps 0 --rebuild-probe-steps 0 "
                        "--copy-calibration-mib 1024 --timing-reps 1" % fetch_dir,
               "write": "rocprofv3 --pmc WRITE_SIZE -d %s -o w --output-format csv -- "
                        "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-batches --foil-steps 0 "
                        "--snes-gens 0 --nve-steps 0 --paper-steps 0 --rebuild-probe-steps 0 "
                        "--copy-calibration-mib 1024 --timing-reps 1" % write_dir}
        summarize_rocprof(*args.summarize_rocprof, n, cmd, os.path.join(ROOT, "profiles"))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the NEP-ZBL evaluation runs on exactly one GPU (it is not sharded "
              "across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import nep_synth
    import paper_2305_08140_amd as nep

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    model = nep_synth.random_model()
    s = nep_synth.large(n_cells=args.cells)
    N = s.n_atoms
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(model, N, 1, max_neigh_ang=48, max_neigh_rad=96, skin=1.0, check=True)
    out = nep.EFV(N, 1)
    md = dict(dt_max=1.0, max_disp=0.015, dt_min=1e-6)

    # warm-up (includes the first neighbour build and force evaluation)
    ctx.nep_step_verlet(sysd, args.warmup, out, forces_valid=False, **md)
    torch.cuda.synchronize()

    # timed region: K full MD steps in one chunk
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = ctx.nep_step_verlet(sysd, args.steps, out, forces_valid=True, time_kernels=True, **md)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = N * args.steps / wall

    # neighbour rebuilds: the cost of one (HIP events around a forced
    # rebuild of the current configuration, the same kernels the MD loop
    # runs when an atom has moved more than skin / 2), and their rate over a
    # longer probe chunk that carries its rebuilds, timed as a whole
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reb_ms = []
    for _ in range(3):
        ev0.record()
        ctx.nep_build_neighbors(sysd)
        ev1.record()
        torch.cuda.synchronize()
        reb_ms.append(ev0.elapsed_time(ev1))
    rebuild_ms = float(np.median(reb_ms))
    ctx.nep_compute_efv(sysd, out)          # forces of the current positions again
    torch.cuda.synchronize()
    rebuild = None
    if args.rebuild_probe_steps > 0:
        t0 = time.perf_counter()
        pst = ctx.nep_step_verlet(sysd, args.rebuild_probe_steps, out, forces_valid=True, **md)
        torch.cuda.synchronize()
        t_probe = time.perf_counter() - t0
        rps = pst["n_rebuilds"] / args.rebuild_probe_steps
        # per-step time of the timed chunk without its own rebuilds, plus the
        # probe's rebuild rate at the measured rebuild cost
        t_step_plain = (wall - stats["n_rebuilds"] * rebuild_ms * 1e-3) / args.steps
        t_step_amort = t_step_plain + rps * rebuild_ms * 1e-3
        rebuild = {"ms_per_rebuild": rebuild_ms, "rebuilds_in_timed_steps": stats["n_rebuilds"],
                   "probe_steps": args.rebuild_probe_steps, "probe_rebuilds": pst["n_rebuilds"],
                   "rebuilds_per_step": rps, "probe_atom_steps_per_s": N * args.rebuild_probe_steps / t_probe,
                   "amortised_atom_steps_per_s": N / t_step_amort,
                   "amortised_ms_per_step": t_step_amort * 1e3}

    # per-kernel durations: HIP events on the library's stream around the
    # descriptor and force kernels of every timed step (live), and a
    # breakdown of one evaluation at the final state
    klive = {"descriptor": stats["ms_descriptor"], "force": stats["ms_force"], "steps": stats["n_timed_steps"]}
    ctx.nep_compute_efv(sysd, out)
    ktimes = ctx.nep_time_efv(sysd, out, reps=args.timing_reps)
    n_rad, n_ang = ctx.nep_mean_neighbors()
    f_desc, f_force = flops_per_atom(n_rad, n_ang)
    # dominant kernel: the one with the longest launch
    dom = "descriptor" if klive["descriptor"] >= klive["force"] else "force"
    f_dom = f_desc if dom == "descriptor" else f_force
    achieved = f_dom * N / (klive[dom] * 1e-3) / 1e12
    traffic = _traffic("k_" + dom, N)

    # sampled atoms of the final configuration (and the PKA) for the FP64
    # check of the CPU leg; the PKA's force would dominate the norm, so the
    # thermal atoms are also checked on their own
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(N, size=256, replace=False))
    pka = s.meta["pka"]
    idx = np.unique(np.concatenate([idx, [pka]]))
    checks = {"bulk": {"model": model, "pos": sysd.positions().cpu().numpy(), "h": s.h[0], "pbc": (1, 1, 1),
                       "idx": idx, "F": out.forces().cpu().numpy().astype(np.float64)[idx],
                       "e": out.energy_atom.cpu().numpy()[idx].astype(np.float64), "exclude": pka}}

    # Wigner-Seitz defect analysis of the final configuration (HBM-bound:
    # positions read, one occupancy update per atom, occupancy cleared and scanned)
    ws_ref_cells = (args.cells, args.cells, args.cells)
    res_ws = nep.wigner_seitz(sysd, nep_synth.A_W, ws_ref_cells)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        res_ws = nep.wigner_seitz(sysd, nep_synth.A_W, ws_ref_cells)
    torch.cuda.synchronize()
    t_ws = (time.perf_counter() - t0) / 5
    m_sites = 2 * args.cells ** 3
    ws_bytes = 24 * N + 8 * N + 3 * 4 * m_sites
    defects = {"ms": t_ws * 1e3, "algorithmic_bytes": ws_bytes, "GB_per_s": ws_bytes / t_ws / 1e9,
               "n_vacancies": res_ws["n_vacancies"], "n_interstitials": res_ws["n_interstitials"],
               "n_vacancy_clusters": res_ws["n_vacancy_clusters"],
               "n_interstitial_clusters": res_ws["n_interstitial_clusters"]}

    del ctx, sysd, out
    torch.cuda.empty_cache()
    paper = foil = batches = snes = nve = None
    if args.nve_steps > 0:
        nve = bench_nve(args, model)
    if args.paper_steps > 0:
        paper, pc = bench_paper_model(args, s, N)
        checks.update(pc)
    if args.foil_steps > 0:
        foil, checks["foil"] = bench_foil(args, model)
    if args.snes_gens > 0:
        snes = bench_snes(args, model)
    if not args.no_batches:
        batches, bc = bench_batches(model)
        checks.update(bc)

    # CPU leg: the oracle's own throughput, and the FP64 references of the
    # sampled GPU results
    cpu = None
    ferr = ferr_th = eerr = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(model, s)
        samples = {k[len("batch_"):]: ([(pos, h) for pos, h, _ in v["cells"]], k == "batch_diffbatch")
                   for k, v in checks.items() if k in ("batch_batch", "batch_diffbatch")}
        rates = oracle_rates(model, nep_synth.mid() if nve is not None else None, samples)
        if nve is not None:
            nve["cpu_oracle_atom_steps_per_s"] = rates["mid_128000"]["atom_steps_per_s"]
            nve["cpu_oracle_threads"] = rates["threads"]
        if batches is not None:
            for name in batches:
                if name in rates:
                    batches[name]["cpu_oracle_cells_per_s"] = rates[name]["cells_per_s"]
                    batches[name]["cpu_oracle_sample"] = (
                        f"{rates[name]['n_cells']} sampled cells, energy + forces + virial"
                        + (" + dE/dtheta" if rates[name]["with_param_grad"] else "")
                        + f", median of 3 after a warm-up on {rates['threads']} threads")
        acc = fp64_checks(checks)
        ferr = acc["bulk"]["force_rel_err"]
        ferr_th = acc["bulk"]["force_rel_err_without_excluded"]
        eerr = acc["bulk"]["site_energy_max_abs_err"]
        if paper is not None:
            paper["force_rel_err_vs_fp64_thermal_atoms"] = acc["paper_model"]["force_rel_err"]
            paper["matrix_core_network"]["force_rel_err_vs_fp64_thermal_atoms"] = \
                acc["paper_model_mfma"]["force_rel_err"]
        if foil is not None:
            foil["force_rel_err_vs_fp64_sampled"] = acc["foil"]["force_rel_err"]
        if batches is not None:
            for name in batches:
                batches[name]["force_rel_err_vs_fp64"] = acc["batch_" + name]["force_rel_err"]
                for label, v in batches[name].get("precision_variants", {}).items():
                    v["force_rel_err_vs_fp64"] = acc[f"batch_{name}_{label}"]["force_rel_err"]

    line = {
        "metric": "atom-steps/s NEP-ZBL E+F+virial (plain vs batched/differentiable), force err vs FP64",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"plain MD, {N} atom bcc W ({args.cells}^3 cells), 300 K + 1 keV PKA, "
                               "adaptive dt (0.015 A/step, <= 1 fs), 1 A skin",
                   "n_atoms": N, "model": "NEP-ZBL r_c 6/4 A, 9+20 descriptors, 30 tanh, random weights"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic, "kernel": "k_" + dom},
        "cpu_baseline": cpu,
        "kernels_ms_timed_steps": klive,
        "kernels_ms_final_state": ktimes,
        "flops_per_atom": {"descriptor": f_desc, "force": f_force, "mean_neighbors_rad": n_rad,
                           "mean_neighbors_ang": n_ang},
        "kernel_tflops": {"descriptor": f_desc * N / (klive["descriptor"] * 1e-3) / 1e12,
                          "force": f_force * N / (klive["force"] * 1e-3) / 1e12},
        "md": {"n_rebuilds": stats["n_rebuilds"], "dt_last_fs": stats["dt_last"], "time_fs": stats["time"]},
        "rebuild": rebuild,
        "force_rel_err_vs_fp64": ferr, "force_rel_err_vs_fp64_thermal_atoms": ferr_th,
        "site_energy_max_abs_err_eV": eerr,
        "defects": defects,
        "paper_model": paper,
        "foil_cascade": foil,
        "nve_128000": nve,
        "snes": snes,
        "batches": batches,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
