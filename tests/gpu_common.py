"""Shared helpers of the GPU tests: run the HIP library and the oracle on the same inputs."""
import numpy as np

import nep_synth

# Tolerances (the requirement is FP32 forces within 1e-5 relative of FP64 and
# energies within 1e-6 eV/atom):
F_REL_TOL = 1e-5      # ||F - F_ref||_F / ||F_ref||_F
E_ATOM_TOL = 1e-6     # |E - E_ref| / N  (eV/atom), per cell
# Virial: every pair adds an FP32 term of order |f| |r| ~ 1-10 eV with a
# relative rounding of ~1e-7; 60 pairs per atom summed in FP32 per atom then
# in FP64 over atoms give an absolute error ~1e-6 eV per atom, so
# ||W - W_ref||_F <= 1e-5 ||W_ref||_F + 1e-6 N  (eV).
W_REL_TOL = 1e-5
W_ATOM_TOL = 1e-6
# Per atom: |F_i - F_ref_i| <= F_ATOM_TOL max(|F_ref_i|, RMS |F_ref|) (an
# atom's FP32 error is set by its ~60 pair terms, not by its net force, so
# atoms whose net force is far below the RMS are measured against the RMS).
F_ATOM_TOL = 5e-5
# Site energies U_i of atoms in no pair closer than the ZBL outer radius
# (the network output in FP32 on FP64-accurate descriptors), eV.
U_SITE_TOL = 1e-6


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def force_errors(F, Fref, exclude=None):
    """Relative Frobenius error over all atoms, and over atoms not in `exclude`."""
    num = np.linalg.norm(F - Fref)
    den = np.linalg.norm(Fref)
    e_all = num / den
    if exclude is None or len(exclude) == 0:
        return e_all, e_all
    m = np.ones(F.shape[0], bool)
    m[list(exclude)] = False
    return e_all, np.linalg.norm(F[m] - Fref[m]) / np.linalg.norm(Fref[m])


def atom_force_error(F, Fref):
    """max_i |F_i - F_ref_i| / max(|F_ref_i|, RMS |F_ref|)."""
    nref = np.linalg.norm(Fref, axis=1)
    rms = np.sqrt(np.mean(nref ** 2))
    return float(np.max(np.linalg.norm(F - Fref, axis=1) / np.maximum(nref, rms)))


def zbl_atoms_system(s, r2=2.0):
    """Atoms (global indices) of a multi-cell system in a pair closer than r2."""
    import oracle
    out = set()
    for c in range(s.n_cells):
        a, b = int(s.cell_start[c]), int(s.cell_start[c + 1])
        pbc = tuple(getattr(s, "pbc", (1, 1, 1)))
        start, j, n, r = oracle.pairs(s.pos[a:b], s.h[c], pbc, r2, method=0 if b - a < 3000 else 1)
        for i in range(b - a):
            if start[i + 1] > start[i]:
                out.add(a + i)
    return out


def zbl_atoms(pos, h, r2=2.0):
    """Atoms that take part in a pair closer than r2 (they carry the ZBL forces)."""
    import oracle
    start, j, n, r = oracle.pairs(pos, h, (1, 1, 1), r2, method=0 if pos.shape[0] < 3000 else 1)
    out = set()
    for i in range(pos.shape[0]):
        if start[i + 1] > start[i]:
            out.add(i)
    return out


def run_gpu(model, s, max_neigh_ang=48, max_neigh_rad=96, skin=1.0):
    import paper_2305_08140_amd as nep
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(model, s.n_atoms, s.n_cells, max_neigh_ang, max_neigh_rad, skin)
    out = nep.EFV(s.n_atoms, s.n_cells)
    ctx.nep_build_neighbors(sysd)
    ctx.nep_compute_efv(sysd, out)
    import torch
    torch.cuda.synchronize()
    res = {"energy": out.energy.cpu().numpy(), "forces": out.forces().cpu().numpy().astype(np.float64),
           "virial": out.virial.cpu().numpy().reshape(-1, 3, 3), "energy_atom": out.energy_atom.cpu().numpy()}
    return res, ctx, sysd, out


def model():
    return nep_synth.random_model()
