"""Seeded synthetic inputs for the NEP-ZBL tungsten workloads.

This module only draws random numbers and lays out lattices; it holds none of
the potential's arithmetic.  Both the FP64 CPU oracle (test infrastructure)
and the HIP library are fed from here, so that the two sides see identical
inputs while sharing no code.

Workloads (synthetic body-centred-cubic tungsten, a = 3.165 A, Z = 74,
m = 183.84 u; the paper's cascades use bcc W, Sec. II.B and Table I):

* ``tiny``      2,000 atoms, 10x10x10 cells, sigma = 0.05 A noise and three
                atom pairs pulled to 0.8-1.6 A so that the ZBL branch (Eq. 2)
                is exercised.
* ``mid``       128,000 atoms, 40x40x40 cells, Maxwell-Boltzmann 300 K.
* ``large``     8,192,000 atoms, 160x160x160 cells, 300 K plus one 1 keV
                primary knock-on atom (PKA) near the box centre, moving along a
                seeded random direction (the paper launches PKAs at the box
                centre, Sec. II.B).
* ``diffbatch`` 512 periodic cells of 16-256 atoms, sigma = 0.1 A, random
                +-3 % symmetric strain.
* ``batch``     4,096 cells of 8-512 atoms (log-uniform), 1-3 % vacancies,
                half of the cells strained, sigma = 0.1 A.

Random model parameters follow a fixed recipe (uniform descriptor
coefficients, Gaussian network weights); the descriptor scale and the output
weight factor are read from ``model_scales.json``, which is written by a
calibration script that runs the reference CPU implementation.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

A_W = 3.165          # bcc W lattice constant, Angstrom
Z_W = 74             # atomic number of W
MASS_W = 183.84      # atomic mass of W, u

# Physical constants used only to draw velocities (CODATA 2018).
_KB_EV = 8.617333262e-5                      # Boltzmann constant, eV/K
_E_C = 1.602176634e-19                       # elementary charge, C
_AMU = 1.66053906660e-27                     # atomic mass unit, kg
_EV_PER_U_TO_A2_PER_FS2 = _E_C / _AMU * 1e-10  # (eV/u) -> (A/fs)^2

SEEDS = {"model": 8140, "tiny": 1, "mid": 2, "large": 3, "diffbatch": 4, "batch": 5, "cascade": 6}

_HERE = os.path.dirname(os.path.abspath(__file__))
SCALES_PATH = os.path.join(_HERE, "model_scales.json")


# --------------------------------------------------------------------------
# model
# --------------------------------------------------------------------------
@dataclass
class Model:
    """Hyperparameters and parameters of one NEP-ZBL model (single species).

    Descriptor ordering: radial components nu = n (n = 0..n_rad-1) first,
    then angular components nu = n_rad + n_ang*(l-1) + n for l = 1..l_max.
    """
    n_rad: int = 9            # radial descriptor components (n_max^R = 8)
    n_ang: int = 5            # angular radial functions (n_max^A = 4)
    k_rad: int = 9            # Chebyshev basis functions, radial (k = 0..8)
    k_ang: int = 9            # Chebyshev basis functions, angular
    l_max: int = 4
    n_hidden: int = 30
    rc_rad: float = 6.0       # radial cutoff, A (Sec. III.A)
    rc_ang: float = 4.0       # angular cutoff, A (Sec. III.A)
    zbl_r1: float = 1.0       # ZBL blend inner cutoff, A (Sec. II.A)
    zbl_r2: float = 2.0       # ZBL blend outer cutoff, A
    Z: int = Z_W
    mass: float = MASS_W
    c_rad: np.ndarray = field(default=None)   # [n_rad, k_rad]
    c_ang: np.ndarray = field(default=None)   # [n_ang, k_ang]
    q_scale: np.ndarray = field(default=None)  # [D]
    w0: np.ndarray = field(default=None)      # [n_hidden, D]
    b0: np.ndarray = field(default=None)      # [n_hidden]
    w1: np.ndarray = field(default=None)      # [n_hidden]
    b1: float = 0.0

    @property
    def dim(self) -> int:
        return self.n_rad + self.n_ang * self.l_max

    def copy(self) -> "Model":
        m = Model(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        for k in ("c_rad", "c_ang", "q_scale", "w0", "b0", "w1"):
            setattr(m, k, np.array(getattr(self, k), dtype=np.float64, copy=True))
        return m

    def param_vector(self) -> np.ndarray:
        """Trainable parameters flattened as (c_rad, c_ang, w0, b0, w1, b1)."""
        return np.concatenate([self.c_rad.ravel(), self.c_ang.ravel(), self.w0.ravel(),
                               self.b0.ravel(), self.w1.ravel(), [self.b1]])

    def with_param_vector(self, v: np.ndarray) -> "Model":
        m = self.copy()
        o = 0
        for name in ("c_rad", "c_ang", "w0", "b0", "w1"):
            a = getattr(m, name)
            setattr(m, name, np.asarray(v[o:o + a.size], dtype=np.float64).reshape(a.shape).copy())
            o += a.size
        m.b1 = float(v[o])
        return m


def load_scales(path: str = SCALES_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


# The paper's own hyperparameters (Sec. III.A): Chebyshev expansion orders
# n_max^R = 15 and n_max^A = 10 (16 and 11 radial functions on as many basis
# functions), l_max = 4, 100 hidden neurons; same cutoffs.
PAPER_DIMS = {"n_rad": 16, "n_ang": 11, "k_rad": 16, "k_ang": 11, "l_max": 4, "n_hidden": 100}


def random_model(seed: int = SEEDS["model"], scaled: bool = True, size: str = "small") -> Model:
    """Random NEP model.

    c ~ U(-1, 1); w0 ~ N(0, 1/D); b0 ~ N(0, 0.1^2); w1 ~ N(0, 1/H); b1 = 0.
    With ``scaled`` the descriptor scale q_scale and a global factor kappa on
    w1 are taken from ``model_scales.json`` (q_scale = 1 / RMS descriptor on
    the tiny workload; kappa chosen so that the RMS non-ZBL force there is
    1 eV/A and the lattice is restoring).  Without it q_scale = 1, kappa = 1.
    ``size="paper"`` gives the paper's hyperparameters (PAPER_DIMS).
    """
    if size not in ("small", "paper"):
        raise ValueError(size)
    m = Model() if size == "small" else Model(**PAPER_DIMS)
    rng = np.random.Generator(np.random.PCG64(seed))
    D, H = m.dim, m.n_hidden
    m.c_rad = rng.uniform(-1.0, 1.0, size=(m.n_rad, m.k_rad))
    m.c_ang = rng.uniform(-1.0, 1.0, size=(m.n_ang, m.k_ang))
    m.w0 = rng.normal(0.0, 1.0 / np.sqrt(D), size=(H, D))
    m.b0 = rng.normal(0.0, 0.1, size=H)
    m.w1 = rng.normal(0.0, 1.0 / np.sqrt(H), size=H)
    m.b1 = 0.0
    m.q_scale = np.ones(D)
    if scaled:
        sc = load_scales()
        if sc is None or (size == "paper" and "paper" not in sc):
            raise FileNotFoundError(f"{SCALES_PATH} missing or incomplete: run oracle/calibrate.py")
        if size == "paper":
            sc = sc["paper"]
        m.q_scale = np.asarray(sc["q_scale"], dtype=np.float64)
        m.w1 = m.w1 * float(sc["kappa"])
    return m


# --------------------------------------------------------------------------
# structures
# --------------------------------------------------------------------------
@dataclass
class System:
    """A batch of periodic cells (one cell for the MD workloads).

    pos         [N, 3] float64, A
    vel         [N, 3] float64, A/fs (zeros when not drawn)
    cell_start  [n_cells + 1] int64, atoms of cell c are cell_start[c]:cell_start[c+1]
    h           [n_cells, 3, 3] float64, rows are the lattice vectors (x = s @ h)
    pbc         (3,) int, 1 = periodic along that lattice vector
    """
    pos: np.ndarray
    vel: np.ndarray
    cell_start: np.ndarray
    h: np.ndarray
    pbc: tuple = (1, 1, 1)
    mass: float = MASS_W
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.h.shape[0])

    def cell(self, c: int):
        s, e = int(self.cell_start[c]), int(self.cell_start[c + 1])
        return self.pos[s:e], self.h[c]


def bcc_lattice(nx: int, ny: int, nz: int, a: float = A_W):
    """Conventional bcc cells; atom order: cell-major (x fastest), corner then centre."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ix.transpose(2, 1, 0).ravel(), iy.transpose(2, 1, 0).ravel(),
                     iz.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)
    corner = base
    centre = base + 0.5
    pos = np.empty((2 * base.shape[0], 3))
    pos[0::2] = corner
    pos[1::2] = centre
    pos *= a
    h = np.diag([nx * a, ny * a, nz * a]).astype(np.float64)
    return pos, h


def maxwell_boltzmann(rng, n: int, temperature: float, mass: float = MASS_W):
    """Velocities (A/fs) drawn from N(0, kT/m), mean removed, rescaled to T exactly (3N-3 dof)."""
    s = np.sqrt(_KB_EV * temperature / mass * _EV_PER_U_TO_A2_PER_FS2)
    v = rng.normal(0.0, s, size=(n, 3))
    v -= v.mean(axis=0)
    ekin = 0.5 * mass * np.sum(v * v) / _EV_PER_U_TO_A2_PER_FS2   # eV
    t_now = 2.0 * ekin / ((3 * n - 3) * _KB_EV)
    v *= np.sqrt(temperature / t_now)
    return v


def speed_for_energy(e_ev: float, mass: float = MASS_W) -> float:
    """Speed (A/fs) of a particle of the given mass (u) and kinetic energy (eV)."""
    return float(np.sqrt(2.0 * e_ev / mass * _EV_PER_U_TO_A2_PER_FS2))


def _single(pos, h, vel=None, name="", meta=None) -> System:
    if vel is None:
        vel = np.zeros_like(pos)
    return System(pos=np.ascontiguousarray(pos), vel=np.ascontiguousarray(vel),
                  cell_start=np.array([0, pos.shape[0]], dtype=np.int64),
                  h=h.reshape(1, 3, 3).copy(), name=name, meta=meta or {})


def tiny(seed: int = SEEDS["tiny"], n_cells: int = 10, sigma: float = 0.05) -> System:
    """2,000-atom bcc W, sigma = 0.05 A noise, three nearest-neighbour pairs
    pulled symmetrically along their bond to a separation in U(0.8, 1.6) A."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, h = bcc_lattice(n_cells, n_cells, n_cells)
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    ncell = n_cells ** 3
    # three distinct conventional cells, well apart: corner atom 2c and centre atom 2c+1
    cells = rng.choice(ncell, size=3, replace=False)
    pulled = []
    for c in cells:
        i, j = 2 * int(c), 2 * int(c) + 1
        d = pos[j] - pos[i]
        r = np.linalg.norm(d)
        target = rng.uniform(0.8, 1.6)
        mid = 0.5 * (pos[i] + pos[j])
        u = d / r
        pos[i] = mid - 0.5 * target * u
        pos[j] = mid + 0.5 * target * u
        pulled.append((i, j, target))
    return _single(pos, h, name="tiny", meta={"pulled_pairs": pulled, "seed": seed})


def mid(seed: int = SEEDS["mid"], n_cells: int = 40, temperature: float = 300.0) -> System:
    """128,000-atom bcc W on perfect lattice sites with Maxwell-Boltzmann velocities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, h = bcc_lattice(n_cells, n_cells, n_cells)
    vel = maxwell_boltzmann(rng, pos.shape[0], temperature)
    return _single(pos, h, vel, name="mid", meta={"seed": seed, "T": temperature})


def large(seed: int = SEEDS["large"], n_cells: int = 160, temperature: float = 300.0,
          pka_ev: float = 1000.0) -> System:
    """8,192,000-atom bcc W at 300 K plus one PKA of ``pka_ev`` near the box centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, h = bcc_lattice(n_cells, n_cells, n_cells)
    vel = maxwell_boltzmann(rng, pos.shape[0], temperature)
    # corner atom of the central conventional cell
    c = n_cells // 2
    pka = 2 * ((c * n_cells + c) * n_cells + c)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    vel[pka] = speed_for_energy(pka_ev) * d
    return _single(pos, h, vel, name="large",
                   meta={"seed": seed, "T": temperature, "pka": int(pka), "pka_dir": d.tolist(),
                         "pka_ev": pka_ev})


def direction_135(rng, into_negative_z: bool = False):
    """A member of the <135> family (a permutation of (1, 3, 5) with random
    signs), unit length; with into_negative_z its z component is negative."""
    perm = rng.permutation(3)
    d = np.array([1.0, 3.0, 5.0])[perm] * rng.choice([-1.0, 1.0], size=3)
    if into_negative_z and d[2] > 0:
        d[2] = -d[2]
    return d / np.linalg.norm(d)


def cascade(n_cells=(150, 150, 180), foil: bool = True, pka_ev: float = 200e3, temperature: float = 300.0,
            seed: int = SEEDS["cascade"], depth_cells: int = 4, sigma: float = 0.045) -> System:
    """Cascade set-up of Sec. II.B / Table I: bcc W of nx x ny x nz conventional
    cells at `temperature`, one PKA of `pka_ev` along a seeded <135> direction.
    foil: open boundaries along z (free surfaces at z = 0 and the top), the
    PKA is the corner atom of the central column `depth_cells` cells below the
    top surface, heading into the foil; bulk: periodic, the PKA is the corner
    atom of the central cell.  The default is the 200 keV foil (8,100,000 atoms).
    Atoms sit on lattice sites displaced by N(0, sigma^2) per component
    (0.045 A: about the root-mean-square thermal displacement of W at 300 K),
    standing in for the paper's 30 ps equilibration."""
    nx, ny, nz = n_cells
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, h = bcc_lattice(nx, ny, nz)
    vel = maxwell_boltzmann(rng, pos.shape[0], temperature)
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    cz = nz - 1 - depth_cells if foil else nz // 2
    pka = 2 * ((cz * ny + ny // 2) * nx + nx // 2)
    d = direction_135(rng, into_negative_z=foil)
    vel[pka] = speed_for_energy(pka_ev) * d
    s = _single(pos, h, vel, name="foil" if foil else "bulk",
                meta={"seed": seed, "T": temperature, "pka": int(pka), "pka_dir": d.tolist(), "pka_ev": pka_ev,
                      "n_cells": (nx, ny, nz)})
    s.pbc = (1, 1, 0) if foil else (1, 1, 1)
    return s


def most_cubic_cells(n_target: int):
    """(n1, n2, n3) with 2*n1*n2*n3 nearest n_target, preferring the most cubic shape."""
    best = None
    m_target = max(1, int(round(n_target / 2)))
    for m in range(max(1, m_target - 8), m_target + 9):
        for n1 in range(1, m + 1):
            if m % n1:
                continue
            for n2 in range(n1, m // n1 + 1):
                if (m // n1) % n2:
                    continue
                n3 = m // n1 // n2
                if n3 < n2:
                    continue
                key = (abs(2 * m - n_target), n3 / n1, n1, n2, n3)
                if best is None or key < best:
                    best = key
    return best[2], best[3], best[4]


def _random_sym_strain(rng, amp: float):
    e = np.zeros((3, 3))
    d = rng.uniform(-amp, amp, size=6)
    e[0, 0], e[1, 1], e[2, 2] = d[0], d[1], d[2]
    e[0, 1] = e[1, 0] = d[3]
    e[0, 2] = e[2, 0] = d[4]
    e[1, 2] = e[2, 1] = d[5]
    return e


def _batch(rng, sizes, sigma, strain_amp, strain_mask, vac_range, name, seed) -> System:
    pos_all, h_all, starts = [], [], [0]
    shapes = []
    for c, n_target in enumerate(sizes):
        n1, n2, n3 = most_cubic_cells(int(n_target))
        pos, h = bcc_lattice(n1, n2, n3)
        if vac_range is not None:
            f = rng.uniform(*vac_range)
            nv = int(round(f * pos.shape[0]))
            nv = min(nv, pos.shape[0] - 2)
            if nv > 0:
                keep = np.sort(rng.choice(pos.shape[0], size=pos.shape[0] - nv, replace=False))
                pos = pos[keep]
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
        if strain_mask[c]:
            eps = _random_sym_strain(rng, strain_amp)
            F = np.eye(3) + eps
            pos = pos @ F
            h = h @ F
        pos_all.append(pos)
        h_all.append(h)
        starts.append(starts[-1] + pos.shape[0])
        shapes.append((n1, n2, n3))
    pos = np.concatenate(pos_all, axis=0)
    return System(pos=np.ascontiguousarray(pos), vel=np.zeros_like(pos),
                  cell_start=np.array(starts, dtype=np.int64), h=np.stack(h_all),
                  name=name, meta={"seed": seed, "shapes": shapes})


def diffbatch(seed: int = SEEDS["diffbatch"], n_cells: int = 512) -> System:
    """512 periodic cells, sizes U{16..256}, sigma = 0.1 A, random +-3 % strain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(16, 257, size=n_cells)
    return _batch(rng, sizes, 0.1, 0.03, np.ones(n_cells, bool), None, "diffbatch", seed)


def batch(seed: int = SEEDS["batch"], n_cells: int = 4096) -> System:
    """4,096 cells, sizes log-uniform in [8, 512], 1-3 % vacancies, half strained (+-3 %)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(np.log(8.0), np.log(512.0), size=n_cells)).round().astype(int)
    mask = np.zeros(n_cells, bool)
    mask[rng.permutation(n_cells)[: n_cells // 2]] = True
    return _batch(rng, sizes, 0.1, 0.03, mask, (0.01, 0.03), "batch", seed)


def dimer(r: float, box: float = 40.0) -> System:
    """Two atoms separated by r along x in a large periodic box."""
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    return _single(pos, np.eye(3) * box, name="dimer")


WORKLOADS = {"tiny": tiny, "mid": mid, "large": large, "diffbatch": diffbatch, "batch": batch}
