"""Plain velocity-Verlet integration on top of the FP64 oracle (test infrastructure only).

Time step rule (Sec. II.B): at the start of each step the step length is
dt = min(dt_max, d_max / max_i |v_i|), so that the fastest atom moves at most
d_max in one step; ``d_max = 0`` means a fixed dt = dt_max.

Border thermostat (Sec. II.B): atoms within a given thickness (the paper uses
3 a0) of the faces of the box along chosen axes are kept at a temperature by
a Nose-Hoover chain (the paper cites Martyna, Klein and Tuckerman 1992).
Reading: the chain acts on those atoms only, with N_f = 3 N_border degrees of
freedom, masses Q_1 = N_f kT tau^2 and Q_j = kT tau^2 (j > 1); each step is
the usual Trotter factorisation: a half step of the chain (which scales the
border velocities by exp(-v_xi1 dt/2)), the velocity-Verlet step, another
half step of the chain.  The border set is fixed at the start of a run from
the wrapped positions.

Units: A, fs, u, eV.  An acceleration F/m in eV/(u*A) is converted to A/fs^2
with the factor e / u * 1e-10 (CODATA 2018 e and u).
"""
from __future__ import annotations

import numpy as np

K_B_EV = 8.617333262e-5        # Boltzmann constant, eV/K (CODATA 2018)
_E_C = 1.602176634e-19
_AMU = 1.66053906660e-27
EV_PER_U_TO_A2_PER_FS2 = _E_C / _AMU * 1e-10   # (eV/u) -> (A/fs)^2, also eV/(u A) -> A/fs^2


def kinetic_energy(vel, mass):
    return 0.5 * mass * float(np.sum(vel * vel)) / EV_PER_U_TO_A2_PER_FS2


def velocity_verlet(model, pos, vel, h, mass, n_steps, dt_max=1.0, d_max=0.0, pbc=(1, 1, 1),
                    forces0=None, record=False):
    """Advance (pos, vel) by ``n_steps`` velocity-Verlet steps; returns (pos, vel, forces, log).

    Each step: choose dt from the velocities at the step start, half kick,
    drift, new forces, half kick.  Neighbours are found afresh at every force
    evaluation (no skin), which is the plain definition.
    """
    from . import efv_cell
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    if forces0 is None:
        r = efv_cell(model, pos, h, pbc)
        F, E = r["forces"], r["energy"]
    else:
        F, E = forces0, None
    log = []
    c = EV_PER_U_TO_A2_PER_FS2 / mass
    for _ in range(n_steps):
        vmax = float(np.sqrt(np.max(np.sum(vel * vel, axis=1))))
        dt = dt_max
        if d_max > 0.0 and vmax > 0.0:
            dt = min(dt_max, d_max / vmax)
        vel += 0.5 * dt * c * F
        pos += dt * vel
        r = efv_cell(model, pos, h, pbc)
        F, E = r["forces"], r["energy"]
        vel += 0.5 * dt * c * F
        if record:
            log.append({"dt": dt, "epot": E, "ekin": kinetic_energy(vel, mass)})
    return pos, vel, F, log


def border_mask(pos, h, thickness, axes):
    """Atoms whose wrapped coordinate along any axis in `axes` lies within
    `thickness` of a face of the orthorhombic box h."""
    L = np.diag(np.asarray(h, dtype=np.float64))
    m = np.zeros(pos.shape[0], bool)
    for a in axes:
        s = np.mod(pos[:, a], L[a])
        m |= (s < thickness) | (s >= L[a] - thickness)
    return m


class NoseHooverChain:
    """Chain of M thermostats (positions xi, velocities v in 1/fs) at temperature T."""

    def __init__(self, n_dof, temperature, tau, M=3):
        self.M = M
        self.kT = K_B_EV * temperature
        self.n_dof = n_dof
        self.Q = np.array([n_dof * self.kT * tau * tau] + [self.kT * tau * tau] * (M - 1))
        self.xi = np.zeros(M)
        self.v = np.zeros(M)

    def _G(self, j, twoK):
        if j == 0:
            return (twoK - self.n_dof * self.kT) / self.Q[0]
        return (self.Q[j - 1] * self.v[j - 1] ** 2 - self.kT) / self.Q[j]

    def half_step(self, twoK, dt):
        """Advance the chain by dt/2 for a system with kinetic energy twoK/2 (eV);
        returns the factor that scales the thermostatted velocities."""
        M, v = self.M, self.v
        d4, d8 = dt / 4.0, dt / 8.0
        v[M - 1] += self._G(M - 1, twoK) * d4
        for j in range(M - 2, -1, -1):
            v[j] *= np.exp(-v[j + 1] * d8)
            v[j] += self._G(j, twoK) * d4
            v[j] *= np.exp(-v[j + 1] * d8)
        s = np.exp(-v[0] * dt / 2.0)
        twoK *= s * s
        self.xi += v * dt / 2.0
        for j in range(M - 1):
            v[j] *= np.exp(-v[j + 1] * d8)
            v[j] += self._G(j, twoK) * d4
            v[j] *= np.exp(-v[j + 1] * d8)
        v[M - 1] += self._G(M - 1, twoK) * d4
        return s

    def energy(self):
        """Thermostat contribution to the conserved quantity (eV)."""
        return float(0.5 * np.sum(self.Q * self.v ** 2) + self.n_dof * self.kT * self.xi[0]
                     + self.kT * np.sum(self.xi[1:]))


def velocity_verlet_nhc(model, pos, vel, h, mass, n_steps, dt_max=1.0, d_max=0.0, pbc=(1, 1, 1),
                        temperature=300.0, tau=100.0, chain=3, thickness=0.0, axes=(0, 1, 2), record=False):
    """Velocity Verlet with a Nose-Hoover chain on the border atoms; returns
    (pos, vel, forces, log, mask, chain).  log entries hold the conserved
    quantity epot + ekin + thermostat energy."""
    from . import efv_cell
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    mask = border_mask(pos, h, thickness, axes)
    nhc = NoseHooverChain(3 * int(mask.sum()), temperature, tau, chain)
    r = efv_cell(model, pos, h, pbc)
    F, E = r["forces"], r["energy"]
    c = EV_PER_U_TO_A2_PER_FS2 / mass
    log = []
    for _ in range(n_steps):
        vmax = float(np.sqrt(np.max(np.sum(vel * vel, axis=1))))
        dt = dt_max
        if d_max > 0.0 and vmax > 0.0:
            dt = min(dt_max, d_max / vmax)
        twoK = mass * float(np.sum(vel[mask] ** 2)) / EV_PER_U_TO_A2_PER_FS2
        vel[mask] *= nhc.half_step(twoK, dt)
        vel += 0.5 * dt * c * F
        pos += dt * vel
        r = efv_cell(model, pos, h, pbc)
        F, E = r["forces"], r["energy"]
        vel += 0.5 * dt * c * F
        twoK = mass * float(np.sum(vel[mask] ** 2)) / EV_PER_U_TO_A2_PER_FS2
        vel[mask] *= nhc.half_step(twoK, dt)
        if record:
            ek = kinetic_energy(vel, mass)
            log.append({"dt": dt, "epot": E, "ekin": ek, "conserved": E + ek + nhc.energy(),
                        "T_border": 2.0 * 0.5 * mass * float(np.sum(vel[mask] ** 2)) / EV_PER_U_TO_A2_PER_FS2
                        / (nhc.n_dof * K_B_EV)})
    return pos, vel, F, log, mask, nhc
