"""Plain velocity-Verlet integration on top of the FP64 oracle (test infrastructure only).

Time step rule (Sec. II.B): at the start of each step the step length is
dt = min(dt_max, d_max / max_i |v_i|), so that the fastest atom moves at most
d_max in one step; ``d_max = 0`` means a fixed dt = dt_max.

Units: A, fs, u, eV.  An acceleration F/m in eV/(u*A) is converted to A/fs^2
with the factor e / u * 1e-10 (CODATA 2018 e and u).
"""
from __future__ import annotations

import numpy as np

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
