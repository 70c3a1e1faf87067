"""Pins of the oracle's border thermostat (Nose-Hoover chain, Sec. II.B).

The chain's half step is checked against the continuous thermostat flow
integrated to high accuracy (a symmetric splitting has a local error of third
order), the full integrator against its conserved quantity and its second-order
convergence, and the border selection against lattice counts.
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import nep_synth
import oracle


def _thermostat_flow(n_dof, kT, Q, M):
    # Martyna-Klein-Tuckerman chain acting on the kinetic energy alone:
    # d(2K)/dt = -2 v1 (2K), dv_j/dt = G_j - v_j v_{j+1}, dxi_j/dt = v_j
    def f(t, y):
        twoK, v = y[0], y[1:1 + M]
        d = np.zeros_like(y)
        d[0] = -2.0 * v[0] * twoK
        for j in range(M):
            G = (twoK - n_dof * kT) / Q[0] if j == 0 else (Q[j - 1] * v[j - 1] ** 2 - kT) / Q[j]
            d[1 + j] = G - (v[j] * v[j + 1] if j < M - 1 else 0.0)
        d[1 + M:] = v
        return d
    return f


@pytest.mark.parametrize("M", [1, 2, 3, 5])
def test_chain_half_step_follows_the_thermostat_flow(M):
    errs = []
    for dt in (4.0, 2.0, 1.0):
        ch = oracle.NoseHooverChain(30, 600.0, 10.0, M)
        ch.v[:] = np.linspace(0.02, -0.01, M)
        twoK = 30 * oracle.K_B_EV * 300.0
        y0 = np.concatenate([[twoK], ch.v.copy(), ch.xi.copy()])
        sol = solve_ivp(_thermostat_flow(30, ch.kT, ch.Q, M), (0.0, dt / 2), y0, rtol=1e-13, atol=1e-16,
                        method="DOP853")
        y = sol.y[:, -1]
        s = ch.half_step(twoK, dt)
        errs.append(max(abs(s - np.sqrt(y[0] / twoK)), np.abs(ch.v - y[1:1 + M]).max() * dt,
                        np.abs(ch.xi - y[1 + M:]).max()))
    # local error of a symmetric splitting: O(h^3), so halving dt cuts it about 8x
    for a, b in zip(errs, errs[1:]):
        assert 6.5 < a / b < 9.0
    assert errs[-1] < 2e-4


def test_border_mask_counts_on_the_lattice():
    pos, h = nep_synth.bcc_lattice(4, 4, 4)
    a = nep_synth.A_W
    # x layers at 0, a/2, ..., 3.5a: within 0.6a of a face are 0 and a/2 (corner 1 of 4
    # layers, centre 2 of 4 after the wrap of 3.5a) -> 16 + 32
    assert oracle.border_mask(pos, h, 0.6 * a, (0,)).sum() == 48
    # all axes: corners 64 (1 - (3/4)^3) = 37, centres 64 (1 - (1/2)^3) = 56
    assert oracle.border_mask(pos, h, 0.6 * a, (0, 1, 2)).sum() == 93
    # atoms outside the box are wrapped first
    shifted = pos + np.array([4 * a, -8 * a, 0.0])
    assert np.array_equal(oracle.border_mask(shifted, h, 0.6 * a, (0, 1, 2)),
                          oracle.border_mask(pos, h, 0.6 * a, (0, 1, 2)))


def _run(dt, n_steps, tau=20.0, **kw):
    m = nep_synth.random_model()
    s = nep_synth.mid(n_cells=4)
    return s, oracle.velocity_verlet_nhc(m, s.pos, s.vel * np.sqrt(100.0 / 300.0), s.h[0], s.mass, n_steps,
                                         dt_max=dt, temperature=900.0, tau=tau, chain=3,
                                         thickness=0.6 * nep_synth.A_W, axes=(0,), record=True, **kw)


def test_conserved_quantity_and_second_order():
    drift, work = [], None
    for dt in (1.0, 0.5):
        s, (_, _, _, log, mask, _) = _run(dt, int(round(200 / dt)))
        c = np.array([x["conserved"] for x in log])
        drift.append(np.abs(c - c[0]).max() / s.n_atoms)
        if work is None:
            et = np.array([x["epot"] + x["ekin"] for x in log])
            work = np.abs(et - et[0]).max() / s.n_atoms
    # the thermostat pumps ~0.09 eV/atom into the system; the extended energy stays put
    assert work > 0.05
    assert drift[0] < 1e-4 and drift[0] < 1e-3 * work
    assert 3.0 < drift[0] / drift[1] < 5.5


def test_border_heats_toward_the_target():
    s, (_, _, _, log, mask, ch) = _run(1.0, 300)
    assert mask.sum() == 48 and ch.n_dof == 144
    T = np.array([x["T_border"] for x in log])
    # starts near 100 K; a sign error in the chain forces would cool it instead
    assert T[0] < 150.0
    assert 500.0 < T[150:].mean() < 1400.0


def test_slow_chain_reduces_to_plain_verlet():
    m = nep_synth.random_model()
    s = nep_synth.mid(n_cells=4)
    p0, v0, _, _ = oracle.velocity_verlet(m, s.pos, s.vel, s.h[0], s.mass, 20, dt_max=1.0)
    p1, v1, _, _, _, _ = oracle.velocity_verlet_nhc(m, s.pos, s.vel, s.h[0], s.mass, 20, dt_max=1.0,
                                                    temperature=300.0, tau=1e9, thickness=0.6 * nep_synth.A_W)
    assert np.abs(p1 - p0).max() < 1e-12 and np.abs(v1 - v0).max() < 1e-12


# ------------------------------------------------------------------ planted mistakes

_MD_SRC = os.path.join(os.path.dirname(oracle.__file__), "md.py")

MUTATIONS = {
    "G1_sign": ("return (twoK - self.n_dof * self.kT) / self.Q[0]", "return (self.n_dof * self.kT - twoK) / self.Q[0]"),
    "G_chain_index": ("return (self.Q[j - 1] * self.v[j - 1] ** 2 - self.kT) / self.Q[j]",
                      "return (self.Q[j] * self.v[j] ** 2 - self.kT) / self.Q[j]"),
    "scale_sign": ("s = np.exp(-v[0] * dt / 2.0)", "s = np.exp(v[0] * dt / 2.0)"),
    "twoK_not_rescaled": ("        twoK *= s * s\n", "\n"),
    "xi_full_step": ("self.xi += v * dt / 2.0", "self.xi += v * dt"),
    "inner_factor_dropped": ("        for j in range(M - 1):\n            v[j] *= np.exp(-v[j + 1] * d8)\n",
                             "        for j in range(M - 1):\n"),
    "energy_xi_weight": ("+ self.kT * np.sum(self.xi[1:]))", "+ self.n_dof * self.kT * np.sum(self.xi[1:]))"),
}


def _mutated_md(name):
    import importlib.util
    src = open(_MD_SRC).read()
    old, new = MUTATIONS[name]
    assert old in src, name
    spec = importlib.util.spec_from_loader("oracle._md_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new, 1), f"<md mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pins_hold(md):
    """The fast pins above, run against a module providing the chain and integrator."""
    # flow: third-order local error and small at dt = 1 (M = 3)
    errs = []
    for dt in (2.0, 1.0):
        ch = md.NoseHooverChain(30, 600.0, 10.0, 3)
        ch.v[:] = np.linspace(0.02, -0.01, 3)
        twoK = 30 * oracle.K_B_EV * 300.0
        y0 = np.concatenate([[twoK], ch.v.copy(), ch.xi.copy()])
        y = solve_ivp(_thermostat_flow(30, ch.kT, ch.Q, 3), (0.0, dt / 2), y0, rtol=1e-13, atol=1e-16,
                      method="DOP853").y[:, -1]
        s = ch.half_step(twoK, dt)
        errs.append(max(abs(s - np.sqrt(y[0] / twoK)), np.abs(ch.v - y[1:4]).max() * dt,
                        np.abs(ch.xi - y[4:]).max()))
    if not (6.5 < errs[0] / errs[1] < 9.0 and errs[1] < 2e-4):
        return False
    # conserved quantity and heating over 150 steps
    m = nep_synth.random_model()
    s = nep_synth.mid(n_cells=4)
    _, _, _, log, _, _ = md.velocity_verlet_nhc(m, s.pos, s.vel * np.sqrt(100.0 / 300.0), s.h[0], s.mass, 150,
                                                dt_max=1.0, temperature=900.0, tau=20.0, chain=3,
                                                thickness=0.6 * nep_synth.A_W, axes=(0,), record=True)
    c = np.array([x["conserved"] for x in log])
    T = np.array([x["T_border"] for x in log])
    return bool(np.abs(c - c[0]).max() / s.n_atoms < 1e-4 and T[100:].mean() > 300.0)


def test_pins_hold_on_the_real_thermostat():
    import oracle.md as md
    assert _pins_hold(md)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_thermostat_mistake_is_caught(name):
    assert not _pins_hold(_mutated_md(name))
