"""Pins of the oracle's SNES generation and training loss (Sec. III.A).

SNES is pinned by what the method must do rather than by its formulas: the
utilities sum to zero and favour the best members, the update depends on the
losses only through their ranks, it follows a linear loss downhill, and it
converges on the sphere function (and fails to with any of the planted
mistakes).  The loss is pinned by closed forms (uniform energy and force
offsets, constant parameter vectors) and by a population whose member equals
the model that made the targets.
"""
import os

import numpy as np
import pytest

import nep_synth
from oracle import snes

_SRC = os.path.join(os.path.dirname(snes.__file__), "snes.py")


def _sphere_run(mod, n=10, gens=400, lam=20, seed=3):
    rng = np.random.default_rng(seed)
    mu, sigma = np.full(n, 5.0), np.ones(n)
    for _ in range(gens):
        s = rng.standard_normal((lam, n))
        z = mod.sample(mu, sigma, s)
        mu, sigma = mod.update(mu, sigma, s, np.sum(z * z, axis=1))
    return mu, sigma


def test_utilities_sum_to_zero_and_rank_the_best_first():
    for lam in (2, 4, 5, 50, 51):
        u = snes.utilities(lam)
        assert abs(u.sum()) < 1e-14
        assert np.all(np.diff(u) <= 1e-15)
        assert u[0] > 0 > u[-1]
        # only the better half (ranks below lam/2 + 1) carry positive weight
        assert np.all(u[int(np.floor(lam / 2.0 + 1.0)) - 1:] < 0)


def test_update_depends_on_ranks_only():
    rng = np.random.default_rng(0)
    lam, n = 12, 7
    mu, sigma = rng.normal(size=n), rng.uniform(0.5, 2.0, size=n)
    s = rng.standard_normal((lam, n))
    f = rng.normal(size=lam)
    a = snes.update(mu, sigma, s, f)
    b = snes.update(mu, sigma, s, 3.0 * f + 7.0)      # monotone transform
    p = rng.permutation(lam)
    c = snes.update(mu, sigma, s[p], f[p])            # members in another order
    for x, y in ((a, b), (a, c)):
        assert np.allclose(x[0], y[0], rtol=0, atol=1e-13) and np.allclose(x[1], y[1], rtol=0, atol=1e-13)


def test_update_follows_a_linear_loss_downhill():
    rng = np.random.default_rng(1)
    n, lam = 20, 50
    c = rng.normal(size=n)
    mu, sigma = np.zeros(n), np.ones(n)
    for _ in range(5):
        s = rng.standard_normal((lam, n))
        z = snes.sample(mu, sigma, s)
        mu, sigma = snes.update(mu, sigma, s, z @ c)
    cos = -(mu @ c) / (np.linalg.norm(mu) * np.linalg.norm(c))
    assert cos > 0.9


def test_converges_on_the_sphere():
    mu, sigma = _sphere_run(snes)
    assert np.linalg.norm(mu) < 1e-3
    assert sigma.max() < 1e-3


def test_default_rates():
    em, es = snes.default_rates(100)
    assert em == 1.0 and abs(es - (3.0 + np.log(100.0)) / 50.0) < 1e-15


def _small_batch():
    s = nep_synth.diffbatch(n_cells=6)
    return s


def test_loss_closed_forms():
    s = _small_batch()
    C, N = s.n_cells, s.n_atoms
    na = np.diff(s.cell_start).astype(np.float64)
    rng = np.random.default_rng(2)
    E, F, W = rng.normal(size=C), rng.normal(size=(N, 3)), rng.normal(size=(C, 3, 3))
    tg = {"energy": E.copy(), "forces": F.copy(), "virial": W.copy(), "has_virial": np.ones(C, bool)}
    theta = np.full(50, -0.3)
    t = snes.loss_terms(theta, E, F, W, tg, na)
    assert np.allclose(t[1:4], 0.0, atol=0)
    assert abs(t[4] - 0.3) < 1e-15 and abs(t[5] - 0.3) < 1e-15
    assert abs(t[0] - 0.05 * 0.3 * 2) < 1e-15
    # every cell's energy off by 0.02 eV/atom, every force by (0.1, -0.2, 0.2) eV/A
    t = snes.loss_terms(theta, E + 0.02 * na, F + np.array([0.1, -0.2, 0.2]), W, tg, na)
    assert abs(t[1] - 0.02) < 1e-12
    assert abs(t[2] - np.sqrt((0.01 + 0.04 + 0.04) / 3.0)) < 1e-12
    # a symmetric virial offset of 0.05 eV/atom on xx only: one of six components
    dW = np.zeros((C, 3, 3))
    dW[:, 0, 0] = 0.05 * na
    t = snes.loss_terms(theta, E, F, W + dW, tg, na)
    assert abs(t[3] - 0.05 / np.sqrt(6.0)) < 1e-12
    # cells without a virial target do not count
    tg2 = dict(tg, has_virial=np.arange(C) % 2 == 0)
    dW2 = dW.copy()
    dW2[1::2] *= 100.0
    t2 = snes.loss_terms(theta, E, F, W + dW2, tg2, na)
    assert abs(t2[3] - 0.05 / np.sqrt(6.0)) < 1e-12


def test_population_member_equal_to_the_teacher_has_zero_errors():
    s = _small_batch()
    teacher = nep_synth.random_model(seed=77)
    E, F, W = snes.evaluate_cells(teacher, s)
    tg = {"energy": E, "forces": F, "virial": W, "has_virial": np.ones(s.n_cells, bool)}
    student = nep_synth.random_model()
    th_t = teacher.param_vector()
    th_s = student.param_vector()
    L = snes.population_losses(student, s, [th_s, th_t], tg)
    assert np.all(L[0, 1:4] > 1e-3)
    assert np.all(np.abs(L[1, 1:4]) < 1e-12)
    assert abs(L[1, 4] - np.mean(np.abs(th_t))) < 1e-14


# ------------------------------------------------------------------ planted mistakes

MUTATIONS = {
    "utilities_not_centred": ("return raw / raw.sum() - 1.0 / lam", "return raw / raw.sum()"),
    "rank_worst_first": ('order = np.argsort(np.asarray(losses, dtype=np.float64), kind="stable")',
                         'order = np.argsort(-np.asarray(losses, dtype=np.float64), kind="stable")'),
    "mu_step_without_sigma": ("mu = np.asarray(mu, np.float64) + eta_mu * np.asarray(sigma, np.float64) * g_mu",
                              "mu = np.asarray(mu, np.float64) + eta_mu * g_mu"),
    "sigma_wrong_sign": ("np.exp(0.5 * eta_sigma * g_sigma)", "np.exp(-0.5 * eta_sigma * g_sigma)"),
    "sigma_gradient_first_power": ("g_sigma = u @ (s * s - 1.0)", "g_sigma = u @ (s - 1.0)"),
    "utility_by_member_not_rank": ("u[order] = utilities(lam)", "u[:] = utilities(lam)"),
    "energy_not_per_atom": ("rmse_e = np.sqrt(np.mean(((E - targets[\"energy\"]) / na) ** 2))",
                            "rmse_e = np.sqrt(np.mean((E - targets[\"energy\"]) ** 2))"),
    "virial_all_nine": ("for a, b in VIRIAL_COMPONENTS]", "for a in range(3) for b in range(3)]"),
    "l2_not_rooted": ("l2 = np.sqrt(np.sum(theta * theta) / n)", "l2 = np.sum(theta * theta) / n"),
}


def _mutant(name):
    import importlib.util
    src = open(_SRC).read()
    old, new = MUTATIONS[name]
    assert old in src, name
    spec = importlib.util.spec_from_loader("oracle._snes_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new, 1), f"<snes mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pins_hold(mod):
    try:
        u = mod.utilities(50)
        if abs(u.sum()) > 1e-12 or not u[0] > 0 > u[-1]:
            return False
        mu, sigma = _sphere_run(mod, gens=250)
        if not (np.all(np.isfinite(mu)) and np.linalg.norm(mu) < 1e-2):
            return False
        s = _small_batch()
        na = np.diff(s.cell_start).astype(np.float64)
        rng = np.random.default_rng(2)
        C, N = s.n_cells, s.n_atoms
        E, F, W = rng.normal(size=C), rng.normal(size=(N, 3)), rng.normal(size=(C, 3, 3))
        tg = {"energy": E, "forces": F, "virial": W, "has_virial": np.ones(C, bool)}
        dW = np.zeros((C, 3, 3))
        dW[:, 0, 0] = 0.05 * na
        t = mod.loss_terms(np.full(50, -0.3), E + 0.02 * na, F, W + dW, tg, na)
        return bool(abs(t[1] - 0.02) < 1e-12 and abs(t[3] - 0.05 / np.sqrt(6.0)) < 1e-12
                    and abs(t[5] - 0.3) < 1e-15)
    except (FloatingPointError, OverflowError, ValueError):
        return False


def test_pins_hold_on_the_real_snes():
    assert _pins_hold(snes)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_snes_mistake_is_caught(name):
    with np.errstate(all="ignore"):
        assert not _pins_hold(_mutant(name))
