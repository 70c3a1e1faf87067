"""Population evaluation, training loss and SNES generation (test
infrastructure only: the GPU path never imports this).

The paper trains its model with the separable natural evolution strategy
(SNES) of Schaul, Glasmachers and Schmidhuber (2011), population 50
(Sec. III.A), on the NEP loss of the NEP paper it cites, with weights
lambda_1 = lambda_2 = 0.05, lambda_e = lambda_f = 1, lambda_v = 0.1
(Sec. III.A).  That loss is not printed in the paper; the reading here is
the NEP one: root-mean-square errors of the energy per atom, of the force
components and of the six independent virial components per atom (over the
structures that carry a virial target), plus an L1 and an L2 penalty on the
parameters, each averaged over the n parameters:

  L(z) = le RMSE_E + lf RMSE_F + lv RMSE_W + l1 (1/n) sum|z| + l2 sqrt((1/n) sum z^2)

SNES, one generation (Schaul et al. 2011; lower loss is better):
  z_k = mu + sigma * s_k for the given standard-normal draws s_k (k < lambda);
  rank the members by loss (ties keep the member order);
  utilities u_r = max(0, ln(lambda/2 + 1) - ln r) / sum_r' max(...) - 1/lambda
  for rank r = 1..lambda;
  grad_mu = sum_k u_{r(k)} s_k, grad_sigma = sum_k u_{r(k)} (s_k^2 - 1);
  mu += eta_mu sigma * grad_mu; sigma *= exp(eta_sigma / 2 * grad_sigma);
  defaults eta_mu = 1, eta_sigma = (3 + ln n) / (5 sqrt n).
"""
from __future__ import annotations

import numpy as np

LAMBDAS = {"e": 1.0, "f": 1.0, "v": 0.1, "l1": 0.05, "l2": 0.05}   # Sec. III.A
VIRIAL_COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0))


def evaluate_cells(model, system, theta=None):
    """Energy [C], forces [N, 3] and virial [C, 3, 3] of every cell of a batch."""
    from . import efv_cell
    m = model if theta is None else model.with_param_vector(np.asarray(theta, dtype=np.float64))
    C = system.n_cells
    E = np.zeros(C)
    W = np.zeros((C, 3, 3))
    F = np.zeros((system.n_atoms, 3))
    for c in range(C):
        s, e = int(system.cell_start[c]), int(system.cell_start[c + 1])
        r = efv_cell(m, system.pos[s:e], system.h[c], system.pbc)
        E[c] = r["energy"]
        W[c] = r["virial"]
        F[s:e] = r["forces"]
    return E, F, W


def loss_terms(theta, E, F, W, targets, n_atoms_cell, lambdas=LAMBDAS):
    """(total, rmse_e, rmse_f, rmse_v, l1, l2) of one parameter vector.

    targets: dict with "energy" [C], "forces" [N, 3], "virial" [C, 3, 3] and
    "has_virial" [C] bool.  n_atoms_cell [C]."""
    theta = np.asarray(theta, dtype=np.float64)
    n = theta.size
    na = np.asarray(n_atoms_cell, dtype=np.float64)
    rmse_e = np.sqrt(np.mean(((E - targets["energy"]) / na) ** 2))
    rmse_f = np.sqrt(np.mean((F - targets["forces"]) ** 2))
    hv = np.asarray(targets["has_virial"], bool)
    if hv.any():
        d = [(W[hv, a, b] - targets["virial"][hv, a, b]) / na[hv] for a, b in VIRIAL_COMPONENTS]
        rmse_v = np.sqrt(np.mean(np.stack(d) ** 2))
    else:
        rmse_v = 0.0
    l1 = np.sum(np.abs(theta)) / n
    l2 = np.sqrt(np.sum(theta * theta) / n)
    total = (lambdas["e"] * rmse_e + lambdas["f"] * rmse_f + lambdas["v"] * rmse_v + lambdas["l1"] * l1
             + lambdas["l2"] * l2)
    return np.array([total, rmse_e, rmse_f, rmse_v, l1, l2])


def population_losses(model, system, thetas, targets, lambdas=LAMBDAS):
    """Loss terms [P, 6] of every parameter vector of a population."""
    na = np.diff(system.cell_start)
    out = []
    for th in thetas:
        E, F, W = evaluate_cells(model, system, th)
        out.append(loss_terms(th, E, F, W, targets, na, lambdas))
    return np.array(out)


def utilities(lam):
    """Rank-based utilities of SNES for ranks 1..lam (best first); they sum to zero."""
    r = np.arange(1, lam + 1, dtype=np.float64)
    raw = np.maximum(0.0, np.log(lam / 2.0 + 1.0) - np.log(r))
    return raw / raw.sum() - 1.0 / lam


def default_rates(n):
    return 1.0, (3.0 + np.log(n)) / (5.0 * np.sqrt(n))


def sample(mu, sigma, draws):
    """Population z_k = mu + sigma * s_k (draws [lambda, n])."""
    return np.asarray(mu, np.float64)[None, :] + np.asarray(sigma, np.float64)[None, :] * np.asarray(draws, np.float64)


def update(mu, sigma, draws, losses, eta_mu=None, eta_sigma=None):
    """One SNES update from the members' losses; returns (mu, sigma)."""
    s = np.asarray(draws, dtype=np.float64)
    lam, n = s.shape
    em, es = default_rates(n)
    eta_mu = em if eta_mu is None else eta_mu
    eta_sigma = es if eta_sigma is None else eta_sigma
    order = np.argsort(np.asarray(losses, dtype=np.float64), kind="stable")   # best first
    u = np.empty(lam)
    u[order] = utilities(lam)
    g_mu = u @ s
    g_sigma = u @ (s * s - 1.0)
    mu = np.asarray(mu, np.float64) + eta_mu * np.asarray(sigma, np.float64) * g_mu
    sigma = np.asarray(sigma, np.float64) * np.exp(0.5 * eta_sigma * g_sigma)
    return mu, sigma
