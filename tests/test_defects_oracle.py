"""Pins of the Wigner–Seitz defect oracle (CPU): a library routine for the
nearest-site step, planted defects at known neighbour shells, conservation."""
import numpy as np
from scipy.spatial import cKDTree

import nep_synth
from oracle import defects as D

A = nep_synth.A_W


def _site(i, j, k, b):
    return np.array([i + 0.5 * b, j + 0.5 * b, k + 0.5 * b]) * A


def _sid(i, j, k, b, n):
    return 2 * ((k * n + j) * n + i) + b


def test_perfect_lattice_has_no_defects():
    pos, _ = nep_synth.bcc_lattice(6, 6, 6)
    pos = pos + np.random.default_rng(0).normal(0.0, 0.05, pos.shape)
    r = D.wigner_seitz(pos, A, (6, 6, 6))
    assert r["n_vacancies"] == 0 and r["n_interstitials"] == 0
    assert np.all(r["occupancy"] == 1)
    # the atom order of bcc_lattice is the site-id order
    assert np.array_equal(r["assign"], np.arange(pos.shape[0]))


def test_nearest_site_matches_periodic_kdtree():
    n = 5
    rng = np.random.default_rng(1)
    pos = rng.uniform(-3.0, n * A + 3.0, size=(3000, 3))      # some outside the box
    got = D.nearest_sites(pos, A, (n, n, n))
    L = n * A
    tree = cKDTree(D.reference_sites(A, (n, n, n)), boxsize=L)
    dist, ref = tree.query(np.mod(pos, L))
    sites = D.reference_sites(A, (n, n, n))
    d = sites[got] - pos
    d -= L * np.round(d / L)
    assert np.allclose(np.sqrt((d * d).sum(1)), dist, atol=1e-12)
    assert np.mean(got == ref) > 0.999            # differences only at numerical ties


def test_vacancy_clusters_by_second_neighbour_distance():
    n = 8
    pos, _ = nep_synth.bcc_lattice(n, n, n)
    remove = [(1, 1, 1, 0), (1, 1, 1, 1),      # first neighbours: one cluster of 2
              (4, 4, 4, 0), (5, 4, 4, 0),      # second neighbours (a): one cluster of 2
              (1, 5, 1, 0), (2, 6, 1, 0),      # third neighbours (a sqrt 2): two clusters
              (0, 3, 6, 0), (7, 3, 6, 0)]      # second neighbours across the boundary
    ids = [_sid(*s, n) for s in remove]
    keep = np.setdiff1d(np.arange(pos.shape[0]), ids)
    pos = pos[keep] + np.random.default_rng(2).normal(0.0, 0.03, (len(keep), 3))
    r = D.wigner_seitz(pos, A, (n, n, n))
    assert sorted(r["vacancies"].tolist()) == sorted(ids)
    assert r["n_interstitials"] == 0
    assert r["vacancy_clusters"] == [2, 2, 2, 1, 1]


def test_interstitial_clusters_by_third_neighbour_distance():
    n = 8
    pos, _ = nep_synth.bcc_lattice(n, n, n)
    extra = [_site(2, 2, 2, 0) + [0.30, 0.20, 0.10],    # two sites at a sqrt 2: one cluster
             _site(3, 3, 2, 0) + [0.25, -0.15, 0.05],
             _site(6, 6, 6, 1) + [-0.2, 0.3, 0.1],       # a site at 4th-neighbour distance: separate
             _site(6, 6, 6, 1) + [0.1, -0.3, 0.2],       # ... holding two extra atoms
             _site(2, 6, 5, 0) + [0.2, 0.1, -0.3]]       # isolated
    p4 = _site(6, 6, 6, 1)
    p_far = _site(5, 6, 6, 0)
    d = p4 - p_far
    assert abs(np.linalg.norm(d) - A * np.sqrt(11) / 2) < 1e-12
    extra.append(p_far + [0.1, 0.2, -0.2])
    pos = np.concatenate([pos, np.array(extra)])
    r = D.wigner_seitz(pos, A, (n, n, n))
    assert r["n_vacancies"] == 0
    assert r["n_interstitials"] == 6
    assert r["interstitial_clusters"] == [2, 2, 1, 1]
    assert int(r["occupancy"][_sid(6, 6, 6, 1, n)]) == 3


def test_frenkel_pairs_conserve_atoms():
    n = 6
    pos, _ = nep_synth.bcc_lattice(n, n, n)
    rng = np.random.default_rng(3)
    movers = rng.choice(pos.shape[0], size=7, replace=False)
    pos = pos + rng.normal(0.0, 0.04, pos.shape)
    pos[movers] = rng.uniform(0, n * A, size=(7, 3))
    r = D.wigner_seitz(pos, A, (n, n, n))
    M = 2 * n ** 3
    assert int(r["occupancy"].sum()) == pos.shape[0]
    assert r["n_vacancies"] - r["n_interstitials"] == M - pos.shape[0]
    assert 0 < r["n_vacancies"] <= 7


def test_exact_ties_go_to_the_lowest_site_id():
    # with a = 4 A every distance below is exact; the expected sites are the
    # lowest ids among the equidistant ones, listed by hand
    n = (6, 5, 4)
    a = 4.0

    def sid(i, j, k, b):
        return 2 * ((k * n[1] + j) * n[0] + i) + b

    cases = [
        ((2.0, 0.0, 0.0), sid(0, 0, 0, 0)),
        ((4.0 * n[0] - 2.0, 0.0, 0.0), sid(0, 0, 0, 0)),
        ((1.0, 1.0, 1.0), sid(0, 0, 0, 0)),
        ((3.0, 3.0, 3.0), sid(0, 0, 0, 1)),
        ((8.0, 6.0, 6.0), sid(1, 1, 1, 1)),
        ((0.0, 6.0, 6.0), sid(0, 1, 1, 1)),
    ]
    pos = np.array([p for p, _ in cases])
    got = D.nearest_sites(pos, a, n)
    assert got.tolist() == [w for _, w in cases]
