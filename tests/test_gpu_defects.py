"""Wigner-Seitz defect analysis on the GPU against the FP64 oracle: integer
results (occupancies, defect sites, multiplicities, cluster sizes) must be
identical; at 8,192,000 atoms sampled atoms and conservation."""
import numpy as np
import pytest

import nep_synth
from oracle import defects as D
from gpu_common import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

A = nep_synth.A_W


def _site(i, j, k, b):
    return np.array([i + 0.5 * b, j + 0.5 * b, k + 0.5 * b]) * A


def _sid(i, j, k, b, n):
    return 2 * ((k * n + j) * n + i) + b


def _cluster_sizes(labels, weights):
    sizes = {}
    for lab, w in zip(labels, weights):
        sizes[lab] = sizes.get(lab, 0) + int(w)
    return sorted(sizes.values(), reverse=True)


def _gpu(pos, n, capacity=4096):
    import paper_2305_08140_amd as nep
    h = np.diag([n[0] * A, n[1] * A, n[2] * A])
    s = nep_synth._single(pos, h)
    sysd = nep.DeviceSystem.from_synth(s)
    return nep.wigner_seitz(sysd, A, n, capacity=capacity, site_of_atom=True)


def _compare(pos, n):
    g = _gpu(pos, n)
    r = D.wigner_seitz(pos, A, n)
    assert np.array_equal(g["occupancy"].cpu().numpy(), r["occupancy"])
    assert np.array_equal(g["site_of_atom"].cpu().numpy(), r["assign"])
    assert np.array_equal(g["vacancy_sites"].cpu().numpy(), r["vacancies"])
    assert np.array_equal(g["interstitial_sites"].cpu().numpy(), r["interstitial_sites"])
    assert np.array_equal(g["interstitial_mult"].cpu().numpy(), r["interstitial_mult"])
    assert g["n_vacancies"] == r["n_vacancies"] and g["n_interstitials"] == r["n_interstitials"]
    vs = _cluster_sizes(g["vacancy_cluster"].cpu().numpy(), np.ones(g["n_vacancies"]))
    isz = _cluster_sizes(g["interstitial_cluster"].cpu().numpy(), g["interstitial_mult"].cpu().numpy())
    assert vs == r["vacancy_clusters"] and isz == r["interstitial_clusters"]
    assert g["n_vacancy_clusters"] == len(vs) and g["n_interstitial_clusters"] == len(isz)
    assert g["largest_vacancy_cluster"] == (vs[0] if vs else 0)
    assert g["largest_interstitial_cluster"] == (isz[0] if isz else 0)
    return g, r


def test_planted_defects_match_oracle():
    n = 8
    pos, _ = nep_synth.bcc_lattice(n, n, n)
    remove = [(1, 1, 1, 0), (1, 1, 1, 1), (4, 4, 4, 0), (5, 4, 4, 0), (1, 5, 1, 0), (2, 6, 1, 0),
              (0, 3, 6, 0), (7, 3, 6, 0)]
    keep = np.setdiff1d(np.arange(pos.shape[0]), [_sid(*s, n) for s in remove])
    extra = [_site(2, 2, 2, 0) + [0.30, 0.20, 0.10], _site(3, 3, 2, 0) + [0.25, -0.15, 0.05],
             _site(6, 6, 6, 1) + [-0.2, 0.3, 0.1], _site(6, 6, 6, 1) + [0.1, -0.3, 0.2],
             _site(5, 6, 6, 0) + [0.1, 0.2, -0.2], _site(2, 6, 5, 0) + [0.2, 0.1, -0.3]]
    pos = np.concatenate([pos[keep], np.array(extra)])
    pos = pos + np.random.default_rng(5).normal(0.0, 0.03, pos.shape)
    pos[:50] += n * A * np.array([1.0, -2.0, 3.0])          # other periodic images
    g, r = _compare(pos, (n, n, n))
    print(f"[defects] vacancies {g['n_vacancies']} clusters {r['vacancy_clusters']}, interstitials "
          f"{g['n_interstitials']} clusters {r['interstitial_clusters']}", flush=True)


def test_random_frenkel_pairs_and_noncubic_cell_counts():
    rng = np.random.default_rng(6)
    n = (7, 5, 6)
    pos, _ = nep_synth.bcc_lattice(*n)
    pos = pos + rng.normal(0.0, 0.08, pos.shape)
    movers = rng.choice(pos.shape[0], size=40, replace=False)
    pos[movers] = rng.uniform(0.0, 1.0, (40, 3)) * np.array(n) * A
    _compare(pos, n)


def test_capacity_is_checked():
    import paper_2305_08140_amd as nep
    n = 6
    pos, _ = nep_synth.bcc_lattice(n, n, n)
    pos = pos[10:]                       # ten vacancies
    with pytest.raises(nep.NepError) as e:
        _gpu(pos, (n, n, n), capacity=4)
    assert e.value.code == nep.NEP_E_CAPACITY


def test_large_cascade_sampled():
    # the 8,192,000-atom cascade start after 200 MD steps: conservation and
    # the site of sampled atoms against a brute-force search of nearby sites
    import torch
    import paper_2305_08140_amd as nep
    from gpu_common import model
    s = nep_synth.large()
    sysd = nep.DeviceSystem.from_synth(s)
    ctx = nep.Context(model(), s.n_atoms, 1)
    out = nep.EFV(s.n_atoms, 1)
    ctx.nep_step_verlet(sysd, 200, out, dt_max=1.0, max_disp=0.015)
    n = (160, 160, 160)
    g = nep.wigner_seitz(sysd, A, n, site_of_atom=True)
    torch.cuda.synchronize()
    occ = g["occupancy"].cpu().numpy()
    M = occ.shape[0]
    assert int(occ.sum()) == s.n_atoms
    assert g["n_vacancies"] - g["n_interstitials"] == M - s.n_atoms
    pos = sysd.positions().cpu().numpy()
    rng = np.random.default_rng(8)
    idx = np.unique(np.concatenate([rng.choice(s.n_atoms, 256, replace=False), [s.meta["pka"]]]))
    # nearest site among the 2 x 27 candidates around each sampled atom (brute force)
    site = g["site_of_atom"].cpu().numpy()[idx]
    for p, sgot in zip(pos[idx], site):
        best, bd = None, np.inf
        c = np.floor(p / A).astype(int)
        for di in range(-1, 2):
            for dj in range(-1, 2):
                for dk in range(-1, 2):
                    for b in (0, 1):
                        q = (c + [di, dj, dk] + 0.5 * b) * A
                        d = q - p
                        dd = float(d @ d)
                        ijk = np.mod(c + [di, dj, dk], 160)
                        sid = 2 * ((ijk[2] * 160 + ijk[1]) * 160 + ijk[0]) + b
                        if dd < bd:
                            best, bd = sid, dd
        assert sgot == best
    print(f"[defects large] vacancies {g['n_vacancies']} interstitials {g['n_interstitials']}", flush=True)


def _tie_points(n):
    """Points exactly equidistant from two or more sites of the bcc lattice
    with a = 4 A (every coordinate and distance exact in binary)."""
    pts = [
        (2.0, 0.0, 0.0),            # corners (0,0,0) / (1,0,0)
        (4.0 * n - 2.0, 0.0, 0.0),  # corners (n-1,0,0) / (0,0,0) across the face
        (2.0, 2.0 + 8.0, 0.0),      # four corners
        (1.0, 1.0, 1.0),            # corner (0,0,0) / body (0,0,0): corner has the lower id
        (3.0, 3.0, 3.0),            # corner (1,1,1) / body (0,0,0): body has the lower id
        (8.0, 6.0, 6.0),            # bodies (1,1,1) / (2,1,1) (x on a corner plane) and corner ties
        (0.0, 6.0, 6.0),            # bodies (n-1,1,1) / (0,1,1) across the face
        (12.0, 2.0, 2.0),           # bodies (2,0,0) / (3,0,0), corners (3,0,0)/(3,1,0)/(3,0,1)/(3,1,1)
    ]
    return np.array(pts, dtype=np.float64)


def test_exact_ties_go_to_the_lowest_site_id():
    import paper_2305_08140_amd as nep
    n = (6, 5, 4)
    a = 4.0
    pos = _tie_points(n[0])
    h = np.diag([n[0] * a, n[1] * a, n[2] * a])
    s = nep_synth._single(pos, h)
    g = nep.wigner_seitz(nep.DeviceSystem.from_synth(s), a, n, capacity=4096, site_of_atom=True)
    r = D.wigner_seitz(pos, a, n)
    got = g["site_of_atom"].cpu().numpy()
    print("[ws ties] gpu", got.tolist(), "oracle", r["assign"].tolist(), flush=True)
    assert np.array_equal(got, r["assign"])
    assert np.array_equal(g["occupancy"].cpu().numpy(), r["occupancy"])
