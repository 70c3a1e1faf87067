"""Wigner–Seitz defect analysis, FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the GPU library never calls it and shares
no code with it.

The paper identifies vacancies and interstitials with the Wigner–Seitz cell
method and groups them into clusters (Methods, defect-analysis passage):
every atom belongs to the reference site nearest to it; a site holding no
atom is a vacancy, a site holding k > 1 atoms holds k - 1 interstitials.
Two vacancies are in one cluster when their sites are within the
second-nearest-neighbour distance of the reference lattice, two interstitial
sites when within the third-nearest-neighbour distance (clusters are the
connected components of that relation).

Reference lattice (a reading: the paper analyses bcc W cascades started from
a perfect crystal): the perfect bcc lattice of an orthorhombic periodic box
of n0 x n1 x n2 conventional cells with lattice constants a0, a1, a2.  Site
ids: 2 * ((k * n1 + j) * n0 + i) + b, b = 0 for the corner (i, j, k) a and
b = 1 for the body centre (i + 1/2, j + 1/2, k + 1/2) a.  Nearest sites are
found here by brute force over all sites with minimum-image distances, and
clusters by scipy's connected components on the explicit distance matrix.
"""
from __future__ import annotations

import numpy as np


def reference_sites(a, n):
    """Positions [M, 3] of the reference sites in id order."""
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (3,))
    n0, n1, n2 = (int(v) for v in n)
    sites = np.zeros((2 * n0 * n1 * n2, 3))
    idx = 0
    for k in range(n2):
        for j in range(n1):
            for i in range(n0):
                sites[idx] = (i * a[0], j * a[1], k * a[2])
                sites[idx + 1] = ((i + 0.5) * a[0], (j + 0.5) * a[1], (k + 0.5) * a[2])
                idx += 2
    return sites


def _min_image(d, L):
    return d - L * np.round(d / L)


def nearest_sites(pos, a, n, chunk=256):
    """Index of the nearest reference site of every atom (brute force, minimum image).
    Exact ties go to the lowest site id."""
    sites = reference_sites(a, n)
    L = np.broadcast_to(np.asarray(a, dtype=np.float64), (3,)) * np.asarray(n, dtype=np.float64)
    out = np.empty(pos.shape[0], dtype=np.int64)
    for s in range(0, pos.shape[0], chunk):
        p = pos[s:s + chunk]
        d = _min_image(sites[None, :, :] - p[:, None, :], L)
        out[s:s + chunk] = np.argmin(np.einsum("ijk,ijk->ij", d, d), axis=1)
    return out


def _clusters(site_ids, weights, sites, L, cutoff):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    m = len(site_ids)
    if m == 0:
        return np.zeros(0, dtype=np.int64), []
    p = sites[site_ids]
    d = _min_image(p[:, None, :] - p[None, :, :], L)
    adj = np.einsum("ijk,ijk->ij", d, d) <= cutoff * cutoff * (1.0 + 1e-9)
    ncomp, lab = connected_components(csr_matrix(adj), directed=False)
    sizes = sorted((int(np.sum(weights[lab == c])) for c in range(ncomp)), reverse=True)
    return lab, sizes


def wigner_seitz(pos, a, n):
    """Occupancy of every site, the vacancy and interstitial sites, and the
    cluster sizes (largest first).  a: lattice constant(s), n: cells per axis."""
    a3 = np.broadcast_to(np.asarray(a, dtype=np.float64), (3,))
    sites = reference_sites(a3, n)
    L = a3 * np.asarray(n, dtype=np.float64)
    assign = nearest_sites(np.asarray(pos, dtype=np.float64), a3, n)
    occ = np.bincount(assign, minlength=sites.shape[0])
    vac = np.flatnonzero(occ == 0)
    inter = np.flatnonzero(occ >= 2)
    mult = occ[inter] - 1
    # bcc: second neighbours at a, third at a sqrt(2) (cubic reference)
    a0 = float(a3[0])
    vlab, vsizes = _clusters(vac, np.ones(len(vac), dtype=np.int64), sites, L, a0)
    ilab, isizes = _clusters(inter, mult, sites, L, a0 * np.sqrt(2.0))
    return {"assign": assign, "occupancy": occ, "vacancies": vac, "interstitial_sites": inter,
            "interstitial_mult": mult, "n_vacancies": int(len(vac)), "n_interstitials": int(mult.sum()),
            "vacancy_clusters": vsizes, "interstitial_clusters": isizes,
            "vacancy_labels": vlab, "interstitial_labels": ilab}
