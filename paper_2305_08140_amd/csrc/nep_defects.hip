// Wigner–Seitz defect analysis against the perfect bcc lattice of an
// orthorhombic periodic box (the paper's defect identification and
// clustering, Methods): every atom belongs to the nearest lattice site, a
// site holding no atom is a vacancy, a site holding k > 1 atoms holds k - 1
// interstitials; vacancy sites within the second-neighbour distance a and
// interstitial sites within the third-neighbour distance a sqrt(2) form
// clusters (connected components).
//
// Site ids: 2 ((k n1 + j) n0 + i) + b, b = 0 for the corner (i, j, k) a,
// b = 1 for the body centre (i + 1/2, j + 1/2, k + 1/2) a.  The nearest site
// of a point is the nearer of its nearest corner (coordinates rounded) and
// its nearest body centre (coordinates floored, plus one half): each
// sublattice is simple cubic.  Exact ties go to the lowest site id: along an
// axis where a coordinate lies exactly halfway between two sites of a
// sublattice the lower (wrapped) index is taken (the id grows with each
// index), and between equidistant corner and body sites the lower id.
#include "nep_device.h"

namespace nep {

__device__ inline int wrap_index(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

__device__ inline void site_position(int id, const BccRef &r, double p[3])
{
    const int b = id & 1, c = id >> 1;
    const int i = c % r.n[0], j = (c / r.n[0]) % r.n[1], k = c / (r.n[0] * r.n[1]);
    p[0] = (i + 0.5 * b) * r.a;
    p[1] = (j + 0.5 * b) * r.a;
    p[2] = (k + 0.5 * b) * r.a;
}

__device__ inline double site_dist2(int s, int t, const BccRef &r)
{
    double p[3], q[3];
    site_position(s, r, p);
    site_position(t, r, q);
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double L = r.n[a] * r.a;
        double d = p[a] - q[a];
        d -= L * rint(d / L);
        d2 += d * d;
    }
    return d2;
}

__global__ void k_ws_fill(int m, int32_t *__restrict__ a, int32_t v)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) a[t] = v;
}

// occupancy[site] += 1 for the site of every atom; site_of[i] (optional).
// A non-finite position sets bad[0].
__global__ void k_ws_assign(int n_atoms, const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, BccRef r, int32_t *__restrict__ occ,
                            int32_t *__restrict__ site_of, int32_t *__restrict__ bad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_atoms) return;
    const double pos[3] = {x[t], y[t], z[t]};
    // non-finite, or so far out that lattice indices would not fit an int
    const double lim = 1.0e8 * r.a;
    if (!(fabs(pos[0]) < lim && fabs(pos[1]) < lim && fabs(pos[2]) < lim)) {
        atomicOr(bad, 1);
        return;
    }
    int ci[3], bi[3];
    double dc2 = 0.0, db2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = pos[a] * r.inv_a;            // lattice units, not wrapped
        const double fl = floor(s), f = s - fl;
        // nearest corner: fl or fl + 1 (both when f is exactly 1/2)
        const double c = f < 0.5 ? fl : fl + 1.0;
        const double dc = (s - c) * r.a, db = (f - 0.5) * r.a;
        dc2 += dc * dc;
        db2 += db * db;
        const int c0 = wrap_index((int)fl, r.n[a]), c1 = wrap_index((int)fl + 1, r.n[a]);
        ci[a] = f == 0.5 ? min(c0, c1) : (f < 0.5 ? c0 : c1);
        // nearest body centre: fl + 1/2, or also fl - 1/2 when s is an integer
        const int b1 = wrap_index((int)fl - 1, r.n[a]);
        bi[a] = f == 0.0 ? min(c0, b1) : c0;
    }
    const int cid = 2 * ((ci[2] * r.n[1] + ci[1]) * r.n[0] + ci[0]);
    const int bid = 2 * ((bi[2] * r.n[1] + bi[1]) * r.n[0] + bi[0]) + 1;
    const int site = dc2 < db2 ? cid : (db2 < dc2 ? bid : min(cid, bid));
    atomicAdd(&occ[site], 1);
    if (site_of) site_of[t] = site;
}

// Vacancy sites (occupancy 0) and interstitial sites (occupancy > 1), in
// arbitrary order, into vac_tmp / int_tmp (at most cap each); cnt[0] and
// cnt[1] count them, cnt[2] the interstitial atoms.
__global__ void k_ws_collect(int m, const int32_t *__restrict__ occ, int cap, int32_t *__restrict__ vac_tmp,
                             int32_t *__restrict__ int_tmp, int32_t *__restrict__ cnt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    const int o = occ[s];
    if (o == 0) {
        const int k = atomicAdd(&cnt[0], 1);
        if (k < cap) vac_tmp[k] = s;
    } else if (o > 1) {
        const int k = atomicAdd(&cnt[1], 1);
        atomicAdd(&cnt[2], o - 1);
        if (k < cap) int_tmp[k] = s;
    }
}

// Sorted by site id: out[rank(d)] = in[d] (site ids are distinct), and the
// multiplicity occupancy - 1 alongside (mult may be null).
__global__ void k_ws_sort(int d_n, const int32_t *__restrict__ in, int32_t *__restrict__ out,
                          const int32_t *__restrict__ occ, int32_t *__restrict__ mult)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= d_n) return;
    const int s = in[d];
    int rank = 0;
    for (int e = 0; e < d_n; ++e) rank += in[e] < s;
    out[rank] = s;
    if (mult) mult[rank] = occ[s] - 1;
}

__global__ void k_ws_label_init(int d_n, int32_t *__restrict__ label)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < d_n) label[d] = d;
}

// One round of minimum-label propagation over the pairs within the cutoff,
// then one pointer jump; sets *changed when a label decreased.  Labels only
// decrease and stay inside the component, so repeated rounds reach the
// smallest index of every component.
__global__ void k_ws_label_step(int d_n, const int32_t *__restrict__ sites, double cut2, BccRef r,
                                int32_t *__restrict__ label, int32_t *__restrict__ changed)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= d_n) return;
    int m = label[d];
    const int s = sites[d];
    for (int e = 0; e < d_n; ++e) {
        if (e == d) continue;
        const int le = label[e];
        if (le < m && site_dist2(s, sites[e], r) <= cut2) m = le;
    }
    m = min(m, label[m]);
    if (m < label[d]) {
        atomicMin(&label[d], m);
        atomicOr(changed, 1);
    }
}

// Cluster count and largest cluster (weights: interstitial multiplicities,
// or 1 when w is null): out[0] += clusters, out[1] = max size.
__global__ void k_ws_cluster_sizes(int d_n, const int32_t *__restrict__ label, const int32_t *__restrict__ w,
                                   int32_t *__restrict__ out)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= d_n || label[d] != d) return;
    int size = 0;
    for (int e = 0; e < d_n; ++e)
        if (label[e] == d) size += w ? w[e] : 1;
    atomicAdd(&out[0], 1);
    atomicMax(&out[1], size);
}

}  // namespace nep
