/*
 * FP64 CPU oracle for the NEP-ZBL potential: site energies, forces, virial.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may call this code;
 * it exists so that tests, the smoke check and the CPU baseline of the
 * benchmark can compare the GPU library against a plain, slow, obviously
 * correct statement of the method.  It shares no code with the GPU library.
 *
 * What it computes (paper: Sec. II.A, Eqs. 1-4; the NEP descriptor and
 * network follow the NEP framework that Sec. II.A and Sec. III.A cite):
 *
 *   pair sets   P_rc(i) = {(j, n) : n in Z^3 on periodic axes, (j,n) != (i,0),
 *                          |x_j + n.h - x_i| < rc}          (every image counts)
 *   cutoff      fc(r) = (1 + cos(pi r / rc)) / 2 for r < rc, else 0
 *   basis       f_k(r) = (T_k(x) + 1) fc(r) / 2,  x = 2 (r/rc - 1)^2 - 1
 *   radial fns  g_n(r) = sum_k c_nk f_k(r)
 *   radial q    q_n = sum_{P_rcR(i)} g^R_n(r_ij)
 *   angular q   q_nl = sum_{j in P_rcA(i)} sum_{k in P_rcA(i)} g^A_n(r_ij) g^A_n(r_ik) P_l(cos theta_ijk)
 *               (l = 1..l_max, the j = k terms included)
 *   network     U^NEP_i = sum_mu w1_mu tanh(sum_nu w0_mu,nu s_nu q_nu - b0_mu) - b1
 *   ZBL (Eq.2)  U_ZBL(r) = k_e Z^2 / r * phi(r/a) * f_T(r), phi from Eq. 3, a from Eq. 4,
 *               f_T the Tersoff switch between r1 and r2
 *   energy      U_i = U^NEP_i + 1/2 sum_{P_r2(i)} U_ZBL(r_ij)           (Eq. 1)
 *   forces      F_i = -dE/dx_i = sum_j [dU_i/dr_ij - dU_j/dr_ji],  r_ij = x_j + n.h - x_i
 *   virial      W_ab = -sum_i sum_j (dU_i/dr_ij)_a (r_ij)_b   (= -dE/d(strain) at zero strain)
 *
 * The angular derivative is taken through cos(theta_ijk) in the double sum,
 * never through spherical harmonics.  Everything is double precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* Coulomb constant e^2 / (4 pi eps0) in eV*A, computed from CODATA 2018
 * exact/recommended values: e = 1.602176634e-19 C, eps0 = 8.8541878128e-12 F/m. */
static double orc_coulomb_ev_a(void)
{
    const double e = 1.602176634e-19;
    const double eps0 = 8.8541878128e-12;
    /* e^2/(4 pi eps0) in J*m, divide by e (J -> eV) and multiply by 1e10 (m -> A) */
    return e / (4.0 * ORC_PI * eps0) * 1e10;
}

typedef struct {
    int32_t n_rad;      /* radial descriptor components, n = 0..n_rad-1 */
    int32_t n_ang;      /* angular radial functions, n = 0..n_ang-1 */
    int32_t k_rad;      /* Chebyshev basis size for the radial functions */
    int32_t k_ang;      /* Chebyshev basis size for the angular radial functions */
    int32_t l_max;      /* Legendre orders l = 1..l_max */
    int32_t n_hidden;   /* hidden tanh neurons */
    double rc_rad, rc_ang;   /* cutoffs, A */
    double zbl_r1, zbl_r2;   /* Tersoff switch of the ZBL term, A */
    double Z;                /* nuclear charge (single species) */
    const double *c_rad;     /* [n_rad][k_rad] */
    const double *c_ang;     /* [n_ang][k_ang] */
    const double *q_scale;   /* [D] */
    const double *w0;        /* [n_hidden][D] */
    const double *b0;        /* [n_hidden] */
    const double *w1;        /* [n_hidden] */
    double b1;
} orc_model;

static int orc_dim(const orc_model *m) { return m->n_rad + m->n_ang * m->l_max; }

/* ------------------------------------------------------------------ */
/* one-dimensional building blocks                                     */
/* ------------------------------------------------------------------ */

/* Smooth descriptor cutoff and its derivative. */
static void orc_fc(double r, double rc, double *f, double *df)
{
    if (r >= rc) { *f = 0.0; *df = 0.0; return; }
    *f = 0.5 * (1.0 + cos(ORC_PI * r / rc));
    *df = -0.5 * ORC_PI / rc * sin(ORC_PI * r / rc);
}

/* Chebyshev polynomials of the first kind T_0..T_{K-1} at x and dT/dx,
 * from the three-term recurrence T_{k+1} = 2x T_k - T_{k-1}. */
void orc_chebyshev(int K, double x, double *T, double *dT)
{
    for (int k = 0; k < K; ++k) {
        if (k == 0) { T[0] = 1.0; dT[0] = 0.0; }
        else if (k == 1) { T[1] = x; dT[1] = 1.0; }
        else {
            T[k] = 2.0 * x * T[k - 1] - T[k - 2];
            dT[k] = 2.0 * T[k - 1] + 2.0 * x * dT[k - 1] - dT[k - 2];
        }
    }
}

/* Basis f_k(r) = (T_k(x)+1) fc(r) / 2 with x = 2(r/rc-1)^2 - 1, and df_k/dr. */
void orc_basis(int K, double r, double rc, double *f, double *df)
{
    double T[64], dT[64], fc, dfc;
    orc_fc(r, rc, &fc, &dfc);
    double t = r / rc - 1.0;
    double x = 2.0 * t * t - 1.0;
    double dxdr = 4.0 * t / rc;
    orc_chebyshev(K, x, T, dT);
    for (int k = 0; k < K; ++k) {
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        df[k] = 0.5 * dT[k] * dxdr * fc + 0.5 * (T[k] + 1.0) * dfc;
    }
}

/* g_n(r) = sum_k c[n][k] f_k(r) and its derivative, n = 0..N-1. */
static void orc_radial_fns(int N, int K, const double *c, double r, double rc, double *g, double *dg)
{
    double f[64], df[64];
    orc_basis(K, r, rc, f, df);
    for (int n = 0; n < N; ++n) {
        double s = 0.0, ds = 0.0;
        for (int k = 0; k < K; ++k) { s += c[n * K + k] * f[k]; ds += c[n * K + k] * df[k]; }
        g[n] = s; dg[n] = ds;
    }
}

/* Legendre polynomials P_l(c) and dP_l/dc for l = 0..4, explicit forms. */
void orc_legendre(double c, double *P, double *dP)
{
    P[0] = 1.0;                                  dP[0] = 0.0;
    P[1] = c;                                    dP[1] = 1.0;
    P[2] = 0.5 * (3.0 * c * c - 1.0);            dP[2] = 3.0 * c;
    P[3] = 0.5 * (5.0 * c * c * c - 3.0 * c);    dP[3] = 0.5 * (15.0 * c * c - 3.0);
    P[4] = (35.0 * c * c * c * c - 30.0 * c * c + 3.0) / 8.0;
    dP[4] = (140.0 * c * c * c - 60.0 * c) / 8.0;
}

/* Tersoff switch: 1 below r1, (1 + cos(pi (r-r1)/(r2-r1)))/2 between, 0 above r2. */
void orc_tersoff_fc(double r, double r1, double r2, double *f, double *df)
{
    if (r < r1) { *f = 1.0; *df = 0.0; return; }
    if (r > r2) { *f = 0.0; *df = 0.0; return; }
    double w = ORC_PI / (r2 - r1);
    *f = 0.5 * (1.0 + cos(w * (r - r1)));
    *df = -0.5 * w * sin(w * (r - r1));
}

/* ZBL-like W-W repulsion, Eqs. 2-4, and dU/dr. */
void orc_zbl(double r, double Zi, double Zj, double r1, double r2, double *U, double *dU)
{
    /* screening function of Eq. 3 */
    static const double cphi[3] = {0.32825, 0.09219, 0.58110};
    static const double ephi[3] = {2.54931, 0.29182, 0.59231};
    if (r >= r2) { *U = 0.0; *dU = 0.0; return; }
    double a = 0.46848 / (pow(Zi, 0.23) + pow(Zj, 0.23));     /* Eq. 4 */
    double x = r / a;
    double phi = 0.0, dphi = 0.0;
    for (int q = 0; q < 3; ++q) {
        double t = cphi[q] * exp(-ephi[q] * x);
        phi += t;
        dphi += -ephi[q] / a * t;                 /* d phi / d r */
    }
    double ft, dft;
    orc_tersoff_fc(r, r1, r2, &ft, &dft);
    double k = orc_coulomb_ev_a() * Zi * Zj;
    *U = k / r * phi * ft;
    *dU = k * (-phi * ft / (r * r) + dphi * ft / r + phi * dft / r);
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static void orc_inv3(const double *h, double *hi)
{
    /* rows of h are lattice vectors; x = s h  =>  s = x hi with hi = h^-1 */
    double a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], k = h[7], l = h[8];
    double det = a * (e * l - f * k) - b * (d * l - f * g) + c * (d * k - e * g);
    hi[0] = (e * l - f * k) / det; hi[1] = (c * k - b * l) / det; hi[2] = (b * f - c * e) / det;
    hi[3] = (f * g - d * l) / det; hi[4] = (a * l - c * g) / det; hi[5] = (c * d - a * f) / det;
    hi[6] = (d * k - e * g) / det; hi[7] = (b * g - a * k) / det; hi[8] = (a * e - b * d) / det;
}

/* perpendicular widths of the cell (distance between opposite faces) */
static void orc_widths(const double *h, double *w)
{
    double hi[9];
    orc_inv3(h, hi);
    /* the columns of hi are the reciprocal vectors; width_a = 1/|column a| */
    for (int a = 0; a < 3; ++a) {
        double s = hi[0 * 3 + a] * hi[0 * 3 + a] + hi[1 * 3 + a] * hi[1 * 3 + a] + hi[2 * 3 + a] * hi[2 * 3 + a];
        w[a] = 1.0 / sqrt(s);
    }
}

typedef struct {
    int64_t j;
    int32_t n[3];
    double d[3];   /* r_ij = x_j + n.h - x_i */
    double r;
} orc_pair;

typedef struct {
    int64_t count, cap;
    orc_pair *p;
} orc_plist;

static void orc_plist_push(orc_plist *L, const orc_pair *q)
{
    if (L->count == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->p = (orc_pair *)realloc(L->p, (size_t)L->cap * sizeof(orc_pair));
    }
    L->p[L->count++] = *q;
}

/* All (j, n) within rc of atom i by explicit enumeration of every image:
 * for each j, n_a ranges over the integers with |s_j - s_i + n_a| < rc / width_a. */
static void orc_pairs_brute(int64_t N, const double *x, const double *h, const double *hi,
                            const double *wid, const int32_t *pbc, int64_t i, double rc, orc_plist *L)
{
    double si[3];
    for (int a = 0; a < 3; ++a) si[a] = x[3 * i] * hi[a] + x[3 * i + 1] * hi[3 + a] + x[3 * i + 2] * hi[6 + a];
    for (int64_t j = 0; j < N; ++j) {
        double sj[3], lo[3], hi_[3];
        int32_t nlo[3], nhi[3];
        for (int a = 0; a < 3; ++a) {
            sj[a] = x[3 * j] * hi[a] + x[3 * j + 1] * hi[3 + a] + x[3 * j + 2] * hi[6 + a];
            if (pbc[a]) {
                double ds = sj[a] - si[a];
                lo[a] = -ds - rc / wid[a];
                hi_[a] = -ds + rc / wid[a];
                nlo[a] = (int32_t)ceil(lo[a]);
                nhi[a] = (int32_t)floor(hi_[a]);
            } else { nlo[a] = 0; nhi[a] = 0; }
        }
        for (int32_t n0 = nlo[0]; n0 <= nhi[0]; ++n0)
            for (int32_t n1 = nlo[1]; n1 <= nhi[1]; ++n1)
                for (int32_t n2 = nlo[2]; n2 <= nhi[2]; ++n2) {
                    if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                    orc_pair q;
                    q.j = j; q.n[0] = n0; q.n[1] = n1; q.n[2] = n2;
                    for (int b = 0; b < 3; ++b)
                        q.d[b] = x[3 * j + b] + n0 * h[b] + n1 * h[3 + b] + n2 * h[6 + b] - x[3 * i + b];
                    q.r = sqrt(q.d[0] * q.d[0] + q.d[1] * q.d[1] + q.d[2] * q.d[2]);
                    if (q.r < rc) orc_plist_push(L, &q);
                }
    }
}

/* Simple binning for large fully periodic cells (every width >= 3 rc):
 * atoms are wrapped into the cell, binned on a grid of cells at least rc wide,
 * and the 27 surrounding bins are searched.  Images are reported in the frame
 * of the unwrapped input coordinates, exactly as the brute-force search does. */
typedef struct {
    int nb[3];
    int64_t *start;    /* [nbins+1] */
    int64_t *atoms;    /* [N] */
    int32_t *wrap;     /* [N][3] integer shift removed by wrapping */
    int32_t *bin3;     /* [N][3] */
    double *xw;        /* [N][3] wrapped positions */
} orc_bins;

static void orc_bins_build(int64_t N, const double *x, const double *h, const double *hi,
                           const double *wid, double rc, orc_bins *B)
{
    for (int a = 0; a < 3; ++a) { B->nb[a] = (int)floor(wid[a] / rc); }
    int64_t nbins = (int64_t)B->nb[0] * B->nb[1] * B->nb[2];
    B->start = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    B->atoms = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    B->wrap = (int32_t *)malloc((size_t)N * 3 * sizeof(int32_t));
    B->bin3 = (int32_t *)malloc((size_t)N * 3 * sizeof(int32_t));
    B->xw = (double *)malloc((size_t)N * 3 * sizeof(double));
    int64_t *bin = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) {
        double s[3];
        for (int a = 0; a < 3; ++a) {
            s[a] = x[3 * i] * hi[a] + x[3 * i + 1] * hi[3 + a] + x[3 * i + 2] * hi[6 + a];
            double fl = floor(s[a]);
            B->wrap[3 * i + a] = (int32_t)fl;
            s[a] -= fl;
            int b = (int)floor(s[a] * B->nb[a]);
            if (b >= B->nb[a]) b = B->nb[a] - 1;
            if (b < 0) b = 0;
            B->bin3[3 * i + a] = b;
        }
        for (int b = 0; b < 3; ++b)
            B->xw[3 * i + b] = x[3 * i + b] - B->wrap[3 * i] * h[b] - B->wrap[3 * i + 1] * h[3 + b]
                               - B->wrap[3 * i + 2] * h[6 + b];
        bin[i] = ((int64_t)B->bin3[3 * i + 2] * B->nb[1] + B->bin3[3 * i + 1]) * B->nb[0] + B->bin3[3 * i];
        B->start[bin[i] + 1]++;
    }
    for (int64_t b = 0; b < nbins; ++b) B->start[b + 1] += B->start[b];
    int64_t *fill = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) B->atoms[B->start[bin[i]] + fill[bin[i]]++] = i;
    free(fill);
    free(bin);
}

static void orc_bins_free(orc_bins *B)
{
    free(B->start); free(B->atoms); free(B->wrap); free(B->bin3); free(B->xw);
}

static void orc_pairs_binned(const orc_bins *B, const double *h, int64_t i, double rc, orc_plist *L)
{
    const int32_t *bi = B->bin3 + 3 * i;
    for (int o2 = -1; o2 <= 1; ++o2)
        for (int o1 = -1; o1 <= 1; ++o1)
            for (int o0 = -1; o0 <= 1; ++o0) {
                int o[3] = {o0, o1, o2}, bb[3], m[3];
                for (int a = 0; a < 3; ++a) {
                    int b = bi[a] + o[a];
                    m[a] = (int)floor((double)b / B->nb[a]);
                    bb[a] = b - m[a] * B->nb[a];
                }
                int64_t bin = ((int64_t)bb[2] * B->nb[1] + bb[1]) * B->nb[0] + bb[0];
                for (int64_t t = B->start[bin]; t < B->start[bin + 1]; ++t) {
                    int64_t j = B->atoms[t];
                    orc_pair q;
                    for (int b = 0; b < 3; ++b)
                        q.d[b] = B->xw[3 * j + b] + m[0] * h[b] + m[1] * h[3 + b] + m[2] * h[6 + b] - B->xw[3 * i + b];
                    q.r = sqrt(q.d[0] * q.d[0] + q.d[1] * q.d[1] + q.d[2] * q.d[2]);
                    if (q.r >= rc) continue;
                    q.j = j;
                    for (int a = 0; a < 3; ++a) q.n[a] = m[a] - B->wrap[3 * j + a] + B->wrap[3 * i + a];
                    if (j == i && q.n[0] == 0 && q.n[1] == 0 && q.n[2] == 0) continue;
                    orc_plist_push(L, &q);
                }
            }
}

/* ------------------------------------------------------------------ */
/* public: neighbour enumeration (for tests)                           */
/* ------------------------------------------------------------------ */

/* Count (mode 0) or list (mode 1) every pair within rc for every atom.
 * method 0 = brute force over all images, 1 = binned (requires widths >= 3 rc
 * on all axes and pbc on all axes).  On listing, out_j/out_n receive the pairs
 * of atom i at offsets start[i]..start[i+1]-1 (start computed in mode 0 by the
 * caller as a prefix sum of the counts).  Returns 0, or -1 on bad arguments. */
int orc_pairs(int64_t N, const double *x, const double *h, const int32_t *pbc, double rc, int method,
              int mode, int64_t *counts, const int64_t *start, int64_t *out_j, int32_t *out_n,
              double *out_r)
{
    double hi[9], wid[3];
    orc_inv3(h, hi);
    orc_widths(h, wid);
    orc_bins B;
    memset(&B, 0, sizeof B);
    if (method == 1) {
        for (int a = 0; a < 3; ++a) if (!pbc[a] || wid[a] < 3.0 * rc) return -1;
        orc_bins_build(N, x, h, hi, wid, rc, &B);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        orc_plist L = {0, 0, NULL};
        if (method == 1) orc_pairs_binned(&B, h, i, rc, &L);
        else orc_pairs_brute(N, x, h, hi, wid, pbc, i, rc, &L);
        if (mode == 0) counts[i] = L.count;
        else {
            for (int64_t t = 0; t < L.count; ++t) {
                out_j[start[i] + t] = L.p[t].j;
                for (int a = 0; a < 3; ++a) out_n[3 * (start[i] + t) + a] = L.p[t].n[a];
                if (out_r) out_r[start[i] + t] = L.p[t].r;
            }
        }
        free(L.p);
    }
    if (method == 1) orc_bins_free(&B);
    return 0;
}

/* ------------------------------------------------------------------ */
/* per-atom site energy and pair derivatives                           */
/* ------------------------------------------------------------------ */

/* For one atom i with its radial pair list (r < rc_rad), compute:
 *   q[D]      descriptor (unscaled),
 *   U         site energy U_i (NEP + half of the ZBL pair terms),
 *   dUdq[D]   dU^NEP_i/dq_nu,
 *   Dij[3*M]  dU_i/dr_ij for each of the M pairs (pair vector gradient). */
static void orc_site(const orc_model *m, const orc_plist *L, double *q, double *U, double *dUdq,
                     double *Dij)
{
    const int D = orc_dim(m), nR = m->n_rad, nA = m->n_ang, H = m->n_hidden, LM = m->l_max;
    const int64_t M = L->count;
    double *gA = (double *)malloc((size_t)(M * nA + 1) * sizeof(double));
    double *dgA = (double *)malloc((size_t)(M * nA + 1) * sizeof(double));
    int64_t *ang = (int64_t *)malloc((size_t)(M + 1) * sizeof(int64_t));
    int64_t MA = 0;
    double g[64], dg[64];

    for (int nu = 0; nu < D; ++nu) q[nu] = 0.0;
    /* radial descriptor */
    for (int64_t p = 0; p < M; ++p) {
        orc_radial_fns(nR, m->k_rad, m->c_rad, L->p[p].r, m->rc_rad, g, dg);
        for (int n = 0; n < nR; ++n) q[n] += g[n];
        if (L->p[p].r < m->rc_ang) {
            orc_radial_fns(nA, m->k_ang, m->c_ang, L->p[p].r, m->rc_ang, gA + MA * nA, dgA + MA * nA);
            ang[MA++] = p;
        }
    }
    /* angular descriptor: plain double sum with Legendre polynomials */
    for (int64_t a = 0; a < MA; ++a) {
        const orc_pair *pa = &L->p[ang[a]];
        for (int64_t b = 0; b < MA; ++b) {
            const orc_pair *pb = &L->p[ang[b]];
            double c = (pa->d[0] * pb->d[0] + pa->d[1] * pb->d[1] + pa->d[2] * pb->d[2]) / (pa->r * pb->r);
            double P[5], dP[5];
            orc_legendre(c, P, dP);
            for (int l = 1; l <= LM; ++l)
                for (int n = 0; n < nA; ++n)
                    q[nR + nA * (l - 1) + n] += gA[a * nA + n] * gA[b * nA + n] * P[l];
        }
    }
    /* network */
    double e = -m->b1;
    double *dz = (double *)malloc((size_t)H * sizeof(double));
    for (int mu = 0; mu < H; ++mu) {
        double z = -m->b0[mu];
        for (int nu = 0; nu < D; ++nu) z += m->w0[mu * D + nu] * m->q_scale[nu] * q[nu];
        double t = tanh(z);
        e += m->w1[mu] * t;
        dz[mu] = m->w1[mu] * (1.0 - t * t);
    }
    for (int nu = 0; nu < D; ++nu) {
        double s = 0.0;
        for (int mu = 0; mu < H; ++mu) s += dz[mu] * m->w0[mu * D + nu];
        dUdq[nu] = s * m->q_scale[nu];
    }
    free(dz);

    /* pair derivatives: radial part and ZBL */
    for (int64_t p = 0; p < M; ++p) {
        const orc_pair *pp = &L->p[p];
        orc_radial_fns(nR, m->k_rad, m->c_rad, pp->r, m->rc_rad, g, dg);
        double s = 0.0;
        for (int n = 0; n < nR; ++n) s += dUdq[n] * dg[n];
        if (pp->r < m->zbl_r2) {
            double uz, duz;
            orc_zbl(pp->r, m->Z, m->Z, m->zbl_r1, m->zbl_r2, &uz, &duz);
            e += 0.5 * uz;
            s += 0.5 * duz;
        }
        for (int b = 0; b < 3; ++b) Dij[3 * p + b] = s * pp->d[b] / pp->r;
    }
    /* pair derivatives: angular part through cos(theta) of the double sum:
     * dq_nl/dr_ij = 2 sum_k [ g'_j g_k P_l(c_jk) u_j + g_j g_k P_l'(c_jk) (u_k - c_jk u_j) / r_j ] */
    for (int64_t a = 0; a < MA; ++a) {
        const orc_pair *pa = &L->p[ang[a]];
        double ua[3] = {pa->d[0] / pa->r, pa->d[1] / pa->r, pa->d[2] / pa->r};
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t b = 0; b < MA; ++b) {
            const orc_pair *pb = &L->p[ang[b]];
            double ub[3] = {pb->d[0] / pb->r, pb->d[1] / pb->r, pb->d[2] / pb->r};
            double c = ua[0] * ub[0] + ua[1] * ub[1] + ua[2] * ub[2];
            if (b == a) c = 1.0;
            double P[5], dP[5];
            orc_legendre(c, P, dP);
            for (int l = 1; l <= LM; ++l)
                for (int n = 0; n < nA; ++n) {
                    double w = dUdq[nR + nA * (l - 1) + n];
                    double t1 = 2.0 * w * dgA[a * nA + n] * gA[b * nA + n] * P[l];
                    double t2 = (b == a) ? 0.0 : 2.0 * w * gA[a * nA + n] * gA[b * nA + n] * dP[l] / pa->r;
                    for (int k = 0; k < 3; ++k) acc[k] += t1 * ua[k] + t2 * (ub[k] - c * ua[k]);
                }
        }
        for (int k = 0; k < 3; ++k) Dij[3 * ang[a] + k] += acc[k];
    }
    *U = e;
    free(gA); free(dgA); free(ang);
}

/* ------------------------------------------------------------------ */
/* public: energy, forces, virial of one periodic cell                 */
/* ------------------------------------------------------------------ */

/* Evaluate one cell.
 *   N, x[N][3]        positions (A), h[9] lattice vectors as rows, pbc[3]
 *   n_targets/targets atoms whose outputs are wanted; targets == NULL means all
 *                     atoms in order (then n_targets must equal N)
 *   energy_atom[T]    site energies U_i (eV)
 *   forces[T][3]      forces F_i (eV/A)
 *   virial[9]         W (eV), only when targets == NULL, else must be NULL
 *   desc[T][D]        unscaled descriptors q_nu (optional)
 *   method            0 brute-force images, 1 binned (large periodic cells), -1 choose
 * Returns 0 on success, -1 on bad arguments. */
int orc_efv(const orc_model *m, int64_t N, const double *x, const double *h, const int32_t *pbc,
            int64_t n_targets, const int64_t *targets, double *energy_atom, double *forces,
            double *virial, double *desc, int method)
{
    if (!m || N <= 0 || !x || !h || !pbc) return -1;
    if (targets == NULL && n_targets != N) return -1;
    if (targets != NULL && virial != NULL) return -1;
    const int D = orc_dim(m);
    double hi[9], wid[3];
    orc_inv3(h, hi);
    orc_widths(h, wid);
    double rc = m->rc_rad;
    if (method < 0) {
        method = 1;
        for (int a = 0; a < 3; ++a) if (!pbc[a] || wid[a] < 3.0 * rc) method = 0;
    }
    orc_bins B;
    memset(&B, 0, sizeof B);
    if (method == 1) {
        for (int a = 0; a < 3; ++a) if (!pbc[a] || wid[a] < 3.0 * rc) return -1;
        orc_bins_build(N, x, h, hi, wid, rc, &B);
    }

    /* active set: the targets and every atom that has a target in its pair list */
    char *active = (char *)calloc((size_t)N, 1);
    int64_t *tlist = (int64_t *)malloc((size_t)n_targets * sizeof(int64_t));
    for (int64_t t = 0; t < n_targets; ++t) {
        tlist[t] = targets ? targets[t] : t;
        if (tlist[t] < 0 || tlist[t] >= N) { free(active); free(tlist); if (method == 1) orc_bins_free(&B); return -1; }
    }
    orc_plist *PL = (orc_plist *)calloc((size_t)N, sizeof(orc_plist));
    if (targets == NULL) {
        memset(active, 1, (size_t)N);
    } else {
        for (int64_t t = 0; t < n_targets; ++t) active[tlist[t]] = 1;
        /* neighbours of targets (pair relation is symmetric) */
        char *tmark = (char *)calloc((size_t)N, 1);
        for (int64_t t = 0; t < n_targets; ++t) tmark[tlist[t]] = 1;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < n_targets; ++t) {
            int64_t i = tlist[t];
            if (method == 1) orc_pairs_binned(&B, h, i, rc, &PL[i]);
            else orc_pairs_brute(N, x, h, hi, wid, pbc, i, rc, &PL[i]);
        }
        for (int64_t t = 0; t < n_targets; ++t) {
            int64_t i = tlist[t];
            for (int64_t p = 0; p < PL[i].count; ++p) active[PL[i].p[p].j] = 1;
        }
        free(tmark);
    }
    int64_t n_act = 0;
    for (int64_t i = 0; i < N; ++i) n_act += active[i];
    int64_t *act = (int64_t *)malloc((size_t)(n_act + 1) * sizeof(int64_t));
    n_act = 0;
    for (int64_t i = 0; i < N; ++i) if (active[i]) act[n_act++] = i;

    double *U = (double *)calloc((size_t)N, sizeof(double));
    double **Dp = (double **)calloc((size_t)N, sizeof(double *));
    double *Q = desc ? (double *)calloc((size_t)N * D, sizeof(double)) : NULL;

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < n_act; ++t) {
        int64_t i = act[t];
        if (PL[i].count == 0 && PL[i].p == NULL) {
            if (method == 1) orc_pairs_binned(&B, h, i, rc, &PL[i]);
            else orc_pairs_brute(N, x, h, hi, wid, pbc, i, rc, &PL[i]);
        }
        double q[256], dUdq[256];
        Dp[i] = (double *)malloc((size_t)(3 * PL[i].count + 1) * sizeof(double));
        orc_site(m, &PL[i], q, &U[i], dUdq, Dp[i]);
        if (Q) for (int nu = 0; nu < D; ++nu) Q[i * D + nu] = q[nu];
    }

    /* forces: F_i = sum_j dU_i/dr_ij - sum over pairs (a, i) of dU_a/dr_ai */
    double *F = (double *)calloc((size_t)N * 3, sizeof(double));
    for (int64_t t = 0; t < n_act; ++t) {
        int64_t a = act[t];
        for (int64_t p = 0; p < PL[a].count; ++p) {
            int64_t b = PL[a].p[p].j;
            for (int k = 0; k < 3; ++k) {
                F[3 * a + k] += Dp[a][3 * p + k];
                F[3 * b + k] -= Dp[a][3 * p + k];
            }
        }
    }
    if (virial) {
        for (int k = 0; k < 9; ++k) virial[k] = 0.0;
        for (int64_t a = 0; a < N; ++a)
            for (int64_t p = 0; p < PL[a].count; ++p)
                for (int al = 0; al < 3; ++al)
                    for (int be = 0; be < 3; ++be)
                        virial[3 * al + be] -= Dp[a][3 * p + al] * PL[a].p[p].d[be];
    }
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t i = tlist[t];
        if (energy_atom) energy_atom[t] = U[i];
        if (forces) for (int k = 0; k < 3; ++k) forces[3 * t + k] = F[3 * i + k];
        if (desc) for (int nu = 0; nu < D; ++nu) desc[t * D + nu] = Q[i * D + nu];
    }

    for (int64_t i = 0; i < N; ++i) { free(PL[i].p); free(Dp[i]); }
    free(PL); free(Dp); free(U); free(F); free(Q); free(act); free(active); free(tlist);
    if (method == 1) orc_bins_free(&B);
    return 0;
}

/* ------------------------------------------------------------------ */
/* public: gradient of the energy with respect to the model parameters */
/* ------------------------------------------------------------------ */

/* Number of trainable parameters: c_rad, c_ang, w0, b0, w1, b1. */
int orc_num_params(const orc_model *m)
{
    return m->n_rad * m->k_rad + m->n_ang * m->k_ang + m->n_hidden * orc_dim(m) + 2 * m->n_hidden + 1;
}

/* dE/dtheta of one cell, theta = (c_rad, c_ang, w0, b0, w1, b1) flattened in
 * that order (row-major), by the chain rule through the definitions:
 *   dU/dw1_mu = tanh z_mu,  dU/db1 = -1,
 *   dU/dw0_mu,nu = w1_mu (1 - tanh^2 z_mu) s_nu q_nu,  dU/db0_mu = -w1_mu (1 - tanh^2 z_mu),
 *   dU/dc^R_nk = (dU/dq_n) sum_j f_k(r_ij),
 *   dU/dc^A_nk = sum_l (dU/dq_nl) 2 sum_j sum_k' f_k(r_ij) g_n(r_ik') P_l(cos theta_ijk').
 * The ZBL term has no parameters.  grad must hold orc_num_params doubles. */
int orc_param_grad(const orc_model *m, int64_t N, const double *x, const double *h, const int32_t *pbc,
                   int method, double *grad)
{
    if (!m || N <= 0 || !x || !h || !pbc || !grad) return -1;
    const int D = orc_dim(m), nR = m->n_rad, nA = m->n_ang, H = m->n_hidden, LM = m->l_max;
    const int KR = m->k_rad, KA = m->k_ang;
    const int P = orc_num_params(m);
    const int o_cA = nR * KR, o_w0 = o_cA + nA * KA, o_b0 = o_w0 + H * D, o_w1 = o_b0 + H, o_b1 = o_w1 + H;
    double hi[9], wid[3];
    orc_inv3(h, hi);
    orc_widths(h, wid);
    const double rc = m->rc_rad;
    if (method < 0) {
        method = 1;
        for (int a = 0; a < 3; ++a) if (!pbc[a] || wid[a] < 3.0 * rc) method = 0;
    }
    orc_bins B;
    memset(&B, 0, sizeof B);
    if (method == 1) {
        for (int a = 0; a < 3; ++a) if (!pbc[a] || wid[a] < 3.0 * rc) return -1;
        orc_bins_build(N, x, h, hi, wid, rc, &B);
    }
    for (int p = 0; p < P; ++p) grad[p] = 0.0;
#pragma omp parallel
    {
        double *g = (double *)calloc((size_t)P, sizeof(double));
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < N; ++i) {
            orc_plist L = {0, 0, NULL};
            if (method == 1) orc_pairs_binned(&B, h, i, rc, &L);
            else orc_pairs_brute(N, x, h, hi, wid, pbc, i, rc, &L);
            double q[256], dUdq[256], U;
            double *Dij = (double *)malloc((size_t)(3 * L.count + 1) * sizeof(double));
            orc_site(m, &L, q, &U, dUdq, Dij);
            free(Dij);
            /* network parameters */
            for (int mu = 0; mu < H; ++mu) {
                double z = -m->b0[mu];
                for (int nu = 0; nu < D; ++nu) z += m->w0[mu * D + nu] * m->q_scale[nu] * q[nu];
                const double t = tanh(z), dz = m->w1[mu] * (1.0 - t * t);
                g[o_w1 + mu] += t;
                g[o_b0 + mu] -= dz;
                for (int nu = 0; nu < D; ++nu) g[o_w0 + mu * D + nu] += dz * m->q_scale[nu] * q[nu];
            }
            g[o_b1] -= 1.0;
            /* radial coefficients */
            double f[64], df[64];
            for (int64_t p = 0; p < L.count; ++p) {
                orc_basis(KR, L.p[p].r, m->rc_rad, f, df);
                for (int n = 0; n < nR; ++n)
                    for (int k = 0; k < KR; ++k) g[n * KR + k] += dUdq[n] * f[k];
            }
            /* angular coefficients: 2 sum_l dU/dq_nl sum_j sum_k' f_k(r_j) g_n(r_k') P_l */
            int64_t MA = 0;
            for (int64_t p = 0; p < L.count; ++p) MA += L.p[p].r < m->rc_ang;
            double *fa = (double *)malloc((size_t)(MA * KA + 1) * sizeof(double));
            double *ga = (double *)malloc((size_t)(MA * nA + 1) * sizeof(double));
            double *dga = (double *)malloc((size_t)(MA * nA + 1) * sizeof(double));
            const orc_pair **pa = (const orc_pair **)malloc((size_t)(MA + 1) * sizeof(orc_pair *));
            int64_t a = 0;
            for (int64_t p = 0; p < L.count; ++p) {
                if (L.p[p].r >= m->rc_ang) continue;
                orc_basis(KA, L.p[p].r, m->rc_ang, fa + a * KA, df);
                orc_radial_fns(nA, KA, m->c_ang, L.p[p].r, m->rc_ang, ga + a * nA, dga + a * nA);
                pa[a++] = &L.p[p];
            }
            for (int64_t j = 0; j < MA; ++j)
                for (int64_t k = 0; k < MA; ++k) {
                    double c = (pa[j]->d[0] * pa[k]->d[0] + pa[j]->d[1] * pa[k]->d[1] + pa[j]->d[2] * pa[k]->d[2]) /
                               (pa[j]->r * pa[k]->r);
                    if (j == k) c = 1.0;
                    double Pl[5], dPl[5];
                    orc_legendre(c, Pl, dPl);
                    for (int n = 0; n < nA; ++n) {
                        double w = 0.0;
                        for (int l = 1; l <= LM; ++l) w += dUdq[nR + nA * (l - 1) + n] * Pl[l];
                        w *= 2.0 * ga[k * nA + n];
                        for (int kk = 0; kk < KA; ++kk) g[o_cA + n * KA + kk] += w * fa[j * KA + kk];
                    }
                }
            free(fa); free(ga); free(dga); free(pa);
            free(L.p);
        }
#pragma omp critical
        for (int p = 0; p < P; ++p) grad[p] += g[p];
        free(g);
    }
    if (method == 1) orc_bins_free(&B);
    return 0;
}

/* Number of OpenMP threads the oracle will use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Coulomb constant used by the ZBL term, eV*A (exposed for tests). */
double orc_coulomb(void) { return orc_coulomb_ev_a(); }
