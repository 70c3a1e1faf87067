// Kernels of the paper-size model (see nep_wide.h for the phases).  The
// arithmetic follows the default model's kernels (nep_kernels.hip) term by
// term: FP64 pair geometry, Chebyshev basis, radial sums and l <= 3 angular
// sums; FP32 l = 4 sums, network, gradient walk and force kernel, whose
// distance, Chebyshev argument and series stay FP64.  In bin-offset mode (one
// periodic cell) the walks gather 16-byte fixed-point positions and form the
// FP64 pair vectors from them as the force kernels do.  One lane per atom,
// blocks in XCD-aware order.
#include <type_traits>

#include "nep_wide.h"
#include "nep_pairs.h"

namespace nep {

// FP64 basis f_k = (T_k(x) + 1) fc / 2 without the halving: fc and T_k,
// k < K, x = 2 (r/rc - 1)^2 - 1 (the default model's basis_d for any K).
template <int K>
__device__ inline void basis_w(double r, double inv_rc, double &fc, double T[K])
{
    const double PI = 3.14159265358979323846;
    const double tt = r * inv_rc - 1.0;
    fc = 0.5 - 0.5 * sin_halfpi_d(PI * (tt + 0.5));
    const double x = 2.0 * tt * tt - 1.0;
    T[0] = 1.0;
    T[1] = x;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = 2; k < K; ++k) T[k] = fma(x2, T[k - 1], -T[k - 2]);
}

// FP32 T_k and dT_k/dx, k < K.
template <int K>
__device__ inline void cheb_w(float x, float T[K], float dT[K])
{
    T[0] = 1.0f;
    T[1] = x;
    dT[0] = 0.0f;
    dT[1] = 1.0f;
    const float x2 = 2.0f * x;
#pragma unroll
    for (int k = 2; k < K; ++k) {
        T[k] = fmaf(x2, T[k - 1], -T[k - 2]);
        dT[k] = fmaf(x2, dT[k - 1], fmaf(2.0f, T[k - 1], -dT[k - 2]));
    }
}

template <int BS = WBS>
__device__ inline int tile_atom(int n)
{
    const int ntiles = (n + BS - 1) / BS;
    const int tile = xcd_block(ntiles);
    return tile < ntiles ? tile * BS + (int)threadIdx.x : n;
}

// Bin-offset mode: the record's position as fixed-point offsets (units
// 1/qsinv) from the corner of the atom's bin at the last list build; an
// offset beyond the 32-bit range means the atom moved far past the list
// skin (error -9, as for any list that no longer holds).
__device__ inline void w_bin_offsets(const CellGeom *cg, int lbin, const double4 &p, double qsinv, int32_t o[3],
                                     int32_t *status)
{
    const int b0 = lbin % cg->nb[0], b1 = (lbin / cg->nb[0]) % cg->nb[1], b2 = lbin / (cg->nb[0] * cg->nb[1]);
    const double *bv = cg->bv;
    const double d[3] = {p.x - (b0 * bv[0] + b1 * bv[3] + b2 * bv[6]), p.y - (b0 * bv[1] + b1 * bv[4] + b2 * bv[7]),
                         p.z - (b0 * bv[2] + b1 * bv[5] + b2 * bv[8])};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = rint(d[k] * qsinv);
        if (!(fabs(v) < 2147483000.0)) latch_error(status, -9);
        o[k] = (int32_t)fmin(fmax(v, -2147483000.0), 2147483000.0);
    }
}

// One atom's force record: FP64 position, or with bin_sorted set (bin-offset
// mode, a single cell) the 80-byte fixed-point form.
__device__ inline void w_store_record(WAtomRec *__restrict__ xw, int t, const double4 &p, const float a[WKR],
                                      const CellGeom *__restrict__ cells, const int32_t *__restrict__ bin_sorted,
                                      double qsinv, int32_t *__restrict__ status)
{
    if (bin_sorted) {
        WAtomRec80 r;
        w_bin_offsets(cells, bin_sorted[t], p, qsinv, r.o, status);
#pragma unroll
        for (int k = 0; k < WKR; ++k) r.a[k] = a[k];
        r.pad = 0.0f;
        reinterpret_cast<WAtomRec80 *>(xw)[t] = r;
    } else {
        WAtomRec r;
        r.x = p.x;
        r.y = p.y;
        r.z = p.z;
#pragma unroll
        for (int k = 0; k < WKR; ++k) r.a[k] = a[k];
        r.pad[0] = r.pad[1] = 0.0f;
        xw[t] = r;
    }
}

__global__ void k_w_params64(const float *__restrict__ P, double *__restrict__ C64)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < WA * WKA) C64[i] = (double)P[W_CA + i];
    if (i < WA) {
        double s = 0.0;
        for (int k = 0; k < WKA; ++k) s += (double)P[W_CA + i * WKA + k];
        C64[WA * WKA + i] = s;
    }
}

// Parameter blocks of population members: theta[m] (the gradient's layout,
// W_NPARAM floats) with the descriptor scales of `base`, and their double
// angular coefficients and row sums (as k_w_params64).
__global__ __launch_bounds__(256) void k_w_pop_params(const float *__restrict__ theta, const float *__restrict__ base,
                                                      float *__restrict__ P, double *__restrict__ C64)
{
    const int m = blockIdx.x;
    const float *th = theta + (size_t)m * W_NPARAM;
    float *pm = P + (size_t)m * W_SIZE;
    for (int i = threadIdx.x; i < W_SIZE; i += blockDim.x)
        pm[i] = i < W_QS ? th[i] : (i < W_W0 ? base[i] : th[i - WDIM]);
    double *cm = C64 + (size_t)m * W_C64;
    for (int i = threadIdx.x; i < WA * WKA; i += blockDim.x) cm[i] = (double)th[W_CA + i];
    const int i = threadIdx.x;
    if (i < WA) {
        double s = 0.0;
        for (int k = 0; k < WKA; ++k) s += (double)th[W_CA + i * WKA + k];
        cm[WA * WKA + i] = s;
    }
}

// The software pipelines of NeighbourPipe (every entry) and MaskPipe (the
// entries of a bitmask) over the 16-byte fixed-point positions: entries two
// neighbours ahead, the neighbour's position one ahead.
struct FixedNeighbourPipe {
    ListWalk w;
    int count, s;
    int32_t e_cur, e_nx;
    int4 p_cur;
    __device__ FixedNeighbourPipe(const int32_t *__restrict__ nl, const int4 *__restrict__ xf, int base,
                                  uint32_t jmask, int t, int n, int nf, int nb, int cap)
        : w(t, n, nf, nb, cap), count(nf + nb), s(0), e_cur(0), e_nx(0), p_cur(make_int4(0, 0, 0, 0))
    {
        if (count > 0) {
            e_cur = nl[w.off];
            p_cur = xf[(int)((uint32_t)e_cur & jmask) + base];
        }
        w.next();
        if (w.s < count) e_nx = nl[w.off];
    }
    __device__ void pop(const int32_t *__restrict__ nl, const int4 *__restrict__ xf, int base, uint32_t jmask,
                        int32_t &e, int4 &p)
    {
        e = e_cur;
        p = p_cur;
        ++s;
        if (s < count) {
            e_cur = e_nx;
            p_cur = xf[(int)((uint32_t)e_cur & jmask) + base];
            w.next();
            if (w.s < count) e_nx = nl[w.off];
        }
    }
};

struct FixedMaskPipe {
    MaskWalk mw;
    size_t n;
    int t, nf, nb, cap;
    int s_cur, s_nx;
    int32_t e_cur, e_nx;
    int4 p_cur;
    __device__ size_t off(int s) const { return (size_t)list_slot(s, nf, nb, cap) * n + t; }
    __device__ FixedMaskPipe(const uint32_t *__restrict__ mask, const int32_t *__restrict__ nl,
                             const int4 *__restrict__ xf, int base, uint32_t jmask, int t_, int n_, int nf_,
                             int nb_, int cap_)
        : mw(mask, n_, t_, nf_ + nb_), n((size_t)n_), t(t_), nf(nf_), nb(nb_), cap(cap_), e_cur(0), e_nx(0),
          p_cur(make_int4(0, 0, 0, 0))
    {
        s_cur = mw.next();
        if (s_cur >= 0) {
            e_cur = nl[off(s_cur)];
            p_cur = xf[(int)((uint32_t)e_cur & jmask) + base];
        }
        s_nx = mw.next();
        if (s_nx >= 0) e_nx = nl[off(s_nx)];
    }
    __device__ bool valid() const { return s_cur >= 0; }
    __device__ void pop(const int32_t *__restrict__ nl, const int4 *__restrict__ xf, int base, uint32_t jmask,
                        int32_t &e, int4 &p, int &s)
    {
        e = e_cur;
        p = p_cur;
        s = s_cur;
        s_cur = s_nx;
        if (s_cur >= 0) {
            e_cur = e_nx;
            p_cur = xf[(int)((uint32_t)e_cur & jmask) + base];
            s_nx = mw.next();
            if (s_nx >= 0) e_nx = nl[off(s_nx)];
        }
    }
};

// Pair vector of bin-offset mode: the neighbour bin's edge-vector sum from
// the block's LDS table plus the difference of the fixed-point offsets,
// exactly antisymmetric in the two ends.
__device__ __forceinline__ void pair_vector_f(int32_t e, const PairConsts &pc, const int4 &pj, const int4 &pi,
                                              const double *__restrict__ btab, double &dx, double &dy, double &dz)
{
    const double *b = btab + 4 * (int)(((uint32_t)e >> pc.jbits) & 31u);
    dx = fma(pc.qs, (double)pj.x - (double)pi.x, b[0]);
    dy = fma(pc.qs, (double)pj.y - (double)pi.y, b[1]);
    dz = fma(pc.qs, (double)pj.z - (double)pi.z, b[2]);
}

// Radial sums F_k = sum_j f_k(r_ij) over both lists (FP64), descriptors
// q_n = sum_k c_nk F_k -> Q[n][t]; ZBL half energies -> e_atom[t].  The
// radial list is walked in full when *cflag is set, else over the candidates
// of the last full walk (see the default model's descriptor_sums).  D16:
// bin-offset mode, the neighbours' positions gathered as 16-byte fixed-point
// offsets (xf) instead of 32-byte FP64 positions, with the pair vectors of
// the force kernel (this walk is bound by its gathers' tag lookups).
// (three waves per SIMD: 168 registers, a few spilled, measured faster than
// two waves without spills)
template <int BS, bool D16>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void k_w_radial(
    PairConsts pc, const double4 *__restrict__ xq, const int4 *__restrict__ xf,
    const int32_t *__restrict__ cell_of, const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt, const float *__restrict__ P,
    float *__restrict__ Q, double *__restrict__ e_atom, int32_t *__restrict__ status,
    const int32_t *__restrict__ cflag)
{
    __shared__ __align__(16) double btab[D16 ? BIN_TAB : 2];
    if constexpr (D16) stage_bin_vectors(cells, btab);   // one cell in this mode
    const int t = tile_atom<BS>(pc.n);
    if (t >= pc.n || lists_blocked(status)) return;
    const CellGeom *cg = D16 ? cells : cells + cell_of[t];
    const int base = cg->atom_start;
    double4 pi = make_double4(0.0, 0.0, 0.0, 0.0);
    int4 fi = make_int4(0, 0, 0, 0);
    if constexpr (D16) fi = xf[t];
    else pi = xq[t];
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
    const double inv_rR = 1.0 / (double)pc.rc_rad, rcR2 = (double)pc.rc_rad * pc.rc_rad;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    double AR[WKR];
#pragma unroll
    for (int k = 0; k < WKR; ++k) AR[k] = 0.0;
    double ezbl = 0.0;
    bool overlap = false;
    auto radial_term = [&](double r2) {
        const double r = dist_d(r2);
        overlap |= (r < 1e-3);
        double fc, T[WKR];
        basis_w<WKR>(r, inv_rR, fc, T);
#pragma unroll
        for (int k = 0; k < WKR; ++k) AR[k] = fma(fc, T[k], AR[k]);
        if (r < (double)pc.zbl_r2) {
            double U, dU;
            zbl_pair(r, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
            ezbl += 0.5 * U;
        }
    };
    // |r_ij|^2 of a popped entry, in either position form
    auto dist2_p = [&](int32_t e, double px, double py, double pz) {
        double dx, dy, dz;
        pair_vector_p(e, pc, px, py, pz, pi.x, pi.y, pi.z, cg, dx, dy, dz);
        return dx * dx + dy * dy + dz * dz;
    };
    auto dist2_f = [&](int32_t e, const int4 &pj) {
        double dx, dy, dz;
        pair_vector_f(e, pc, pj, fi, btab, dx, dy, dz);
        return dx * dx + dy * dy + dz * dz;
    };
    {
        // angular list: every entry, marking those within the pair-gradient
        // write radius (with a margin) for the angular phases
        const double awr = (double)pc.rc_ang2_write * (1.0 + 0x1p-15);
        MaskWriter mw;
        auto entry = [&](int s, int count, double r2) {
            mw.add(pc.amask, pc.n, t, s, count, r2 < awr);
            if (r2 < rcR2) radial_term(r2);
        };
        if constexpr (D16) {
            for (FixedNeighbourPipe q(nl_ang, xf, base, jmask, t, pc.n, naf, nab, pc.capA); q.s < q.count;) {
                const int s = q.s;
                int32_t e;
                int4 pj;
                q.pop(nl_ang, xf, base, jmask, e, pj);
                entry(s, q.count, dist2_f(e, pj));
            }
        } else {
            for (NeighbourPipe q(nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.s < q.count;) {
                const int s = q.s;
                int32_t e;
                double px, py, pz;
                q.pop(nl_ang, xq, base, jmask, e, px, py, pz);
                entry(s, q.count, dist2_p(e, px, py, pz));
            }
        }
    }
    // radial list: the entries inside rc_rad marked for the force kernel; in
    // full (with the candidate mask written, as the default model's
    // descriptor) or over the last full walk's candidates
    if (*cflag == 0) {
        SparseMaskWriter mw(pc.rmask, pc.n, t, nrf + nrb);
        auto entry = [&](int s, double r2) {
            if (r2 >= rcR2) return;
            mw.set(s);
            radial_term(r2);
        };
        if constexpr (D16) {
            for (FixedMaskPipe q(pc.cmask, nl_rad, xf, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.valid();) {
                int32_t e;
                int4 pj;
                int s;
                q.pop(nl_rad, xf, base, jmask, e, pj, s);
                entry(s, dist2_f(e, pj));
            }
        } else {
            for (MaskPipe q(pc.cmask, nl_rad, xq, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.valid();) {
                int32_t e;
                double px, py, pz;
                int s;
                q.pop(nl_rad, xq, base, jmask, e, px, py, pz, s);
                entry(s, dist2_p(e, px, py, pz));
            }
        }
        mw.finish();
    } else {
        const double rcC2 = (double)pc.rc_cand * pc.rc_cand;
        MaskWriter mw, cw;
        auto entry = [&](int s, int count, double r2) {
            mw.add(pc.rmask, pc.n, t, s, count, r2 < rcR2);
            cw.add(pc.cmask, pc.n, t, s, count, r2 < rcC2);
            if (r2 < rcR2) radial_term(r2);
        };
        if constexpr (D16) {
            for (FixedNeighbourPipe q(nl_rad, xf, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.s < q.count;) {
                const int s = q.s;
                int32_t e;
                int4 pj;
                q.pop(nl_rad, xf, base, jmask, e, pj);
                entry(s, q.count, dist2_f(e, pj));
            }
        } else {
            for (NeighbourPipe q(nl_rad, xq, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.s < q.count;) {
                const int s = q.s;
                int32_t e;
                double px, py, pz;
                q.pop(nl_rad, xq, base, jmask, e, px, py, pz);
                entry(s, q.count, dist2_p(e, px, py, pz));
            }
        }
    }
    if (overlap) latch_error(status, -4);
    const size_t n = (size_t)pc.n;
#pragma unroll 1
    for (int m = 0; m < WR; ++m) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < WKR; ++k) s = fmaf(P[W_CR + m * WKR + k], (float)(0.5 * (AR[k] + AR[0])), s);
        Q[m * n + t] = s;
    }
    e_atom[t] = ezbl;
}

// The angular-list entries within the pair-gradient write radius (amask)
// with their FP64 pair vectors: from the FP64 positions, or in bin-offset
// mode (D16) from the 16-byte fixed-point positions and the block's table of
// bin-offset vectors.  body(e, off, dx, dy, dz), off = the slot's offset.
template <bool D16, class Body>
__device__ __forceinline__ void angular_walk(const PairConsts &pc, const double4 *__restrict__ xq,
                                             const int4 *__restrict__ xf, const double *__restrict__ btab, int t,
                                             const CellGeom *cg, const int32_t *__restrict__ nl_ang, int naf,
                                             int nab, Body &&body)
{
    const int base = cg->atom_start;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    if constexpr (D16) {
        const int4 fi = xf[t];
        for (FixedMaskPipe q(pc.amask, nl_ang, xf, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
            int32_t e;
            int4 pj;
            int s;
            q.pop(nl_ang, xf, base, jmask, e, pj, s);
            double dx, dy, dz;
            pair_vector_f(e, pc, pj, fi, btab, dx, dy, dz);
            body(e, q.off(s), dx, dy, dz);
        }
    } else {
        const double4 pi = xq[t];
        for (MaskPipe q(pc.amask, nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
            int32_t e;
            double px, py, pz;
            int s;
            q.pop(nl_ang, xq, base, jmask, e, px, py, pz, s);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, pi.x, pi.y, pi.z, cg, dx, dy, dz);
            body(e, q.off(s), dx, dy, dz);
        }
    }
}

// Angular sums of the channels c0 .. c0+NC-1 over the angular list:
// S[(c*24 + lm)][t] (l <= 3 in FP64, l = 4 in FP32, rounded once) and the
// descriptors q_cl = sum_m S^2 -> Q[WR + WA (l-1) + c][t].
template <int NC, bool D16>
__device__ __forceinline__ void w_angular_group(const PairConsts &pc, const double4 *__restrict__ xq,
                                                const int4 *__restrict__ xf, const double *__restrict__ btab, int t,
                                                const CellGeom *cg, const int32_t *__restrict__ nl_ang, int naf,
                                                int nab, const double *__restrict__ C64, int c0,
                                                float *__restrict__ S, float *__restrict__ Q)
{
    const double inv_rA = 1.0 / (double)pc.rc_ang, rcA2 = (double)pc.rc_ang * pc.rc_ang;
    double A[NC][15];
    float A4[NC][9];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int m = 0; m < 15; ++m) A[c][m] = 0.0;
#pragma unroll
        for (int m = 0; m < 9; ++m) A4[c][m] = 0.0f;
    }
    angular_walk<D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab, [&](int32_t, size_t, double dx, double dy, double dz) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rcA2) return;
        const double r = dist_d(r2);
        double rinv = (double)frcp((float)r);
        rinv = rinv * fma(-r, rinv, 2.0);
        rinv = rinv * fma(-r, rinv, 2.0);
        const double ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
        double fc, T[WKA];
        basis_w<WKA>(r, inv_rA, fc, T);
        double g[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double sn = C64[WA * WKA + c0 + c];
#pragma unroll
            for (int k = 0; k < WKA; ++k) sn = fma(C64[(c0 + c) * WKA + k], T[k], sn);
            g[c] = 0.5 * fc * sn;
        }
        // unnormalised harmonics; the normalisations are applied to the sums
        double Y[15];
        sph_unnorm_degree_d<1>(ux, uy, uz, Y);
        sph_unnorm_degree_d<2>(ux, uy, uz, Y + 3);
        sph_unnorm_degree_d<3>(ux, uy, uz, Y + 8);
        float Yf[NLM];
        sph_unnorm(SphMono((float)ux, (float)uy, (float)uz), Yf);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int m = 0; m < 15; ++m) A[c][m] = fma(g[c], Y[m], A[c][m]);
            const float gf = (float)g[c];
#pragma unroll
            for (int m = 0; m < 9; ++m) A4[c][m] = fmaf(gf, Yf[15 + m], A4[c][m]);
        }
    });
    const size_t n = (size_t)pc.n;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float ql[LMAX] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            const float v = lm < 15 ? (float)(A[c][lm] * (double)sph_norm(lm)) : A4[c][lm - 15] * sph_norm(lm);
            const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
            ql[l - 1] = fmaf(v, v, ql[l - 1]);
            S[((size_t)(c0 + c) * NLM + lm) * n + t] = v;
        }
#pragma unroll
        for (int l = 1; l <= LMAX; ++l) Q[(size_t)(WR + WA * (l - 1) + c0 + c) * n + t] = ql[l - 1];
    }
}

template <int BS, bool D16>
__global__ __launch_bounds__(BS) void k_w_angular(
    PairConsts pc, const double4 *__restrict__ xq, const int4 *__restrict__ xf, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang, const uint32_t *__restrict__ ncnt,
    const double *__restrict__ C64, int group, float *__restrict__ S, float *__restrict__ Q)
{
    __shared__ __align__(16) double btab[D16 ? BIN_TAB : 2];
    if constexpr (D16) stage_bin_vectors(cells, btab);   // one cell in this mode
    const int t = tile_atom<BS>(pc.n);
    if (t >= pc.n) return;
    const CellGeom *cg = D16 ? cells : cells + cell_of[t];
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff;
    const int c0 = group * WGA;
    if (WA - c0 >= WGA) w_angular_group<WGA, D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab, C64, c0, S, Q);
    else w_angular_group<WA - (WNGA - 1) * WGA, D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab, C64, c0, S, Q);
}

// Network forward and backward of one atom: U (added to the ZBL half
// energies in e_atom), dU/dq; the radial adjoints a_k = sum_n dU/dq_n c_nk
// go into the atom's record, the angular dU/dq into FpA[(nu - WR)][t].
template <int BS>
__global__ __launch_bounds__(BS) void k_w_network(int n_atoms, const double4 *__restrict__ xq,
                                                   const float *__restrict__ P, const float *__restrict__ Q,
                                                   WAtomRec *__restrict__ xw, float *__restrict__ FpA,
                                                   double *__restrict__ e_atom, const CellGeom *__restrict__ cells,
                                                   const int32_t *__restrict__ bin_sorted, double qsinv,
                                                   int32_t *__restrict__ status)
{
    const int t = tile_atom<BS>(n_atoms);
    if (t >= n_atoms) return;
    const size_t n = (size_t)n_atoms;
    float qt[WDIM], Fp[WDIM];
#pragma unroll
    for (int nu = 0; nu < WDIM; ++nu) {
        qt[nu] = P[W_QS + nu] * Q[nu * n + t];
        Fp[nu] = 0.0f;
    }
    float U = -P[W_B1];
#pragma unroll 1
    for (int mu = 0; mu < WH; ++mu) {
        const float *w = P + W_W0 + mu * WDIM;
        float z = -P[W_B0 + mu];
#pragma unroll
        for (int nu = 0; nu < WDIM; ++nu) z = fmaf(w[nu], qt[nu], z);
        const float th = ftanh(z);
        const float w1 = P[W_W1 + mu];
        U = fmaf(w1, th, U);
        const float dz = w1 * fmaf(-th, th, 1.0f);
#pragma unroll
        for (int nu = 0; nu < WDIM; ++nu) Fp[nu] = fmaf(dz, w[nu], Fp[nu]);
    }
#pragma unroll
    for (int nu = 0; nu < WDIM; ++nu) Fp[nu] *= P[W_QS + nu];
    e_atom[t] += (double)U;
    float ak[WKR];
#pragma unroll
    for (int k = 0; k < WKR; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int m = 0; m < WR; ++m) s = fmaf(Fp[m], P[W_CR + m * WKR + k], s);
        ak[k] = s;
    }
    w_store_record(xw, t, xq[t], ak, cells, bin_sorted, qsinv, status);
#pragma unroll
    for (int nu = WR; nu < WDIM; ++nu) FpA[(nu - WR) * n + t] = Fp[nu];
}

// The same network on the matrix cores with FP32 operands
// (v_mfma_f32_32x32x2_f32: FP32 products and accumulation, the precision of
// the vector version in another summation order).  Per 32-atom column tile:
//   forward   Z^T  [128 x 32] = W0 [128 x 60] . Qs^T [60 x 32]
//             (four 32-neuron row tiles, the rows past 100 zero; 30 K steps)
//   backward  Fp^T [64 x 32]  = W0^T [64 x 128] . dZ^T [128 x 32]
// Operand layouts (lane l, hi = l/32, lo = l%32): A[lo][hi], B[hi][lo],
// result D[8(v/4) + 4 hi + v%4][lo], v = 0..15.  The backward's K order is
// the forward result's own layout: K step (mt, v) pairs the neurons
// mt*32 + 8(v/4) + 4 hi + v%4 of the two half-waves, so every lane feeds
// its own dU/dz values as the B operand, straight from registers; the steps
// whose neurons are all past 100 are skipped (52 of 64).  w0 is staged in
// LDS once per block (row stride 65 floats: conflict-free in both
// orientations) and the grid is persistent over 64-atom tiles, one per
// wavefront at a time.
constexpr int WN_MT = 4;          // 32-neuron tiles of the forward
constexpr int WN_LD = 65;         // LDS row stride of w0 (floats)
typedef __attribute__((ext_vector_type(16))) float w_f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 w_bf16x8;

// With BF16 operands (precision mode 1: v_mfma_f32_32x32x16_bf16, FP32
// accumulation) the same products take K steps of 16: operand layouts
// A[lo][8 hi + u], B[8 hi + u][lo] (u = 0..7), the result layout unchanged.
// The forward takes four steps over the 60 (+4 zero) descriptors; the
// backward's step (mt, h) pairs the result registers v = 8h .. 8h+7 of each
// half-wave (neurons mt*32 + 8(v/4) + 4 hi + v%4), seven steps with a real
// neuron.
template <bool BF16>
__global__ __launch_bounds__(WN_BS) __attribute__((amdgpu_waves_per_eu(3))) void k_w_network_mfma(
    int n_atoms, int ntiles, const double4 *__restrict__ xq, const float *__restrict__ P, const float *__restrict__ Q,
    WAtomRec *__restrict__ xw, float *__restrict__ FpA, double *__restrict__ e_atom,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ bin_sorted, double qsinv,
    int32_t *__restrict__ status)
{
    __shared__ float w0s[WN_MT * 32 * WN_LD];      // w0[mu][nu] at mu * WN_LD + nu, zero past 100 x 60
    __shared__ float b0s[WN_MT * 32], w1s[WN_MT * 32];
    __shared__ float qss[64];
    __shared__ float crs[WR * WKR];
    for (int i = threadIdx.x; i < WN_MT * 32 * WN_LD; i += WN_BS) {
        const int mu = i / WN_LD, nu = i - mu * WN_LD;
        w0s[i] = (mu < WH && nu < WDIM) ? P[W_W0 + mu * WDIM + nu] : 0.0f;
    }
    for (int i = threadIdx.x; i < WN_MT * 32; i += WN_BS) {
        b0s[i] = i < WH ? P[W_B0 + i] : 0.0f;
        w1s[i] = i < WH ? P[W_W1 + i] : 0.0f;
    }
    for (int i = threadIdx.x; i < WR * WKR; i += WN_BS) crs[i] = P[W_CR + i];
    if (threadIdx.x < 64) qss[threadIdx.x] = threadIdx.x < WDIM ? P[W_QS + threadIdx.x] : 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hi = lane >> 5, lo = lane & 31;
    const float b1 = P[W_B1];
    for (int tile = blockIdx.x * (WN_BS / 64) + wave; tile < ntiles; tile += gridDim.x * (WN_BS / 64)) {
#pragma unroll 1
        for (int nt = 0; nt < 2; ++nt) {
            const int atom = tile * 64 + nt * 32 + lo;
            const bool valid = atom < n_atoms;
            const int a = valid ? atom : n_atoms - 1;
            // The component stride and the lane's LDS offsets, opaque to the
            // compiler inside the loop: the per-component addresses it would
            // otherwise hoist out of the loop hold ~100 registers (here they
            // are recomputed with an add each).
            size_t ns = (size_t)n_atoms;
            int of = lo * WN_LD + hi;       // forward A: w0[mt*32 + lo][2 st + hi]
            int ob = 4 * hi * WN_LD + lo;   // backward A: w0[mu][dt*32 + lo], mu = mt*32 + 8j + 4 hi + r
            int oh = 4 * hi;                // neuron (and descriptor) offset of this half-wave
            asm volatile("" : "+s"(ns), "+v"(of), "+v"(ob), "+v"(oh));
            w_f32x16 z[WN_MT];
            if constexpr (!BF16) {
                // B operand of the forward: Qs[atom lo][nu = 2 st + hi]
                float qb[WDIM / 2];
                const float *qp = Q + (size_t)hi * ns + a;
#pragma unroll
                for (int st = 0; st < WDIM / 2; ++st) {
                    qb[st] = qss[2 * st + hi] * *qp;
                    qp += 2 * ns;
                }
#pragma unroll
                for (int mt = 0; mt < WN_MT; ++mt) {
                    w_f32x16 acc = {};
#pragma unroll
                    for (int st = 0; st < WDIM / 2; ++st) {
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w0s[of + mt * 32 * WN_LD + 2 * st], qb[st], acc, 0,
                                                                   0, 0);
                        // bound the scheduler's window (it would otherwise
                        // hoist every LDS operand of the tile into registers)
                        if ((st & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
                    z[mt] = acc;
                }
            } else {
                // B operand: Qs[atom lo][nu = 16 st + 8 hi + u], zero past 60
                w_bf16x8 qb[4];
                const float *qp = Q + (size_t)(8 * hi) * ns + a;
#pragma unroll
                for (int st = 0; st < 4; ++st)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        // (components past 60 read the last one's row and
                        // are multiplied by their zero scale)
                        const int nu = 16 * st + 8 * hi + u;
                        const int rowq = nu < WDIM ? 16 * st + u : WDIM - 1 - 8 * hi;
                        qb[st][u] = (__bf16)(qss[nu] * qp[(size_t)rowq * ns]);
                    }
                // A operand rows start at w0[mt*32 + lo][16 st + 8 hi]
                const int ofb = of - hi + 8 * hi;
#pragma unroll
                for (int mt = 0; mt < WN_MT; ++mt) {
                    w_f32x16 acc = {};
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        w_bf16x8 wa;
#pragma unroll
                        for (int u = 0; u < 8; ++u) wa[u] = (__bf16)w0s[ofb + mt * 32 * WN_LD + 16 * st + u];
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, qb[st], acc, 0, 0, 0);
                    }
                    z[mt] = acc;
                }
            }
            // activation in the result layout: tanh, the energy, dU/dz in place
            float Up = 0.0f;
#pragma unroll
            for (int mt = 0; mt < WN_MT; ++mt)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int mu = oh + mt * 32 + 8 * (v >> 2) + (v & 3);
                    const float th = ftanh(z[mt][v] - b0s[mu]);
                    Up = fmaf(w1s[mu], th, Up);
                    z[mt][v] = w1s[mu] * fmaf(-th, th, 1.0f);
                }
            w_f32x16 f[2] = {};
            if constexpr (!BF16) {
#pragma unroll
                for (int mt = 0; mt < WN_MT; ++mt)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        if (mt * 32 + 8 * (v >> 2) >= WH) continue;     // both half-waves' neurons past 100
                        const int row = mt * 32 + 8 * (v >> 2) + (v & 3);
#pragma unroll
                        for (int dt = 0; dt < 2; ++dt)
                            f[dt] = __builtin_amdgcn_mfma_f32_32x32x2f32(w0s[ob + row * WN_LD + dt * 32], z[mt][v],
                                                                         f[dt], 0, 0, 0);
                        if ((v & 1) == 1) __builtin_amdgcn_sched_barrier(0);
                    }
            } else {
#pragma unroll
                for (int mt = 0; mt < WN_MT; ++mt)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (mt * 32 + 16 * h >= WH) continue;           // every neuron of the step past 100
                        w_bf16x8 dzb;
#pragma unroll
                        for (int u = 0; u < 8; ++u) dzb[u] = (__bf16)z[mt][8 * h + u];
#pragma unroll
                        for (int dt = 0; dt < 2; ++dt) {
                            w_bf16x8 wa;
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int row = mt * 32 + 8 * ((8 * h + u) >> 2) + (u & 3);
                                wa[u] = (__bf16)w0s[ob + row * WN_LD + dt * 32];
                            }
                            f[dt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, dzb, f[dt], 0, 0, 0);
                        }
                    }
            }
            const float U = (Up + __shfl_xor(Up, 32, 64)) - b1;
            // dU/dq in the result layout: descriptor nu = dt*32 + 8(v/4) + 4 hi + v%4
            float ak[WKR];
#pragma unroll
            for (int k = 0; k < WKR; ++k) ak[k] = 0.0f;
#pragma unroll
            for (int dt = 0; dt < 2; ++dt)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int nu0 = dt * 32 + 8 * (v >> 2) + (v & 3);   // this component, less 4 hi
                    const float fp = f[dt][v] * qss[oh + nu0];
                    if (dt == 0 && v < 8) {
                        // radial components nu < 16: this half-wave's share of a_k
#pragma unroll
                        for (int k = 0; k < WKR; ++k) ak[k] = fmaf(fp, crs[oh * WKR + nu0 * WKR + k], ak[k]);
                    } else if (valid && oh + nu0 < WDIM) {
                        FpA[(size_t)(oh + nu0 - WR) * ns + atom] = fp;
                    }
                }
#pragma unroll
            for (int k = 0; k < WKR; ++k) ak[k] += __shfl_xor(ak[k], 32, 64);
            if (valid && hi == 0) {
                e_atom[atom] += (double)U;
                w_store_record(xw, atom, xq[atom], ak, cells, bin_sorted, qsinv, status);
            }
        }
    }
}

template __global__ void k_w_network_mfma<false>(int, int, const double4 *, const float *, const float *, WAtomRec *,
                                                  float *, double *, const CellGeom *, const int32_t *, double,
                                                  int32_t *);
template __global__ void k_w_network_mfma<true>(int, int, const double4 *, const float *, const float *, WAtomRec *,
                                                  float *, double *, const CellGeom *, const int32_t *, double,
                                                  int32_t *);

// Contributions of the channels c0 .. c0+NC-1 to dU_i/dr_ij of every angular
// slot, added into pair_grad (the first group writes), and to the atom's own
// force and virial sums.
template <int NC, bool D16>
__device__ __forceinline__ void w_grad_group(const PairConsts &pc, const double4 *__restrict__ xq,
                                             const int4 *__restrict__ xf, const double *__restrict__ btab, int t,
                                             const CellGeom *cg, const int32_t *__restrict__ nl_ang, int naf,
                                             int nab, const float *__restrict__ P, const double *__restrict__ C64,
                                             const float *__restrict__ S,
                                             const float *__restrict__ FpA, int c0, float4 *__restrict__ pair_grad,
                                             float &Fx, float &Fy, float &Fz, float W[9])
{
    const size_t n = (size_t)pc.n;
    // B_{c,lm} = 2 (dU/dq_cl) s_{c,lm}, times the harmonic's normalisation
    // (the walk uses the unnormalised polynomials y_lm = Y_lm / sph_norm(lm))
    float B[NC][NLM];
    float csA[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float cs = 0.0f;
#pragma unroll
        for (int k = 0; k < WKA; ++k) cs += P[W_CA + (c0 + c) * WKA + k];
        csA[c] = cs;
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
            B[c][lm] = (2.0f * sph_norm(lm)) * FpA[(WA * (l - 1) + c0 + c) * n + t] *
                       S[((size_t)(c0 + c) * NLM + lm) * n + t];
        }
    }
    const bool first = c0 == 0;
    const double inv_rA = 1.0 / (double)pc.rc_ang;
    angular_walk<D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab,
                      [&](int32_t, size_t off, double ddx, double ddy, double ddz) {
        const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_ang2) {
            if (first && r2 < pc.rc_ang2_write) pair_grad[off] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            return;
        }
        const float r = fsqrt(r2);
        const float tt = scaled_minus_one(r, pc.inv_rc_ang, pc.inv_rc_ang_lo);
        float fc, dfc;
        cutoff(tt, pc.inv_rc_ang, fc, dfc);
        // x and the Chebyshev terms in FP64 (their rounding is amplified
        // ~k^4 in dT_k near x = -1), the channel sums rounded once; 1/r and
        // the unit vector from the FP64 pair vector too (as the default
        // model's gradient walk)
        const double rd = dist_d(ddx * ddx + ddy * ddy + ddz * ddz);
        const double ttd = rd * inv_rA - 1.0;
        double rinvd = (double)frcp((float)rd);
        rinvd = rinvd * fma(-rd, rinvd, 2.0);
        const float rinv = (float)rinvd;
        const double xd = 2.0 * ttd * ttd - 1.0;
        const float dxdr = (float)(4.0 * ttd * inv_rA);
        double sn[NC], sp[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *cc = C64 + (c0 + c) * WKA;
            sn[c] = C64[WA * WKA + c0 + c] + cc[0] + cc[1] * xd;
            sp[c] = cc[1];
        }
        double Tm2 = 1.0, Tm1 = xd, dTm2 = 0.0, dTm1 = 1.0;
#pragma unroll
        for (int k = 2; k < WKA; ++k) {
            const double Tk = fma(2.0 * xd, Tm1, -Tm2);
            const double dTk = fma(2.0 * xd, dTm1, fma(2.0, Tm1, -dTm2));
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double ck = C64[(c0 + c) * WKA + k];
                sn[c] = fma(ck, Tk, sn[c]);
                sp[c] = fma(ck, dTk, sp[c]);
            }
            Tm2 = Tm1; Tm1 = Tk; dTm2 = dTm1; dTm1 = dTk;
        }
        float g[NC], gp[NC];
        const float hfc = 0.5f * fc, hdx = hfc * dxdr, hdfc = 0.5f * dfc;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            g[c] = hfc * (float)sn[c];
            gp[c] = fmaf(hdx, (float)sp[c], hdfc * (float)sn[c]);
        }
        const float ux = (float)(ddx * rinvd), uy = (float)(ddy * rinvd), uz = (float)(ddz * rinvd);
        const SphMono mono(ux, uy, uz);
        float Y[NLM];
        sph_unnorm(mono, Y);
        // D_lm = sum_c B_{c,lm} g_c; the radial term sum_c g'_c E_c with
        // E_c = sum_lm B_{c,lm} y_lm
        float Dc[NLM], Ec[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) Ec[c] = 0.0f;
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            float D = 0.0f;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                D = fmaf(B[c][lm], g[c], D);
                Ec[c] = fmaf(B[c][lm], Y[lm], Ec[c]);
            }
            Dc[lm] = D;
        }
        float s1 = 0.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) s1 = fmaf(gp[c], Ec[c], s1);
        float vx, vy, vz;
        sph_unnorm_grad_contract(mono, Dc, vx, vy, vz);
        const float uv = ux * vx + uy * vy + uz * vz;
        const float gx = fmaf(s1, ux, (vx - uv * ux) * rinv);
        const float gy = fmaf(s1, uy, (vy - uv * uy) * rinv);
        const float gz = fmaf(s1, uz, (vz - uv * uz) * rinv);
        float4 acc = make_float4(gx, gy, gz, 0.0f);
        if (!first) {
            const float4 old = pair_grad[off];
            acc.x += old.x;
            acc.y += old.y;
            acc.z += old.z;
        }
        pair_grad[off] = acc;
        Fx += gx; Fy += gy; Fz += gz;
        W[0] = fmaf(gx, dx, W[0]); W[1] = fmaf(gx, dy, W[1]); W[2] = fmaf(gx, dz, W[2]);
        W[3] = fmaf(gy, dx, W[3]); W[4] = fmaf(gy, dy, W[4]); W[5] = fmaf(gy, dz, W[5]);
        W[6] = fmaf(gz, dx, W[6]); W[7] = fmaf(gz, dy, W[7]); W[8] = fmaf(gz, dz, W[8]);
    });
}

template <int BS, bool D16>
__global__ __launch_bounds__(BS, 2) void k_w_grad(
    PairConsts pc, const double4 *__restrict__ xq, const int4 *__restrict__ xf, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, const double *__restrict__ C64, const float *__restrict__ S,
    const float *__restrict__ FpA, float4 *__restrict__ pair_grad, float4 *__restrict__ f_own,
    float *__restrict__ w_atom)
{
    __shared__ __align__(16) double btab[D16 ? BIN_TAB : 2];
    if constexpr (D16) stage_bin_vectors(cells, btab);   // one cell in this mode
    const int t = tile_atom<BS>(pc.n);
    if (t >= pc.n) return;
    const CellGeom *cg = D16 ? cells : cells + cell_of[t];
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff;
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = 0.0f;
#pragma unroll 1
    for (int g = 0; g < WNG; ++g) {
        if (WA - g * WG >= WG)
            w_grad_group<WG, D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab, P, C64, S, FpA, g * WG, pair_grad, Fx,
                                  Fy, Fz, W);
        else
            w_grad_group<WA - (WNG - 1) * WG, D16>(pc, xq, xf, btab, t, cg, nl_ang, naf, nab, P, C64, S, FpA, g * WG,
                                                   pair_grad, Fx, Fy, Fz, W);
    }
    f_own[t] = make_float4(Fx, Fy, Fz, 0.0f);
    float *w = w_atom + (size_t)t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = -W[k];
}

// Forces: the default model's force kernel with 16 radial adjoints.  D80:
// bin-offset mode, 80-byte records (WAtomRec80): the pair vector is the sum
// of the neighbour bin's edge vectors (the list entry's bin offset, from the
// block's LDS table) and the difference of the two fixed-point offsets,
// exactly antisymmetric as the FP64 positions' difference.  Both walks load
// the neighbour's record one entry ahead.
template <int BS, bool D80>
__global__ __launch_bounds__(BS) void k_w_force(
    PairConsts pc, const WAtomRec *__restrict__ xw_, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang, const int32_t *__restrict__ nl_rad,
    const uint32_t *__restrict__ ncnt, const uint8_t *__restrict__ rev, const float4 *__restrict__ pair_grad,
    const float4 *__restrict__ f_own, const int32_t *__restrict__ perm, float *__restrict__ fx,
    float *__restrict__ fy, float *__restrict__ fz, float *__restrict__ w_atom, int32_t *__restrict__ status)
{
    using Rec = typename std::conditional<D80, WAtomRec80, WAtomRec>::type;
    const Rec *__restrict__ xw = reinterpret_cast<const Rec *>(xw_);
    __shared__ __align__(16) double btab[D80 ? BIN_TAB : 2];
    if constexpr (D80) stage_bin_vectors(cells, btab);   // one cell in this mode
    const int t = tile_atom<BS>(pc.n);
    if (t >= pc.n || lists_blocked(status)) return;
    const Rec own = xw[t];
    // bin-offset mode has one cell: its geometry is uniform (scalar loads)
    const CellGeom *cg = D80 ? cells : cells + cell_of[t];
    const int base = cg->atom_start;
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    const float4 fo = f_own[t];
    float Fx = fo.x, Fy = fo.y, Fz = fo.z;
    float W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = 0.0f;
    bool bad = false;
    const double inv_rR = 1.0 / (double)pc.rc_rad;

    auto radial = [&](int32_t e, const Rec &rj, float &r2out) -> bool {
        double ddx, ddy, ddz;
        if constexpr (D80) {
            const double *b = btab + 4 * (int)(((uint32_t)e >> pc.jbits) & 31u);
            ddx = fma(pc.qs, (double)rj.o[0] - (double)own.o[0], b[0]);
            ddy = fma(pc.qs, (double)rj.o[1] - (double)own.o[1], b[1]);
            ddz = fma(pc.qs, (double)rj.o[2] - (double)own.o[2], b[2]);
        } else {
            ddx = rj.x - own.x;
            ddy = rj.y - own.y;
            ddz = rj.z - own.z;
            add_image(e, pc, cg, ddx, ddy, ddz);
        }
        const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        r2out = r2;
        if (r2 >= pc.rc_rad2) return false;
        // with 16 Chebyshev terms the rounding of x is amplified ~k^4 in dT_k
        // near x = -1 (the outer shells): the distance, x, the series and
        // their sums with the adjoints in FP64, the cutoff factor in FP32
        const double rd = dist_d(ddx * ddx + ddy * ddy + ddz * ddz);
        const double ttd = rd * inv_rR - 1.0;
        float fc, dfc;
        cutoff((float)ttd, pc.inv_rc_rad, fc, dfc);
        const double xd = 2.0 * ttd * ttd - 1.0;
        double Tm2 = 1.0, Tm1 = xd, dTm2 = 0.0, dTm1 = 1.0;
        const double a0 = (double)own.a[0] + (double)rj.a[0], a1 = (double)own.a[1] + (double)rj.a[1];
        double s0d = fma(a1, xd, a0), s1d = a1, sa = a0 + a1;
#pragma unroll
        for (int k = 2; k < WKR; ++k) {
            const double Tk = fma(2.0 * xd, Tm1, -Tm2);
            const double dTk = fma(2.0 * xd, dTm1, fma(2.0, Tm1, -dTm2));
            const double ah = (double)own.a[k] + (double)rj.a[k];
            s0d = fma(ah, Tk, s0d);
            s1d = fma(ah, dTk, s1d);
            sa += ah;
            Tm2 = Tm1; Tm1 = Tk; dTm2 = dTm1; dTm1 = dTk;
        }
        double dGdr = 0.5 * (4.0 * ttd * inv_rR * (double)fc * s1d + (double)dfc * (s0d + sa));
        if (rd < (double)pc.zbl_r2) {
            double U, dU;
            zbl_pair(rd, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
            dGdr += dU;
        }
        double rinv = (double)frcp((float)rd);
        rinv = rinv * fma(-rd, rinv, 2.0);
        rinv = rinv * fma(-rd, rinv, 2.0);
        const float c = (float)(dGdr * rinv);
        const float px = c * dx, py = c * dy, pz = c * dz;
        Fx += px; Fy += py; Fz += pz;
        W[0] = fmaf(px, dx, W[0]); W[1] = fmaf(px, dy, W[1]); W[2] = fmaf(px, dz, W[2]);
        W[3] = fmaf(py, dx, W[3]); W[4] = fmaf(py, dy, W[4]); W[5] = fmaf(py, dz, W[5]);
        W[6] = fmaf(pz, dx, W[6]); W[7] = fmaf(pz, dy, W[7]); W[8] = fmaf(pz, dz, W[8]);
        return true;
    };

    const int nA = naf + nab;
    {
        ListWalk wa(t, pc.n, naf, nab, pc.capA);
        int32_t e_nx = 0;
        int sj_nx = 255;
        Rec r_nx;
        if (nA > 0) {
            e_nx = nl_ang[wa.off];
            sj_nx = rev[wa.off];
            r_nx = xw[(int)((uint32_t)e_nx & jmask) + base];
        }
        for (int s = 0; s < nA; ++s) {
            const int32_t e = e_nx;
            const int sj = sj_nx;
            const Rec rj = r_nx;
            wa.next();
            if (s + 1 < nA) {
                e_nx = nl_ang[wa.off];
                sj_nx = rev[wa.off];
                r_nx = xw[(int)((uint32_t)e_nx & jmask) + base];
            }
            float r2;
            if (!radial(e, rj, r2) || r2 >= pc.rc_ang2_read) continue;
            if (sj == 255) { bad = true; continue; }
            const float4 gj = pair_grad[(size_t)sj * pc.n + (int)((uint32_t)e & jmask) + base];
            Fx -= gj.x; Fy -= gj.y; Fz -= gj.z;
        }
    }
    // radial list: only the entries k_w_radial found inside rc_rad
    {
        MaskWalk mr(pc.rmask, pc.n, t, nrf + nrb);
        int sr = mr.next();
        int32_t e_nx = 0;
        Rec r_nx;
        if (sr >= 0) {
            e_nx = nl_rad[(size_t)list_slot(sr, nrf, nrb, pc.capR) * pc.n + t];
            r_nx = xw[(int)((uint32_t)e_nx & jmask) + base];
        }
        while (sr >= 0) {
            const int32_t e = e_nx;
            const Rec rj = r_nx;
            sr = mr.next();
            if (sr >= 0) {
                e_nx = nl_rad[(size_t)list_slot(sr, nrf, nrb, pc.capR) * pc.n + t];
                r_nx = xw[(int)((uint32_t)e_nx & jmask) + base];
            }
            float r2;
            radial(e, rj, r2);
        }
    }
    if (bad) latch_error(status, -9);
    const int i = perm[t];
    fx[i] = Fx;
    fy[i] = Fy;
    fz[i] = Fz;
    float *w = w_atom + (size_t)t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = fmaf(-0.5f, W[k], w[k]);
}


// ------------------------------------------------------------------ parameter gradients

// Per-atom factors of the two outer-product blocks in LDS (odd row stride):
// g dz_mu, s q (unweighted), g dU/dq_n (radial), F_k (unweighted); and the
// tile sums of the factors that enter linearly: g tanh z_mu, g G_ck, g.
constexpr int WPG_DZ = 0, WPG_QT = WPG_DZ + WH, WPG_FPR = WPG_QT + WDIM, WPG_F = WPG_FPR + WR,
              WPG_REC = WPG_F + WKR + 1;
constexpr int WPS_TH = 0, WPS_G = WPS_TH + WH, WPS_W = WPS_G + WA * WKA, WPS_N = WPS_W + 1;

// G_ck = sum_j f_k(r_ij) sum_lm B_{c,lm} y_lm(u_ij) of the channels
// c0 .. c0+NC-1 over the marked angular entries, with B_{c,lm} =
// 2 sph_norm(lm) (dU/dq_cl) s_{c,lm}; the tile sums of g G_ck go to tsum.
template <int NC>
__device__ __forceinline__ void w_pg_angular_group(const PairConsts &pc, const double4 *__restrict__ xq, int t,
                                                   const CellGeom *cg, const int32_t *__restrict__ nl_ang,
                                                   int naf, int nab, const float *__restrict__ S,
                                                   const float *__restrict__ FpA, int c0, float g,
                                                   float *__restrict__ tsum)
{
    const size_t n = (size_t)pc.n;
    const double4 pi = xq[t];
    const int base = cg->atom_start;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    const double inv_rA = 1.0 / (double)pc.rc_ang, rcA2 = (double)pc.rc_ang * pc.rc_ang;
    float B[NC][NLM], G[NC][WKA];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
            B[c][lm] = (2.0f * sph_norm(lm)) * FpA[(WA * (l - 1) + c0 + c) * n + t] *
                       S[((size_t)(c0 + c) * NLM + lm) * n + t];
        }
#pragma unroll
        for (int k = 0; k < WKA; ++k) G[c][k] = 0.0f;
    }
    for (MaskPipe q(pc.amask, nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
        int32_t e;
        double px, py, pz;
        int s;
        q.pop(nl_ang, xq, base, jmask, e, px, py, pz, s);
        double dx, dy, dz;
        pair_vector_p(e, pc, px, py, pz, pi.x, pi.y, pi.z, cg, dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rcA2) continue;
        const double r = dist_d(r2);
        double rinv = (double)frcp((float)r);
        rinv = rinv * fma(-r, rinv, 2.0);
        rinv = rinv * fma(-r, rinv, 2.0);
        double fc, T[WKA];
        basis_w<WKA>(r, inv_rA, fc, T);
        float Y[NLM];
        sph_unnorm(SphMono((float)(dx * rinv), (float)(dy * rinv), (float)(dz * rinv)), Y);
        const float hfc = (float)(0.5 * fc);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            float E = 0.0f;
#pragma unroll
            for (int lm = 0; lm < NLM; ++lm) E = fmaf(B[c][lm], Y[lm], E);
            const float hE = hfc * E;      // f_k = (T_k + 1) fc / 2
#pragma unroll
            for (int k = 0; k < WKA; ++k) G[c][k] = fmaf(hE, (float)(T[k] + 1.0), G[c][k]);
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < WKA; ++k) {
            const float sg = wave_sum64(g * G[c][k]);
            if (threadIdx.x == 0) tsum[WPS_G + (c0 + c) * WKA + k] = sg;
        }
}

// Gradient of sum_i gE[cell(i)] U_i with respect to theta for the
// paper-size model, from the staged descriptors Q, angular sums S and
// angular adjoints FpA of the current positions (the first three phases):
//   dU/dw1_mu = tanh z_mu, dU/db0_mu = -dz_mu, dU/dw0_mu,nu = dz_mu s_nu q_nu,
//   dU/db1 = -1, dU/dc^R_nk = (dU/dq_n) F_k,
//   dU/dc^A_ck = sum_j f_k(r_ij) sum_lm B_{c,lm} y_lm(u_ij),
// with dz_mu = w1_mu (1 - tanh^2 z_mu), F_k = sum_j f_k(r_ij) over rc_rad
// (Eqs. 2-4; the same decomposition as the default model's gradient).
// 64-atom tiles, one wavefront per block; the outer products are summed
// per output over the tile from LDS, one FP64 partial row per block.  Lanes
// past the last atom evaluate atom 0 with weight 0.
__global__ __launch_bounds__(64) void k_w_param_grad(
    PairConsts pc, const double4 *__restrict__ xq, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang, const int32_t *__restrict__ nl_rad,
    const uint32_t *__restrict__ ncnt, const float *__restrict__ P, const float *__restrict__ Q,
    const float *__restrict__ S, const float *__restrict__ FpA, const double *__restrict__ gE,
    double *__restrict__ part, int32_t *__restrict__ status, int ntiles)
{
    __shared__ float rec[64][WPG_REC];
    __shared__ float tsum[WPS_N];
    constexpr int NOWN = (W_NPARAM + 63) / 64;
    const int lane = threadIdx.x;
    const size_t n = (size_t)pc.n;
    double *pb = part + (size_t)blockIdx.x * W_NPARAM;
    const bool ok = !lists_blocked(status);
    for (int k = 0; k < NOWN; ++k) {
        const int o = lane + 64 * k;
        if (o < W_NPARAM) pb[o] = 0.0;
    }
    const double inv_rR = 1.0 / (double)pc.rc_rad, rcR2 = (double)pc.rc_rad * pc.rc_rad;
    const uint32_t jmask = (1u << pc.jbits) - 1u;

    for (int tile = blockIdx.x; tile < ntiles && ok; tile += gridDim.x) {
        const bool valid = tile * 64 + lane < pc.n;
        const int t = valid ? tile * 64 + lane : 0;
        float *r = rec[lane];
        const float g = valid ? (float)gE[cell_of[t]] : 0.0f;
        // network forward and backward
        float qt[WDIM], Fp[WDIM];
#pragma unroll
        for (int nu = 0; nu < WDIM; ++nu) {
            qt[nu] = P[W_QS + nu] * Q[nu * n + t];
            r[WPG_QT + nu] = qt[nu];
            Fp[nu] = 0.0f;
        }
#pragma unroll 1
        for (int mu = 0; mu < WH; ++mu) {
            const float *w = P + W_W0 + mu * WDIM;
            float z = -P[W_B0 + mu];
#pragma unroll
            for (int nu = 0; nu < WDIM; ++nu) z = fmaf(w[nu], qt[nu], z);
            const float th = ftanh(z);
            const float dz = P[W_W1 + mu] * fmaf(-th, th, 1.0f);
            const float sth = wave_sum64(g * th);
            if (lane == 0) tsum[WPS_TH + mu] = sth;
            r[WPG_DZ + mu] = g * dz;
#pragma unroll
            for (int nu = 0; nu < WR; ++nu) Fp[nu] = fmaf(dz, w[nu], Fp[nu]);
        }
#pragma unroll
        for (int m = 0; m < WR; ++m) r[WPG_FPR + m] = g * (Fp[m] * P[W_QS + m]);
        // radial basis sums F_k over both lists (FP64, as the radial phase)
        const CellGeom *cg = cells + cell_of[t];
        const int base = cg->atom_start;
        const double4 pi = xq[t];
        const uint32_t cnt = ncnt[t];
        const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
        double AR[WKR];
#pragma unroll
        for (int k = 0; k < WKR; ++k) AR[k] = 0.0;
        auto radial_term = [&](double r2) {
            double fc, T[WKR];
            basis_w<WKR>(dist_d(r2), inv_rR, fc, T);
#pragma unroll
            for (int k = 0; k < WKR; ++k) AR[k] = fma(fc, T[k], AR[k]);
        };
        for (NeighbourPipe q(nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.s < q.count;) {
            int32_t e;
            double px, py, pz;
            q.pop(nl_ang, xq, base, jmask, e, px, py, pz);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, pi.x, pi.y, pi.z, cg, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rcR2) radial_term(r2);
        }
        for (MaskPipe q(pc.rmask, nl_rad, xq, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.valid();) {
            int32_t e;
            double px, py, pz;
            int s;
            q.pop(nl_rad, xq, base, jmask, e, px, py, pz, s);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, pi.x, pi.y, pi.z, cg, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rcR2) radial_term(r2);
        }
#pragma unroll
        for (int k = 0; k < WKR; ++k) r[WPG_F + k] = (float)(0.5 * (AR[k] + AR[0]));
        // angular coefficient sums, channel group by channel group
#pragma unroll 1
        for (int grp = 0; grp < WNG; ++grp) {
            const int c0 = grp * WG;
            if (WA - c0 >= WG) w_pg_angular_group<WG>(pc, xq, t, cg, nl_ang, naf, nab, S, FpA, c0, g, tsum);
            else w_pg_angular_group<WA - (WNG - 1) * WG>(pc, xq, t, cg, nl_ang, naf, nab, S, FpA, c0, g, tsum);
        }
        const float sw = wave_sum64(g);
        if (lane == 0) tsum[WPS_W] = sw;
        __syncthreads();
        constexpr int O_CA = WR * WKR, O_W0 = O_CA + WA * WKA, O_B0 = O_W0 + WH * WDIM, O_W1 = O_B0 + WH,
                      O_B1 = O_W1 + WH;
        for (int k = 0; k < NOWN; ++k) {
            const int o = lane + 64 * k;
            if (o >= W_NPARAM) break;
            float sum = 0.0f;
            if (o < O_CA) {
                const int i1 = WPG_FPR + o / WKR, i2 = WPG_F + o % WKR;
                for (int a = 0; a < 64; ++a) sum = fmaf(rec[a][i1], rec[a][i2], sum);
            } else if (o < O_W0) {
                sum = tsum[WPS_G + (o - O_CA)];
            } else if (o < O_B0) {
                const int p = o - O_W0;
                const int i1 = WPG_DZ + p / WDIM, i2 = WPG_QT + p % WDIM;
                for (int a = 0; a < 64; ++a) sum = fmaf(rec[a][i1], rec[a][i2], sum);
            } else if (o < O_W1) {
                const int i1 = WPG_DZ + (o - O_B0);
                for (int a = 0; a < 64; ++a) sum += rec[a][i1];
                sum = -sum;
            } else if (o < O_B1) {
                sum = tsum[WPS_TH + (o - O_W1)];
            } else {
                sum = -tsum[WPS_W];
            }
            pb[o] += (double)sum;
        }
        __syncthreads();
    }
}

// launch shapes: 64, 128 and 256 threads per block (chosen by nep_autotune)
#define NEP_W_INST(BS)                                                                                               \
    template __global__ void k_w_radial<BS, false>(PairConsts, const double4 *, const int4 *, const int32_t *,       \
                                                   const CellGeom *, const int32_t *, const int32_t *,                \
                                                   const uint32_t *, const float *, float *, double *, int32_t *,     \
                                                   const int32_t *);                                                  \
    template __global__ void k_w_radial<BS, true>(PairConsts, const double4 *, const int4 *, const int32_t *,        \
                                                  const CellGeom *, const int32_t *, const int32_t *,                 \
                                                  const uint32_t *, const float *, float *, double *, int32_t *,      \
                                                  const int32_t *);                                                   \
    template __global__ void k_w_angular<BS, false>(PairConsts, const double4 *, const int4 *, const int32_t *,      \
                                                    const CellGeom *, const int32_t *, const uint32_t *,              \
                                                    const double *, int, float *, float *);                           \
    template __global__ void k_w_angular<BS, true>(PairConsts, const double4 *, const int4 *, const int32_t *,       \
                                                   const CellGeom *, const int32_t *, const uint32_t *,               \
                                                   const double *, int, float *, float *);                            \
    template __global__ void k_w_network<BS>(int, const double4 *, const float *, const float *, WAtomRec *, float *, \
                                             double *, const CellGeom *, const int32_t *, double, int32_t *);         \
    template __global__ void k_w_grad<BS, false>(PairConsts, const double4 *, const int4 *, const int32_t *,         \
                                                 const CellGeom *, const int32_t *, const uint32_t *, const float *,  \
                                                 const double *, const float *, const float *, float4 *, float4 *,    \
                                                 float *);                                                            \
    template __global__ void k_w_grad<BS, true>(PairConsts, const double4 *, const int4 *, const int32_t *,          \
                                                const CellGeom *, const int32_t *, const uint32_t *, const float *,   \
                                                const double *, const float *, const float *, float4 *, float4 *,     \
                                                float *);                                                             \
    template __global__ void k_w_force<BS, false>(PairConsts, const WAtomRec *, const int32_t *, const CellGeom *,    \
                                                  const int32_t *, const int32_t *, const uint32_t *,                 \
                                                  const uint8_t *, const float4 *, const float4 *, const int32_t *,   \
                                                  float *, float *, float *, float *, int32_t *);                     \
    template __global__ void k_w_force<BS, true>(PairConsts, const WAtomRec *, const int32_t *, const CellGeom *,     \
                                                 const int32_t *, const int32_t *, const uint32_t *,                  \
                                                 const uint8_t *, const float4 *, const float4 *, const int32_t *,    \
                                                 float *, float *, float *, float *, int32_t *);
NEP_W_INST(64)
NEP_W_INST(128)
NEP_W_INST(256)

}  // namespace nep
