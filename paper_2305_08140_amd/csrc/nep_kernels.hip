// NEP-ZBL hot-path kernels for gfx950 (MI355X).
//
// Atom data live in a cell-list ("sorted") order: within every cell, atoms
// are grouped by bin, so that a 64-wide wavefront works on spatially close
// atoms and its neighbour gathers hit the same cache lines.  Positions are
// FP64 structure-of-arrays; every pair vector is formed in FP64, so absolute
// coordinates of a 500 A box never lose precision in the pair geometry.  The
// descriptor's pair geometry, Chebyshev basis and the l <= 3 angular sums
// stay in FP64 (on CDNA an FP64 FMA issues at the rate of an unpacked FP32
// FMA): near a lattice site those sums are small differences of large terms,
// and FP32 rounding there would dominate the force error.  The l = 4 sums,
// the network, the angular gradient walk and the force kernel are FP32.
//
// Energy (Eq. 1): the descriptor kernel computes, per atom i,
//   radial   A_k = sum_j fc(r_ij) T_k(x_ij)  ->  F_k = (A_k + A_0)/2 = sum_j f_k(r_ij)
//            q_n = sum_k c^R_nk F_k
//   angular  s_{n,lm} = sum_j g_n(r_ij) Y_lm(u_ij) ->  q_nl = sum_m s_{n,lm}^2
//            (Y scaled so that sum_m Y_lm(u) Y_lm(v) = P_l(u.v), i.e. q_nl is the
//             Legendre double sum over neighbour pairs, j = k included)
//   network  U_i = sum_mu w1 tanh(w0 (s q) - b0) - b1, plus 1/2 sum_j U_ZBL(r_ij)
// and stores the adjoints dU_i/dF_k (9 floats) and B_{n,lm} = dU_i/ds_{n,lm}
// (120 floats).
//
// Forces: F_i = sum_j [dU_i/dr_ij - dU_j/dr_ji].
//   radial part: both terms depend on |r_ij| only, so together they are
//     (a^i + a^j) . f'(r_ij) u_ij, one evaluation per pair with the neighbour's
//     9 adjoint floats gathered;
//   angular part: the descriptor kernel, which holds B^i in registers, stores
//     dU_i/dr_ij for every angular pair (16 bytes per pair) and the force
//     kernel subtracts the stored dU_j/dr_ji found through a reverse index
//     built with the lists.
// Inside-cutoff bitmasks: the descriptor kernel records which radial-list
// entries lie inside rc_rad (the force kernel then walks only those) and,
// in its first angular walk, which angular-list entries lie within the
// pair-gradient write radius (its later angular walks take only those), so
// the skin entries of the lists are loaded once per evaluation.
// No atomics: every atom gathers its own force, deterministically.  The pair
// vector seen from j is the exact negative of the one seen from i, so both
// ends agree bit for bit on which pairs are inside a cutoff.
// Virial: W = -sum_i sum_j dU_i/dr_ij (x) r_ij (angular, per owner) plus
// -1/2 sum_i sum_j f_ij (x) r_ij for the radial and ZBL pair forces f_ij.
#include <type_traits>
#include "nep_device.h"
#include "nep_pairs.h"

namespace nep {

// Angular radial functions g_n(r) = sum_k c_nk f_k(r) and the unit vector,
// in double precision (C64: c^A_nk [NA][KB], then the row sums [NA]).
__device__ inline void angular_g_d(double r, double dx, double dy, double dz, double inv_rA,
                                   const double *__restrict__ C64, double g[NA], double &ux, double &uy,
                                   double &uz)
{
    const float rf = (float)r;
    double rinv = (double)frcp(rf);
    rinv = rinv * fma(-r, rinv, 2.0);        // one Newton step: relative error ~1e-14
    rinv = rinv * fma(-r, rinv, 2.0);
    ux = dx * rinv;
    uy = dy * rinv;
    uz = dz * rinv;
    double fc, T[KB];
    basis_d(r, inv_rA, fc, T);
    const double hfc = 0.5 * fc;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        double sn = C64[NA * KB + n];
#pragma unroll
        for (int k = 0; k < KB; ++k) sn = fma(C64[n * KB + k], T[k], sn);
        g[n] = hfc * sn;
    }
}

// The l = 3 and l = 4 angular sums, S[n][lm] = sum_j g_n(r_ij) Y_lm(u_ij),
// over the angular list: l = 3 formed and accumulated in double precision,
// l = 4 in single precision (its sums do not cancel to the same degree near
// a lattice site), both rounded once into S.
__device__ __forceinline__ void angular_sums_l34(const PairConsts &pc, const double4 *__restrict__ xq, int t,
                                                 double xi, double yi, double zi, const CellGeom *cg, int base,
                                                 const int32_t *__restrict__ nl_ang, int naf, int nab,
                                                 const double *__restrict__ C64, float S[NA][NLM])
{
    const double inv_rA = 1.0 / (double)pc.rc_ang, rcA2 = (double)pc.rc_ang * pc.rc_ang;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    double A3[NA][7];
    float A4[NA][9];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
#pragma unroll
        for (int m = 0; m < 7; ++m) A3[n][m] = 0.0;
#pragma unroll
        for (int m = 0; m < 9; ++m) A4[n][m] = 0.0f;
    }
    for (MaskPipe q(pc.amask, nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
        int32_t e;
        double px, py, pz;
        int s;
        q.pop(nl_ang, xq, base, jmask, e, px, py, pz, s);
        double dx, dy, dz;
        pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rcA2) continue;
        double g[NA], ux, uy, uz;
        angular_g_d(dist_d(r2), dx, dy, dz, inv_rA, C64, g, ux, uy, uz);
        // unnormalised harmonics; the normalisations are applied to the sums
        double Y3[7];
        sph_unnorm_degree_d<3>(ux, uy, uz, Y3);
        float Y[NLM];
        sph_unnorm(SphMono((float)ux, (float)uy, (float)uz), Y);
#pragma unroll
        for (int n = 0; n < NA; ++n) {
#pragma unroll
            for (int m = 0; m < 7; ++m) A3[n][m] = fma(g[n], Y3[m], A3[n][m]);
            const float gf = (float)g[n];
#pragma unroll
            for (int m = 0; m < 9; ++m) A4[n][m] = fmaf(gf, Y[15 + m], A4[n][m]);
        }
    }
#pragma unroll
    for (int n = 0; n < NA; ++n) {
#pragma unroll
        for (int m = 0; m < 7; ++m) S[n][8 + m] = (float)(A3[n][m] * (double)sph_norm(8 + m));
#pragma unroll
        for (int m = 0; m < 9; ++m) S[n][15 + m] = A4[n][m] * sph_norm(15 + m);
    }
}

// Radial walk modes of descriptor_sums: every entry of the radial list, or
// every entry and the candidate mask (entries within rc_cand) written, or the
// candidates of the last full walk only (valid while no atom has moved by
// half of rc_cand - rc_rad since then).
constexpr int CAND_OFF = 0, CAND_WRITE = 1, CAND_READ = 2;

// Descriptor sums of one atom.  The radial sums F_k = sum_j f_k(r_ij) and
// the angular sums S[n][lm] = sum_j g_n(r_ij) Y_lm(u_ij) for l <= 3 are
// formed and accumulated in double precision: near a lattice site the odd-l
// (and, in cubic crystals, the l = 2) sums are small differences of large
// terms.  To keep the accumulators in registers the angular list is walked
// twice: l = 1, 2 together with the radial and ZBL terms of that list, then
// l = 3 (and l = 4 in single precision); the sums are rounded to single
// precision after each pass.  Returns F, S and the ZBL half-energy.
__device__ __forceinline__ void descriptor_sums(const PairConsts &pc, const double4 *__restrict__ xq, int t,
                                                double xi, double yi, double zi, const CellGeom *cg, int base,
                                                const int32_t *__restrict__ nl_ang,
                                                const int32_t *__restrict__ nl_rad, int naf, int nab, int nrf,
                                                int nrb, const double *__restrict__ C64, float F[KB],
                                                float S[NA][NLM], double &ezbl, bool &overlap, int cand_mode)
{
    const double inv_rR = 1.0 / (double)pc.rc_rad, inv_rA = 1.0 / (double)pc.rc_ang;
    const double rcR2 = (double)pc.rc_rad * pc.rc_rad, rcA2 = (double)pc.rc_ang * pc.rc_ang;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    double AR[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) AR[k] = 0.0;
    ezbl = 0.0;
    overlap = false;

    {
        double A[NA][8];
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int m = 0; m < 8; ++m) A[n][m] = 0.0;
        // entries within the pair-gradient write radius (with a margin over
        // the FP32 radius the gradient walk tests) for the later angular walks
        const double awr = (double)pc.rc_ang2_write * (1.0 + 0x1p-15);
        MaskWriter amw;
        for (NeighbourPipe q(nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.s < q.count;) {
            const int s = q.s;
            int32_t e;
            double px, py, pz;
            q.pop(nl_ang, xq, base, jmask, e, px, py, pz);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            amw.add(pc.amask, pc.n, t, s, q.count, r2 < awr);
            if (r2 >= rcR2) continue;
            const double r = dist_d(r2);
            overlap |= (r < 1e-3);
            {
                double fc, T[KB];
                basis_d(r, inv_rR, fc, T);
#pragma unroll
                for (int k = 0; k < KB; ++k) AR[k] = fma(fc, T[k], AR[k]);
            }
            if (r2 < rcA2) {
                double g[NA], ux, uy, uz;
                angular_g_d(r, dx, dy, dz, inv_rA, C64, g, ux, uy, uz);
                double Y[8];
                sph_unnorm_degree_d<1>(ux, uy, uz, Y);
                sph_unnorm_degree_d<2>(ux, uy, uz, Y + 3);
#pragma unroll
                for (int n = 0; n < NA; ++n)
#pragma unroll
                    for (int m = 0; m < 8; ++m) A[n][m] = fma(g[n], Y[m], A[n][m]);
            }
            if (r < (double)pc.zbl_r2) {
                double U, dU;
                zbl_pair(r, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
                ezbl += 0.5 * U;
            }
        }
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int m = 0; m < 8; ++m) S[n][m] = (float)(A[n][m] * (double)sph_norm(m));
    }
    if (cand_mode == CAND_READ) {
        // the candidates of the last full walk: every entry inside rc_rad now
        // is among them; the inside bits of the others are stored as zero
        SparseMaskWriter mw(pc.rmask, pc.n, t, nrf + nrb);
        for (MaskPipe q(pc.cmask, nl_rad, xq, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.valid();) {
            int32_t e;
            double px, py, pz;
            int s;
            q.pop(nl_rad, xq, base, jmask, e, px, py, pz, s);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= rcR2) continue;
            mw.set(s);
            double fc, T[KB];
            basis_d(dist_d(r2), inv_rR, fc, T);
#pragma unroll
            for (int k = 0; k < KB; ++k) AR[k] = fma(fc, T[k], AR[k]);
        }
        mw.finish();
    } else {
        const double rcC2 = (double)pc.rc_cand * pc.rc_cand;
        MaskWriter mw, cw;
        for (NeighbourPipe q(nl_rad, xq, base, jmask, t, pc.n, nrf, nrb, pc.capR); q.s < q.count;) {
            const int s = q.s;
            int32_t e;
            double px, py, pz;
            q.pop(nl_rad, xq, base, jmask, e, px, py, pz);
            double dx, dy, dz;
            pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            mw.add(pc.rmask, pc.n, t, s, q.count, r2 < rcR2);
            if (cand_mode == CAND_WRITE) cw.add(pc.cmask, pc.n, t, s, q.count, r2 < rcC2);
            if (r2 >= rcR2) continue;
            double fc, T[KB];
            basis_d(dist_d(r2), inv_rR, fc, T);
#pragma unroll
            for (int k = 0; k < KB; ++k) AR[k] = fma(fc, T[k], AR[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) F[k] = (float)(0.5 * (AR[k] + AR[0]));
    angular_sums_l34(pc, xq, t, xi, yi, zi, cg, base, nl_ang, naf, nab, C64, S);
}

// Descriptor vector q from the sums (radial q_n = sum_k c_nk F_k, angular q_nl = sum_m S^2).
__device__ __forceinline__ void descriptor_vector(const float *__restrict__ P, const float F[KB],
                                                  const float S[NA][NLM], float q[DIM])
{
#pragma unroll
    for (int n = 0; n < NR; ++n) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < KB; ++k) s = fmaf(P[P_CR + n * KB + k], F[k], s);
        q[n] = s;
    }
#pragma unroll
    for (int l = 1; l <= LMAX; ++l)
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float s = 0.0f;
#pragma unroll
            for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) s = fmaf(S[n][lm], S[n][lm], s);
            q[NR + NA * (l - 1) + n] = s;
        }
}

// Network forward and backward in one pass over the hidden neurons: row mu of
// w0 gives z_mu, and dU/dz_mu times the same row accumulates dU/dq.  Returns
// U (without ZBL) and Fp = dU/dq (q unscaled).
__device__ __forceinline__ float network(const float *__restrict__ P, const float q[DIM], float Fp[DIM])
{
    float qt[DIM];
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) qt[nu] = P[P_QS + nu] * q[nu];
    float U = -P[P_B1];
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) Fp[nu] = 0.0f;
#pragma unroll 1
    for (int mu = 0; mu < NH; ++mu) {
        const float *w = P + P_W0 + mu * DIM;
        float z = -P[P_B0 + mu];
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) z = fmaf(w[nu], qt[nu], z);
        const float th = ftanh(z);
        const float w1 = P[P_W1 + mu];
        U = fmaf(w1, th, U);
        const float dz = w1 * fmaf(-th, th, 1.0f);
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) Fp[nu] = fmaf(dz, w[nu], Fp[nu]);
    }
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) Fp[nu] *= P[P_QS + nu];
    return U;
}

__device__ __forceinline__ void angular_coef_sums(const float *__restrict__ P, float csA[NA])
{
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < KB; ++k) s += P[P_CA + n * KB + k];
        csA[n] = s;
    }
}

// ------------------------------------------------------------------ MFMA hidden layer (BF16)
// The hidden layer of a whole wavefront (64 atoms) as matrix products on the
// matrix cores, BF16 inputs with FP32 accumulation:
//   forward   Z^T  [32 x 64] = W0 [32 x 32] . Qs^T [32 x 64]     (Qs = scaled descriptors)
//   backward  Fp^T [32 x 64] = W0^T [32 x 32] . dZ^T [32 x 64]   (dZ = dU/dz)
// with v_mfma_f32_32x32x16_bf16 (two 32-atom column tiles, two K steps each).
// Operand layouts (lane l, v = 0..7 / 0..15):  A[l%32][8(l/32)+v],
// B[8(l/32)+v][l%32], D[8(v/4)+4(l/32)+v%4][l%32].  Rows of the padded
// 32 x 32 weight (30 neurons x 29 descriptors) beyond the model are zero.
// Each lane owns one atom; the operands are exchanged through a per-wave LDS
// area (a wave's LDS accesses complete in program order).
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

struct NNLds {
    union {
        __bf16 q[64][40];    // BF16 operands: rows of 32 used; stride 80 B keeps 16 B alignment
        float qf[64][33];    // FP32 operands
    };
    float z[64][33];
};

__device__ __forceinline__ float network_mfma(const float *__restrict__ P, const float q[DIM], float Fp[DIM],
                                              NNLds *L)
{
    const int lane = threadIdx.x & 63;
    const int hi = lane >> 5, lo = lane & 31;
    // own scaled descriptor row
#pragma unroll
    for (int nu = 0; nu < 32; ++nu) L->q[lane][nu] = (__bf16)(nu < DIM ? P[P_QS + nu] * q[nu] : 0.0f);
    // weight operands: forward A[mu = lo][nu = 16 s + 8 hi + v], backward A[nu = lo][mu = 16 s + 8 hi + v]
    bf16x8 wf[2], wb[2];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int k = 16 * st + 8 * hi + v;
            wf[st][v] = (__bf16)((lo < NH && k < DIM) ? P[P_W0 + lo * DIM + k] : 0.0f);
            wb[st][v] = (__bf16)((k < NH && lo < DIM) ? P[P_W0 + k * DIM + lo] : 0.0f);
        }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&L->q[32 * T + lo][16 * st + 8 * hi]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[st], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) L->z[32 * T + lo][8 * (v >> 2) + 4 * hi + (v & 3)] = acc[v];
    }
    __builtin_amdgcn_wave_barrier();
    float U = -P[P_B1];
    float dz[32];
#pragma unroll
    for (int mu = 0; mu < 32; ++mu) {
        if (mu < NH) {
            const float th = ftanh(L->z[lane][mu] - P[P_B0 + mu]);
            U = fmaf(P[P_W1 + mu], th, U);
            dz[mu] = P[P_W1 + mu] * fmaf(-th, th, 1.0f);
        } else {
            dz[mu] = 0.0f;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mu = 0; mu < 32; ++mu) L->q[lane][mu] = (__bf16)dz[mu];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&L->q[32 * T + lo][16 * st + 8 * hi]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wb[st], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) L->z[32 * T + lo][8 * (v >> 2) + 4 * hi + (v & 3)] = acc[v];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) Fp[nu] = L->z[lane][nu] * P[P_QS + nu];
    __builtin_amdgcn_wave_barrier();
    return U;
}

// The same two products with FP32 operands on the matrix cores
// (v_mfma_f32_32x32x2_f32: exact FP32 products, FP32 accumulation), sixteen
// K steps of two per 32 x 32 tile.  Operand layouts (lane l): A[l%32][l/32],
// B[l/32][l%32]; the result layout is that of the BF16 product.
__device__ __forceinline__ float network_mfma32(const float *__restrict__ P, const float q[DIM], float Fp[DIM],
                                                NNLds *L)
{
    const int lane = threadIdx.x & 63;
    const int hi = lane >> 5, lo = lane & 31;
#pragma unroll
    for (int nu = 0; nu < 32; ++nu) L->qf[lane][nu] = nu < DIM ? P[P_QS + nu] * q[nu] : 0.0f;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int k = 2 * st + hi;
            const float a = (lo < NH && k < DIM) ? P[P_W0 + lo * DIM + k] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, L->qf[32 * T + lo][k], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) L->z[32 * T + lo][8 * (v >> 2) + 4 * hi + (v & 3)] = acc[v];
    }
    __builtin_amdgcn_wave_barrier();
    float U = -P[P_B1];
    float dz[32];
#pragma unroll
    for (int mu = 0; mu < 32; ++mu) {
        if (mu < NH) {
            const float th = ftanh(L->z[lane][mu] - P[P_B0 + mu]);
            U = fmaf(P[P_W1 + mu], th, U);
            dz[mu] = P[P_W1 + mu] * fmaf(-th, th, 1.0f);
        } else {
            dz[mu] = 0.0f;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mu = 0; mu < 32; ++mu) L->qf[lane][mu] = dz[mu];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int T = 0; T < 2; ++T) {
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int k = 2 * st + hi;
            const float a = (k < NH && lo < DIM) ? P[P_W0 + k * DIM + lo] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, L->qf[32 * T + lo][k], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) L->z[32 * T + lo][8 * (v >> 2) + 4 * hi + (v & 3)] = acc[v];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) Fp[nu] = L->z[lane][nu] * P[P_QS + nu];
    __builtin_amdgcn_wave_barrier();
    return U;
}

// Descriptor, site energy, network forward and backward, the radial adjoint
// dU_i/dF_k (stored in the atom's record), and then, with
// B_{n,lm} = dU_i/ds_{n,lm} kept in registers, the gradient of U_i with
// respect to every angular pair vector, dU_i/dr_ij.  Those pair gradients are
// stored per list slot (the force kernel subtracts them at the other end of
// the pair), their sum is this atom's own angular force term, and
// -sum_j dU_i/dr_ij (x) r_ij is its angular virial.
template <int NNMODE>
__device__ __forceinline__ void descriptor_atom(
    int t, bool valid, NNLds *L, const PairConsts &pc, const double4 *__restrict__ xq, AtomRec *__restrict__ xp,
    AtomRec48 *__restrict__ xp48, const int32_t *__restrict__ bin_sorted,
    const int32_t *__restrict__ cell_of, const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, const double *__restrict__ C64, float4 *__restrict__ pair_grad,
    float4 *__restrict__ f_own, float *__restrict__ w_atom, double *__restrict__ e_atom,
    int32_t *__restrict__ status, int cand_mode)
{
    // With the MFMA hidden layer every lane of a wave takes part; lanes past
    // the last atom compute on an empty neighbourhood of atom 0 and store nothing.
    if (!valid) t = 0;
    const double4 pi = xq[t];
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const CellGeom *cg = cells + cell_of[t];
    const int base = cg->atom_start;
    const uint32_t cnt = valid ? ncnt[t] : 0u;
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
    const int nA = naf + nab;

    float csA[NA];
    angular_coef_sums(P, csA);
    float F[KB];
    float S[NA][NLM];
    double ezbl;
    bool overlap;
    descriptor_sums(pc, xq, t, xi, yi, zi, cg, base, nl_ang, nl_rad, naf, nab, nrf, nrb, C64, F, S, ezbl,
                    overlap, cand_mode);
    if (overlap) latch_error(status, -4);
    float q[DIM];
    descriptor_vector(P, F, S, q);
    float Fp[DIM];
    const float U = NNMODE == 1 ? network_mfma(P, q, Fp, L)
                                : (NNMODE == 2 ? network_mfma32(P, q, Fp, L) : network(P, q, Fp));
    if (!valid) return;
    e_atom[t] = (double)U + ezbl;
    // this atom's record for the force kernel: position and radial adjoint
    // a_k = dU_i / dF_k, written whole (four 16-byte stores)
    AtomRec rec;
    rec.x = xi;
    rec.y = yi;
    rec.z = zi;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int n = 0; n < NR; ++n) s = fmaf(Fp[n], P[P_CR + n * KB + k], s);
        rec.a[k] = s;
    }
    rec.pad = 0.0f;
    if (xp48) {
        // bin-offset mode: the position as fixed-point offsets from the
        // corner of the atom's bin at the last build (an offset out of the
        // 32-bit range means the atom moved far beyond the list skin)
        const int lbin = bin_sorted[t];
        const int b0 = lbin % cg->nb[0], b1 = (lbin / cg->nb[0]) % cg->nb[1], b2 = lbin / (cg->nb[0] * cg->nb[1]);
        const double *bv = cg->bv;
        const double p[3] = {xi - (b0 * bv[0] + b1 * bv[3] + b2 * bv[6]), yi - (b0 * bv[1] + b1 * bv[4] + b2 * bv[7]),
                             zi - (b0 * bv[2] + b1 * bv[5] + b2 * bv[8])};
        AtomRec48 r48;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = rint(p[d] * pc.qsinv);
            if (!(fabs(v) < 2147483000.0)) latch_error(status, -9);
            r48.o[d] = (int32_t)fmin(fmax(v, -2147483000.0), 2147483000.0);
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) r48.a[k] = rec.a[k];
        xp48[t] = r48;
    } else {
        xp[t] = rec;
    }
    // angular adjoint B_{n,lm} = 2 (dU/dq_nl) s_{n,lm}, in place of S, times
    // the harmonic's normalisation (the walk below uses the unnormalised
    // polynomials y_lm = Y_lm / sph_norm(lm))
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
            S[n][lm] *= (2.0f * sph_norm(lm)) * Fp[NR + NA * (l - 1) + n];
        }

    // angular pair gradients dU_i/dr_ij = grad_r [sum_{n,lm} B_{n,lm} g_n(|r|) Y_lm(r/|r|)]
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    float W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = 0.0f;
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    // the entries within the write radius only (the first walk's mask):
    // a slot left out is one the other end never reads
    for (MaskPipe q(pc.amask, nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
        // compiler barrier: the 50 angular coefficients are reloaded by
        // scalar loads in every trip instead of being hoisted into scalar
        // registers that then spill to vector-register lanes (one VALU
        // readlane per use); 616 instead of 633 VALU instructions per pair
        asm volatile("" ::: "memory");
        int32_t e;
        double px, py, pz;
        int s;
        q.pop(nl_ang, xq, base, jmask, e, px, py, pz, s);
        const size_t off = q.off(s);
        double ddx, ddy, ddz;
        pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, ddx, ddy, ddz);
        const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_ang2) {
            // outside the angular cutoff; just outside, the other end may
            // still read this slot and subtracts a zero
            if (r2 < pc.rc_ang2_write) pair_grad[off] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            continue;
        }
        // distance and Chebyshev argument from the FP64 pair vector (a
        // rounded x would be amplified by up to k^2 and k^4 near x = -1, where
        // the outer neighbour shells sit)
        const double rd = dist_d(ddx * ddx + ddy * ddy + ddz * ddz);
        const double ttd = rd * (1.0 / (double)pc.rc_ang) - 1.0;
        // 1/r and the unit vector from the FP64 pair vector as well (one
        // Newton step on the FP32 reciprocal), each rounded once: near a
        // lattice site the pair gradients cancel to a few per cent, and a
        // unit vector formed in FP32 was the largest remaining error there
        double rinvd = (double)frcp((float)rd);
        rinvd = rinvd * fma(-rd, rinvd, 2.0);
        const float rinv = (float)rinvd;
        const float tt = (float)ttd;
        float fc, dfc;
        cutoff(tt, pc.inv_rc_ang, fc, dfc);
        const float dxdr = 4.0f * tt * pc.inv_rc_ang;
        float T[KB], dT[KB];
        cheb_d_from_d(fma(2.0 * ttd, ttd, -1.0), T, dT);
        float g[NA], gp[NA];
        const float hfc = 0.5f * fc, hdx = hfc * dxdr, hdfc = 0.5f * dfc;
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float sn = csA[n], sp = 0.0f;
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                sn = fmaf(P[P_CA + n * KB + k], T[k], sn);
                sp = fmaf(P[P_CA + n * KB + k], dT[k], sp);
            }
            g[n] = hfc * sn;
            gp[n] = fmaf(hdx, sp, hdfc * sn);
        }
        const float ux = (float)(ddx * rinvd), uy = (float)(ddy * rinvd), uz = (float)(ddz * rinvd);
        const SphMono mono(ux, uy, uz);
        float Y[NLM];
        sph_unnorm(mono, Y);
        float Dc[NLM];
        // D_lm = sum_n B_{n,lm} g_n for the angular part of the gradient; the
        // radial part s1 = sum_lm (sum_n B_{n,lm} g'_n) y_lm is taken as
        // sum_n g'_n E_n with E_n = sum_lm B_{n,lm} y_lm (fewer products)
        float En[NA];
#pragma unroll
        for (int n = 0; n < NA; ++n) En[n] = 0.0f;
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) {
            float D = 0.0f;
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                D = fmaf(S[n][lm], g[n], D);
                En[n] = fmaf(S[n][lm], Y[lm], En[n]);
            }
            Dc[lm] = D;
        }
        float s1 = 0.0f;
#pragma unroll
        for (int n = 0; n < NA; ++n) s1 = fmaf(gp[n], En[n], s1);
        float vx, vy, vz;
        sph_unnorm_grad_contract(mono, Dc, vx, vy, vz);
        const float uv = ux * vx + uy * vy + uz * vz;
        const float gx = fmaf(s1, ux, (vx - uv * ux) * rinv);
        const float gy = fmaf(s1, uy, (vy - uv * uy) * rinv);
        const float gz = fmaf(s1, uz, (vz - uv * uz) * rinv);
        pair_grad[off] = make_float4(gx, gy, gz, 0.0f);
        Fx += gx; Fy += gy; Fz += gz;
        W[0] = fmaf(gx, dx, W[0]); W[1] = fmaf(gx, dy, W[1]); W[2] = fmaf(gx, dz, W[2]);
        W[3] = fmaf(gy, dx, W[3]); W[4] = fmaf(gy, dy, W[4]); W[5] = fmaf(gy, dz, W[5]);
        W[6] = fmaf(gz, dx, W[6]); W[7] = fmaf(gz, dy, W[7]); W[8] = fmaf(gz, dz, W[8]);
    }
    f_own[t] = make_float4(Fx, Fy, Fz, 0.0f);
    float *w = w_atom + (size_t)t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = -W[k];
}

// Launch shapes: BS threads per block; PERSISTENT = a fixed grid whose blocks
// stride over the atom tiles (chosen per size bucket by the autotuner),
// otherwise one block per tile in XCD-aware order.  NNMODE 0: hidden layer on
// the vector ALUs in FP32; 1: on the matrix cores in BF16 (FP32 accumulation).
template <int BS, bool PERSISTENT, int NNMODE>
__global__ __launch_bounds__(BS, NNMODE == 1 ? 1 : 2) void k_descriptor(
    PairConsts pc, const double4 *__restrict__ xq, AtomRec *__restrict__ xp, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, const double *__restrict__ C64, float4 *__restrict__ pair_grad,
    float4 *__restrict__ f_own, float *__restrict__ w_atom, double *__restrict__ e_atom,
    int32_t *__restrict__ status, int ntiles, const int32_t *__restrict__ cflag,
    const int32_t *__restrict__ bin_sorted)
{
    __shared__ NNLds lds[NNMODE != 0 ? BS / 64 : 1];
    AtomRec48 *xp48 = pc.delta ? reinterpret_cast<AtomRec48 *>(xp) : nullptr;
    NNLds *L = &lds[NNMODE != 0 ? threadIdx.x / 64 : 0];
    if (lists_blocked(status)) return;
    // radial walk: in full (and the candidate mask written) when *cflag is set
    const int cand_mode = *cflag ? CAND_WRITE : CAND_READ;
    if (PERSISTENT) {
        for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int t = tile * BS + threadIdx.x;
            if (NNMODE != 0 || t < pc.n)
                descriptor_atom<NNMODE>(t, t < pc.n, L, pc, xq, xp, xp48, bin_sorted, cell_of, cells, nl_ang, nl_rad, ncnt,
                                        P, C64, pair_grad,
                                        f_own, w_atom, e_atom, status, cand_mode);
        }
    } else {
        const int tile = xcd_block(ntiles);
        const int t = tile * BS + threadIdx.x;
        if (tile < ntiles && (NNMODE != 0 || t < pc.n))
            descriptor_atom<NNMODE>(t, t < pc.n, L, pc, xq, xp, xp48, bin_sorted, cell_of, cells, nl_ang, nl_rad, ncnt,
                                    P, C64, pair_grad,
                                    f_own, w_atom, e_atom, status, cand_mode);
    }
}

// ------------------------------------------------------------------ forces + virial

// Radial + ZBL force of one pair from its FP64 pair vector d = r_j - r_i and
// both ends' radial adjoints: (a^i + a^j) . f'(r) d/r + U'_ZBL(r) d/r, added to
// F and, as its outer product with d, to W.  The distance, the Chebyshev
// argument x = 2 (r/rc - 1)^2 - 1, the series T_k, dT_k and their sums with
// the adjoints are in FP64: near x = -1, where the outer neighbour shells sit,
// the recurrences amplify a rounding of x by up to k^2 in T_k and k^4 in
// dT_k, and close to a lattice site the net force is a small difference of
// such pair terms.  The cutoff factor and the products with d are FP32, the
// force sums FP64.  Returns false (and adds nothing) outside rc_rad; r2out
// receives |d|^2.
__device__ __forceinline__ bool radial_pair_force(const PairConsts &pc, double dx, double dy, double dz,
                                                  const float ai[KB], const float aj[KB], double &Fx, double &Fy,
                                                  double &Fz, float W[9], float &r2out)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    r2out = (float)r2;
    const double rc = (double)pc.rc_rad;
    if (r2 >= rc * rc) return false;
    const double r = dist_d(r2);
    const double inv = 1.0 / rc;
    const double tt = r * inv - 1.0;
    float fc, dfc;
    cutoff((float)tt, pc.inv_rc_rad, fc, dfc);
    const double x = 2.0 * tt * tt - 1.0, x2 = 2.0 * x;
    double Tm2 = 1.0, Tm1 = x, dTm2 = 0.0, dTm1 = 1.0;
    double ah = (double)ai[0] + (double)aj[0];
    double s0 = ah, s1 = 0.0, sa = ah;
    ah = (double)ai[1] + (double)aj[1];
    s0 = fma(ah, x, s0);
    s1 += ah;
    sa += ah;
#pragma unroll
    for (int k = 2; k < KB; ++k) {
        const double T = fma(x2, Tm1, -Tm2);
        const double dT = fma(x2, dTm1, fma(2.0, Tm1, -dTm2));
        ah = (double)ai[k] + (double)aj[k];
        s0 = fma(ah, T, s0);
        s1 = fma(ah, dT, s1);
        sa += ah;
        Tm2 = Tm1; Tm1 = T; dTm2 = dTm1; dTm1 = dT;
    }
    double dGdr = 0.5 * (4.0 * tt * inv * (double)fc * s1 + (double)dfc * (s0 + sa));
    if (r < (double)pc.zbl_r2) {
        double U, dU;
        zbl_pair(r, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
        dGdr += dU;
    }
    double rinv = (double)frcp((float)r);
    rinv = rinv * fma(-r, rinv, 2.0);
    rinv = rinv * fma(-r, rinv, 2.0);
    const float c = (float)(dGdr * rinv);
    const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
    const float px = c * fdx, py = c * fdy, pz = c * fdz;
    Fx += px; Fy += py; Fz += pz;
    W[0] = fmaf(px, fdx, W[0]); W[1] = fmaf(px, fdy, W[1]); W[2] = fmaf(px, fdz, W[2]);
    W[3] = fmaf(py, fdx, W[3]); W[4] = fmaf(py, fdy, W[4]); W[5] = fmaf(py, fdz, W[5]);
    W[6] = fmaf(pz, fdx, W[6]); W[7] = fmaf(pz, fdy, W[7]); W[8] = fmaf(pz, fdz, W[8]);
    return true;
}

// F_i = sum_j (a^i + a^j) . f'(r_ij) u_ij + U'_ZBL(r_ij) u_ij        (radial + ZBL)
//     + sum_j [dU_i/dr_ij - dU_j/dr_ji]_angular                       (stored pair gradients)
// and the radial + ZBL virial -1/2 sum_j f_ij (x) r_ij added to the angular one.
// Each neighbour costs one 64-byte record gather (position and adjoint) and,
// for angular entries, one 16-byte pair-gradient gather.
// D48: bin-offset mode, 48-byte records (AtomRec48): the pair vector is the
// sum of the neighbour bin's edge vectors (from the block's LDS table btab)
// and the difference of the two fixed-point offsets, exactly antisymmetric
// as the FP64 positions' one.
template <bool D48>
__device__ __forceinline__ void force_atom(
    int t, const PairConsts &pc, const AtomRec *__restrict__ xp_, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const uint8_t *__restrict__ rev, const float4 *__restrict__ pair_grad, const float4 *__restrict__ f_own,
    const int32_t *__restrict__ perm, float *__restrict__ fx, float *__restrict__ fy,
    float *__restrict__ fz, float *__restrict__ w_atom, int32_t *__restrict__ status,
    const double *__restrict__ btab)
{
    using Rec = typename std::conditional<D48, AtomRec48, AtomRec>::type;
    const Rec *__restrict__ xp = reinterpret_cast<const Rec *>(xp_);
    const Rec own = xp[t];
    const CellGeom *cg = cells + cell_of[t];
    const int base = cg->atom_start;
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;

    float ai[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) ai[k] = own.a[k];
    const float4 fo = f_own[t];
    double Fx = fo.x, Fy = fo.y, Fz = fo.z;
    float W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = 0.0f;
    bool bad = false;

    // radial + ZBL force of one pair (both ends); returns false outside rc_rad
    auto radial = [&](int32_t e, const Rec &rj, float &r2out) -> bool {
        double ddx, ddy, ddz;
        if constexpr (D48) {
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
        return radial_pair_force(pc, ddx, ddy, ddz, ai, rj.a, Fx, Fy, Fz, W, r2out);
    };

    // both lists are software-pipelined: entries (and reverse slots) two
    // neighbours ahead, the neighbour's record one ahead
    const uint32_t jmask = (1u << pc.jbits) - 1u;
    const int nA = naf + nab;
    ListWalk wa(t, pc.n, naf, nab, pc.capA);
    int32_t e_cur = 0, e_nx = 0;
    int sj_cur = 255, sj_nx = 255;
    Rec r_cur;
    if (nA > 0) {
        e_cur = nl_ang[wa.off];
        sj_cur = rev[wa.off];
        r_cur = xp[(int)((uint32_t)e_cur & jmask) + base];
    }
    wa.next();
    if (wa.s < nA) { e_nx = nl_ang[wa.off]; sj_nx = rev[wa.off]; }
    for (int s = 0; s < nA; ++s) {
        const int32_t e = e_cur;
        const int sj = sj_cur;
        const Rec rj = r_cur;
        if (s + 1 < nA) {
            e_cur = e_nx;
            sj_cur = sj_nx;
            r_cur = xp[(int)((uint32_t)e_cur & jmask) + base];
            wa.next();
            if (wa.s < nA) { e_nx = nl_ang[wa.off]; sj_nx = rev[wa.off]; }
        }
        float r2;
        if (!radial(e, rj, r2) || r2 >= pc.rc_ang2_read) continue;
        // angular: subtract the other end's stored dU_j/dr_ji (zero outside rc_ang)
        if (sj == 255) { bad = true; continue; }
        const int j = (int)((uint32_t)e & jmask) + base;
        const float4 gj = pair_grad[(size_t)sj * pc.n + j];
        Fx -= gj.x; Fy -= gj.y; Fz -= gj.z;
    }
    // radial list: only the entries the descriptor kernel found inside
    // rc_rad (the skin entries are not loaded); entries two ahead, the
    // neighbour's record one ahead
    const size_t nsz = (size_t)pc.n;
    auto rad_off = [&](int s) { return (size_t)list_slot(s, nrf, nrb, pc.capR) * nsz + t; };
    MaskWalk mr(pc.rmask, pc.n, t, nrf + nrb);
    int s_cur = mr.next();
    e_nx = 0;
    if (s_cur >= 0) {
        e_cur = nl_rad[rad_off(s_cur)];
        r_cur = xp[(int)((uint32_t)e_cur & jmask) + base];
    }
    int s_nx = mr.next();
    if (s_nx >= 0) e_nx = nl_rad[rad_off(s_nx)];
    while (s_cur >= 0) {
        const int32_t e = e_cur;
        const Rec rj = r_cur;
        s_cur = s_nx;
        if (s_cur >= 0) {
            e_cur = e_nx;
            r_cur = xp[(int)((uint32_t)e_cur & jmask) + base];
            s_nx = mr.next();
            if (s_nx >= 0) e_nx = nl_rad[rad_off(s_nx)];
        }
        float r2;
        radial(e, rj, r2);
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

// (three waves per SIMD: the FP64 pair term needs more registers than the
// default allocation for this block size would leave)
template <int BS, bool PERSISTENT, bool D48>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void k_force(
    PairConsts pc, const AtomRec *__restrict__ xp, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const uint8_t *__restrict__ rev, const float4 *__restrict__ pair_grad, const float4 *__restrict__ f_own,
    const int32_t *__restrict__ perm, float *__restrict__ fx, float *__restrict__ fy,
    float *__restrict__ fz, float *__restrict__ w_atom, int32_t *__restrict__ status, int ntiles)
{
    __shared__ __align__(16) double btab[D48 ? BIN_TAB : 2];
    if constexpr (D48) stage_bin_vectors(cells, btab);   // one cell in this mode
    if (lists_blocked(status)) return;
    if (PERSISTENT) {
        for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int t = tile * BS + threadIdx.x;
            if (t < pc.n)
                force_atom<D48>(t, pc, xp, cell_of, cells, nl_ang, nl_rad, ncnt, rev, pair_grad, f_own, perm, fx,
                                fy, fz, w_atom, status, btab);
        }
    } else {
        const int tile = xcd_block(ntiles);
        const int t = tile * BS + threadIdx.x;
        if (tile < ntiles && t < pc.n)
            force_atom<D48>(t, pc, xp, cell_of, cells, nl_ang, nl_rad, ncnt, rev, pair_grad, f_own, perm, fx, fy,
                            fz, w_atom, status, btab);
    }
}

// Instantiated launch shapes.
#define NEP_SHAPES(X) X(64, false) X(128, false) X(256, false) X(64, true) X(128, true) X(256, true)
#define NEP_INST(BS, PE)                                                                                           \
    template __global__ void k_descriptor<BS, PE, 0>(PairConsts, const double4 *, AtomRec *, const int32_t *,      \
                                                     const CellGeom *,                                             \
                                                     const int32_t *, const int32_t *, const uint32_t *,           \
                                                     const float *, const double *, float4 *, float4 *, float *, double *, int32_t *, \
                                                     int, const int32_t *, const int32_t *);                                          \
    template __global__ void k_descriptor<BS, PE, 1>(PairConsts, const double4 *, AtomRec *, const int32_t *,      \
                                                     const CellGeom *,                                             \
                                                     const int32_t *, const int32_t *, const uint32_t *,           \
                                                     const float *, const double *, float4 *, float4 *, float *, double *, int32_t *, \
                                                     int, const int32_t *, const int32_t *);                                          \
    template __global__ void k_descriptor<BS, PE, 2>(PairConsts, const double4 *, AtomRec *, const int32_t *,      \
                                                     const CellGeom *,                                             \
                                                     const int32_t *, const int32_t *, const uint32_t *,           \
                                                     const float *, const double *, float4 *, float4 *, float *, double *, int32_t *, \
                                                     int, const int32_t *, const int32_t *);                                          \
    template __global__ void k_force<BS, PE, false>(PairConsts, const AtomRec *, const int32_t *, const CellGeom *, \
                                                    const int32_t *, const int32_t *, const uint32_t *,            \
                                                    const uint8_t *, const float4 *, const float4 *,               \
                                                    const int32_t *, float *, float *, float *, float *, int32_t *,\
                                                    int);                                                          \
    template __global__ void k_force<BS, PE, true>(PairConsts, const AtomRec *, const int32_t *, const CellGeom *,  \
                                                   const int32_t *, const int32_t *, const uint32_t *,             \
                                                   const uint8_t *, const float4 *, const float4 *,                \
                                                   const int32_t *, float *, float *, float *, float *, int32_t *, \
                                                   int);
NEP_SHAPES(NEP_INST)
#undef NEP_INST

// Double-precision copy of the angular coefficients for the descriptor sums:
// C64 = (c^A_nk [NA][KB], sum_k c^A_nk [NA]).  One block of 64 threads.
__global__ void k_params64(const float *__restrict__ P, double *__restrict__ C64)
{
    const int i = threadIdx.x;
    if (i < NA * KB) C64[i] = (double)P[P_CA + i];
    if (i < NA) {
        double s = 0.0;
        for (int k = 0; k < KB; ++k) s += (double)P[P_CA + i * KB + k];
        C64[NA * KB + i] = s;
    }
}

// ------------------------------------------------------------------ parameter gradients

// theta = (c_rad [NR][KB], c_ang [NA][KB], w0 [NH][DIM], b0 [NH], w1 [NH], b1)
constexpr int NPARAM = NR * KB + NA * KB + NH * DIM + NH + NH + 1;
constexpr int PG_TILE = 64;
// Per-atom factors of the two outer-product blocks, kept in LDS per tile:
// g dz_mu, s q (unweighted), g dU/dq_n (radial), F_k (unweighted).  The
// row stride is odd (no bank conflicts) and 64 rows take 19.7 KB, so eight
// one-wave blocks fit a CU.
constexpr int PG_DZ = 0, PG_QT = PG_DZ + NH, PG_FPR = PG_QT + DIM, PG_F = PG_FPR + NR, PG_REC = PG_F + KB;
// Tile sums of the factors that enter the gradient linearly: g tanh z_mu,
// g G_nk, g (one value per tile, summed across the wave in a fixed order).
constexpr int PS_TH = 0, PS_G = PS_TH + NH, PS_W = PS_G + NA * KB, PS_N = PS_W + 1;

// Gradient of sum_i gE[cell(i)] U_i with respect to theta.  Per atom:
//   dU/dw1_mu = tanh z_mu, dU/db0_mu = -dz_mu, dU/dw0_mu,nu = dz_mu s_nu q_nu,
//   dU/db1 = -1, dU/dc^R_nk = (dU/dq_n) F_k,
//   dU/dc^A_nk = sum_{lm} B_{n,lm} sum_j f_k(r_ij) Y_lm(u_ij)   (B = dU/ds_{n,lm}),
// with dz_mu = w1_mu (1 - tanh^2 z_mu).  64-atom tiles, one wavefront each:
// the factors of the outer products go to LDS and every thread sums its own
// outputs (o = lane + 64 k) over the tile; the linear factors are summed
// across the wave.  Lanes past the last atom evaluate atom 0 with weight 0.
// One FP64 partial per block and output, reduced afterwards in order.
__global__ __launch_bounds__(64) void k_param_grad(
    PairConsts pc, const double4 *__restrict__ xq, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt, const float *__restrict__ P,
    const double *__restrict__ C64, const double *__restrict__ gE, double *__restrict__ part, int32_t *__restrict__ status, int ntiles)
{
    __shared__ float rec[PG_TILE][PG_REC];
    __shared__ float tsum[PS_N];
    constexpr int NOWN = (NPARAM + PG_TILE - 1) / PG_TILE;
    const int lane = threadIdx.x;
    double *pb = part + (size_t)blockIdx.x * NPARAM;   // this block's partials, added tile by tile
    const bool ok = !lists_blocked(status);
    for (int k = 0; k < NOWN; ++k) {
        const int o = lane + PG_TILE * k;
        if (o < NPARAM) pb[o] = 0.0;
    }
    float csA[NA];
    angular_coef_sums(P, csA);

    for (int tile = blockIdx.x; tile < ntiles && ok; tile += gridDim.x) {
        const bool valid = tile * PG_TILE + lane < pc.n;
        const int t = valid ? tile * PG_TILE + lane : 0;
        float *r = rec[lane];
        const double4 pi = xq[t];
        const double xi = pi.x, yi = pi.y, zi = pi.z;
        const CellGeom *cg = cells + cell_of[t];
        const int base = cg->atom_start;
        const uint32_t cnt = ncnt[t];
        const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
        const float g = valid ? (float)gE[cell_of[t]] : 0.0f;
        float F[KB];
        float S[NA][NLM];
        double ezbl;
        bool overlap;
        descriptor_sums(pc, xq, t, xi, yi, zi, cg, base, nl_ang, nl_rad, naf, nab, nrf, nrb, C64, F, S, ezbl,
                        overlap, CAND_OFF);
        float q[DIM];
        descriptor_vector(P, F, S, q);
        // network with the per-neuron factors (outer-product ones to LDS,
        // tanh summed over the tile)
        float Fp[DIM];
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) {
            Fp[nu] = 0.0f;
            r[PG_QT + nu] = P[P_QS + nu] * q[nu];
        }
#pragma unroll 1
        for (int mu = 0; mu < NH; ++mu) {
            const float *w = P + P_W0 + mu * DIM;
            float z = -P[P_B0 + mu];
#pragma unroll
            for (int nu = 0; nu < DIM; ++nu) z = fmaf(w[nu], P[P_QS + nu] * q[nu], z);
            const float th = ftanh(z);
            const float dz = P[P_W1 + mu] * fmaf(-th, th, 1.0f);
            const float sth = wave_sum64(g * th);
            if (lane == 0) tsum[PS_TH + mu] = sth;
            r[PG_DZ + mu] = g * dz;
#pragma unroll
            for (int nu = 0; nu < DIM; ++nu) Fp[nu] = fmaf(dz, w[nu], Fp[nu]);
        }
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) Fp[nu] *= P[P_QS + nu];
#pragma unroll
        for (int n = 0; n < NR; ++n) r[PG_FPR + n] = g * Fp[n];
#pragma unroll
        for (int k = 0; k < KB; ++k) r[PG_F + k] = F[k];
        // B = 2 (dU/dq_nl) s_{n,lm} in place of S
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int lm = 0; lm < NLM; ++lm) {
                const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
                S[n][lm] *= 2.0f * Fp[NR + NA * (l - 1) + n];
            }
        // G_nk = sum_j f_k(r_ij) sum_lm B_{n,lm} Y_lm(u_ij)
        float G[NA][KB];
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int k = 0; k < KB; ++k) G[n][k] = 0.0f;
        // the entries the first angular walk above marked (within the write
        // radius), software-pipelined
        const uint32_t jmask = (1u << pc.jbits) - 1u;
        for (MaskPipe q(pc.amask, nl_ang, xq, base, jmask, t, pc.n, naf, nab, pc.capA); q.valid();) {
            int32_t e;
            double px, py, pz;
            int s;
            q.pop(nl_ang, xq, base, jmask, e, px, py, pz, s);
            double ddx, ddy, ddz;
            pair_vector_p(e, pc, px, py, pz, xi, yi, zi, cg, ddx, ddy, ddz);
            const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= pc.rc_ang2) continue;
            const float rr = fsqrt(r2);
            const float rinv = frcp(rr);
            const float tt = scaled_minus_one(rr, pc.inv_rc_ang, pc.inv_rc_ang_lo);
            float fc;
            cutoff_value(tt, fc);
            float T[KB];
            cheb(fmaf(2.0f * tt, tt, -1.0f), T);
            float Y[NLM];
            sph(dx * rinv, dy * rinv, dz * rinv, Y);
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float D = 0.0f;
#pragma unroll
                for (int lm = 0; lm < NLM; ++lm) D = fmaf(S[n][lm], Y[lm], D);
                const float hD = 0.5f * fc * D;      // f_k = (T_k + 1) fc / 2
#pragma unroll
                for (int k = 0; k < KB; ++k) G[n][k] = fmaf(hD, T[k] + 1.0f, G[n][k]);
            }
        }
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const float sg = wave_sum64(g * G[n][k]);
                if (lane == 0) tsum[PS_G + n * KB + k] = sg;
            }
        const float sw = wave_sum64(g);
        if (lane == 0) tsum[PS_W] = sw;
        __syncthreads();
        for (int k = 0; k < NOWN; ++k) {
            const int o = lane + PG_TILE * k;
            if (o >= NPARAM) break;
            float sum = 0.0f;
            if (o < NR * KB) {
                const int i1 = PG_FPR + o / KB, i2 = PG_F + o % KB;
                for (int a = 0; a < PG_TILE; ++a) sum = fmaf(rec[a][i1], rec[a][i2], sum);
            } else if (o < NR * KB + NA * KB) {
                sum = tsum[PS_G + (o - NR * KB)];
            } else if (o < NR * KB + NA * KB + NH * DIM) {
                const int p = o - NR * KB - NA * KB;
                const int i1 = PG_DZ + p / DIM, i2 = PG_QT + p % DIM;
                for (int a = 0; a < PG_TILE; ++a) sum = fmaf(rec[a][i1], rec[a][i2], sum);
            } else if (o < NR * KB + NA * KB + NH * DIM + NH) {
                const int i1 = PG_DZ + (o - (NPARAM - 1 - 2 * NH));
                for (int a = 0; a < PG_TILE; ++a) sum += rec[a][i1];
                sum = -sum;
            } else if (o < NPARAM - 1) {
                sum = tsum[PS_TH + (o - (NPARAM - 1 - NH))];
            } else {
                sum = -tsum[PS_W];
            }
            pb[o] += (double)sum;
        }
        __syncthreads();
    }
}

// grad[o] = sum over blocks of part[b][o] in a fixed order (deterministic):
// a block of 256 threads takes 32 consecutive outputs; thread (c, p) sums the
// partials b = c, c + 8, c + 16, ... of output p (each step reads 32
// consecutive doubles per c), and the eight chunk sums of an output are then
// added in chunk order.
// Rows of `nparam` doubles (either model's parameter count).
__global__ __launch_bounds__(256) void k_param_reduce(int nblocks, int nparam, const double *__restrict__ part,
                                                      double *__restrict__ grad)
{
    __shared__ double sh[8][33];
    const int p = threadIdx.x & 31, c = threadIdx.x >> 5;
    const int o = blockIdx.x * 32 + p;
    double s = 0.0;
    if (o < nparam) {
#pragma unroll 4
        for (int b = c; b < nblocks; b += 8) s += part[(size_t)b * nparam + o];
    }
    sh[c][p] = s;
    __syncthreads();
    if (c == 0 && o < nparam) {
        double t = sh[0][p];
#pragma unroll
        for (int k = 1; k < 8; ++k) t += sh[k][p];
        grad[o] = t;
    }
}

// dL/dx_i = -gE[cell(i)] F_i (caller order, FP64).
__global__ void k_grad_pos(int n, const int32_t *__restrict__ cell_of, const double *__restrict__ gE,
                           const float *__restrict__ fx, const float *__restrict__ fy,
                           const float *__restrict__ fz, double *__restrict__ gx, double *__restrict__ gy,
                           double *__restrict__ gz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = gE[cell_of[i]];
    gx[i] = -g * fx[i];
    gy[i] = -g * fy[i];
    gz[i] = -g * fz[i];
}

// dL/dh of every cell at fixed Cartesian positions:
//   dE/dh = h^-T (sum_i x_i (x) F_i - W^T),  times gE[c].
// One block per cell (caller order; a cell's atoms are contiguous).
__global__ __launch_bounds__(256) void k_grad_cell(const CellGeom *__restrict__ cells,
                                                   const double *__restrict__ x, const double *__restrict__ y,
                                                   const double *__restrict__ z, const float *__restrict__ fx,
                                                   const float *__restrict__ fy, const float *__restrict__ fz,
                                                   const double *__restrict__ virial,
                                                   const double *__restrict__ gE, double *__restrict__ gh)
{
    __shared__ double sh[9][256];
    const CellGeom &cg = cells[blockIdx.x];
    double m[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) m[q] = 0.0;
    for (int i = cg.atom_start + threadIdx.x; i < cg.atom_start + cg.n_atoms; i += 256) {
        const double p[3] = {x[i], y[i], z[i]};
        const double f[3] = {fx[i], fy[i], fz[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) m[3 * a + b] += p[a] * f[b];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) sh[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 9; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double *W = virial + (size_t)blockIdx.x * 9;
        double A[9];   // M - W^T
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[3 * a + b] = sh[3 * a + b][0] - W[3 * b + a];
        const double g = gE[blockIdx.x];
        // (h^-T A)_ab = sum_c hinv[c][a] A[c][b]
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                for (int c = 0; c < 3; ++c) v += cg.hinv[3 * c + a] * A[3 * c + b];
                gh[(size_t)blockIdx.x * 9 + 3 * a + b] = g * v;
            }
    }
}

// ------------------------------------------------------------------ reductions

// One block per chunk of atoms of a single cell: FP64 sums of the site
// energies and the per-atom virials, written to part[chunk][10].
__device__ __forceinline__ void reduce_chunk(int k, const int32_t *__restrict__ chunk_begin,
                                             const int32_t *__restrict__ chunk_end,
                                             const double *__restrict__ e_atom, const float *__restrict__ w_atom,
                                             double *__restrict__ part, bool ok)
{
    __shared__ double sh[10][256];
    double acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    if (ok) {
        for (int t = chunk_begin[k] + threadIdx.x; t < chunk_end[k]; t += 256) {
            acc[0] += e_atom[t];
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[1 + q] += (double)w_atom[(size_t)t * 9 + q];
        }
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 10; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 10) part[(size_t)k * 10 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_reduce_chunks(const int32_t *__restrict__ chunk_begin,
                                                       const int32_t *__restrict__ chunk_end,
                                                       const double *__restrict__ e_atom,
                                                       const float *__restrict__ w_atom,
                                                       double *__restrict__ part,
                                                       const int32_t *__restrict__ status)
{
    reduce_chunk(blockIdx.x, chunk_begin, chunk_end, e_atom, w_atom, part, status[ST_ERR] == 0);
}

// One block per cell: sum of its chunk partials (fixed order: strided
// partial sums per thread, then a fixed tree), deterministic.
__device__ __forceinline__ void reduce_cell(int c, const int32_t *__restrict__ cell_chunk,
                                            const double *__restrict__ part, double *__restrict__ energy,
                                            double *__restrict__ virial)
{
    __shared__ double sh[10][256];
    double acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    for (int k = cell_chunk[c] + threadIdx.x; k < cell_chunk[c + 1]; k += 256)
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] += part[(size_t)k * 10 + q];
#pragma unroll
    for (int q = 0; q < 10; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 10; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) energy[c] = sh[0][0];
    if (virial && threadIdx.x < 9) virial[(size_t)c * 9 + threadIdx.x] = sh[1 + threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_reduce_cells(int n_cells, const int32_t *__restrict__ cell_chunk,
                                                      const double *__restrict__ part, double *__restrict__ energy,
                                                      double *__restrict__ virial,
                                                      const int32_t *__restrict__ status)
{
    const int c = blockIdx.x;
    if (c >= n_cells) return;
    if (status[ST_ERR] != 0) return;
    reduce_cell(c, cell_chunk, part, energy, virial);
}

// Site energies to the caller's order (FP32 output).
__global__ void k_energy_atom_out(int n, const int32_t *__restrict__ perm,
                                  const double *__restrict__ e_atom, float *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[perm[t]] = (float)e_atom[t];
}

// Neighbour counts inside the cutoffs (diagnostics for flop accounting).
__global__ __launch_bounds__(256) void k_count_inside(
    PairConsts pc, const double4 *__restrict__ xq, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    unsigned long long *__restrict__ counts)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nr = 0, na = 0;
    if (t < pc.n) {
        const double xi = xq[t].x, yi = xq[t].y, zi = xq[t].z;
        const CellGeom *cg = cells + cell_of[t];
        const uint32_t cnt = ncnt[t];
        const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
        const double rcR2 = (double)pc.rc_rad * pc.rc_rad, rcA2 = (double)pc.rc_ang * pc.rc_ang;
        for (int s = 0; s < naf + nab; ++s) {
            int j;
            double dx, dy, dz;
            pair_vector_d(nl_ang[(size_t)list_slot(s, naf, nab, pc.capA) * pc.n + t], pc, cg->atom_start,
                          xi, yi, zi, xq, cg, j, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            nr += r2 < rcR2;
            na += r2 < rcA2;
        }
        for (int s = 0; s < nrf + nrb; ++s) {
            int j;
            double dx, dy, dz;
            pair_vector_d(nl_rad[(size_t)list_slot(s, nrf, nrb, pc.capR) * pc.n + t], pc, cg->atom_start,
                          xi, yi, zi, xq, cg, j, dx, dy, dz);
            nr += (dx * dx + dy * dy + dz * dz) < rcR2;
        }
    }
    // wave-level sum, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        nr += __shfl_xor(nr, off);
        na += __shfl_xor(na, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(counts, nr);
        atomicAdd(counts + 1, na);
    }
}


// ------------------------------------------------------------------ population (SNES)
//
// The paper trains its model by SNES with a population of 50 (Sec. III.A):
// every generation evaluates energies, forces and virials of the whole
// training set for each member.  Here one launch covers all members: work
// item w (in XCD order over ntiles * n_pop) is member w % n_pop of atom tile
// w / n_pop, so the members of one tile run side by side on one XCD and
// share its L2 for positions and lists.  Member m reads its parameters at
// P + m P_SIZE (C64 + m C64N) and owns records, pair gradients, own terms,
// per-atom virials and energies at offset m (per-atom array size).

// theta [n_pop][NPARAM] (c_rad, c_ang, w0, b0, w1, b1) -> parameter blocks
// [n_pop][P_SIZE] with the descriptor scale q_scale of `base`, and the FP64
// angular coefficients [n_pop][C64N].  One block per member.
__global__ __launch_bounds__(256) void k_pop_params(const float *__restrict__ theta, const float *__restrict__ base,
                                                    float *__restrict__ P, double *__restrict__ C64)
{
    const int m = blockIdx.x;
    const float *th = theta + (size_t)m * NPARAM;
    float *pm = P + (size_t)m * P_SIZE;
    for (int i = threadIdx.x; i < P_SIZE; i += blockDim.x)
        pm[i] = i < P_QS ? th[i] : (i < P_W0 ? base[i] : th[i - DIM]);
    double *cm = C64 + (size_t)m * C64N;
    const int i = threadIdx.x;
    if (i < NA * KB) cm[i] = (double)th[P_CA + i];
    if (i < NA) {
        double s = 0.0;
        for (int k = 0; k < KB; ++k) s += (double)th[P_CA + i * KB + k];
        cm[NA * KB + i] = s;
    }
}

__device__ inline bool pop_item(int ntiles, int n_pop, int &m, int &tile)
{
    const int w = xcd_block(ntiles * n_pop);
    if (w >= ntiles * n_pop) return false;
    m = w % n_pop;
    tile = w / n_pop;
    return true;
}

// POP_DESC_BS threads per block: 64-thread tiles, as for the single-model
// default (a block retires with its slowest wave)
__global__ __launch_bounds__(POP_DESC_BS, 2) void k_pop_descriptor(
    PairConsts pc, const double4 *__restrict__ xq, AtomRec *__restrict__ xp, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, const double *__restrict__ C64, float4 *__restrict__ pair_grad,
    float4 *__restrict__ f_own, float *__restrict__ w_atom, double *__restrict__ e_atom,
    int32_t *__restrict__ status, int ntiles, int n_pop)
{
    __shared__ NNLds lds[1];
    if (lists_blocked(status)) return;
    int m, tile;
    if (!pop_item(ntiles, n_pop, m, tile)) return;
    const int t = tile * POP_DESC_BS + threadIdx.x;
    if (t >= pc.n) return;
    const size_t n = (size_t)pc.n;
    descriptor_atom<0>(t, true, lds, pc, xq, xp + m * n, nullptr, nullptr, cell_of, cells, nl_ang, nl_rad, ncnt,
                       P + (size_t)m * P_SIZE, C64 + (size_t)m * C64N, pair_grad + (size_t)m * pc.capA * n,
                       f_own + m * n, w_atom + 9 * m * n, e_atom + m * n, status, CAND_OFF);
}

// forces of member m go to F + 3 m n (fx), + (3 m + 1) n (fy), + (3 m + 2) n (fz), caller order
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_pop_force(
    PairConsts pc, const AtomRec *__restrict__ xp, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const uint8_t *__restrict__ rev, const float4 *__restrict__ pair_grad, const float4 *__restrict__ f_own,
    const int32_t *__restrict__ perm, float *__restrict__ F, float *__restrict__ w_atom,
    int32_t *__restrict__ status, int ntiles, int n_pop)
{
    if (lists_blocked(status)) return;
    int m, tile;
    if (!pop_item(ntiles, n_pop, m, tile)) return;
    const int t = tile * 256 + threadIdx.x;
    if (t >= pc.n) return;
    const size_t n = (size_t)pc.n;
    float *fm = F + 3 * m * n;
    force_atom<false>(t, pc, xp + m * n, cell_of, cells, nl_ang, nl_rad, ncnt, rev, pair_grad + (size_t)m * pc.capA * n,
               f_own + m * n, perm, fm, fm + n, fm + 2 * n, w_atom + 9 * m * n, status, nullptr);
}

// grid (n_chunks, n_pop): chunk partials of member blockIdx.y
__global__ __launch_bounds__(256) void k_pop_reduce_chunks(int n, int n_chunks, const int32_t *__restrict__ chunk_begin,
                                                           const int32_t *__restrict__ chunk_end,
                                                           const double *__restrict__ e_atom,
                                                           const float *__restrict__ w_atom,
                                                           double *__restrict__ part,
                                                           const int32_t *__restrict__ status)
{
    const size_t m = blockIdx.y;
    reduce_chunk(blockIdx.x, chunk_begin, chunk_end, e_atom + m * n, w_atom + 9 * m * n,
                 part + m * n_chunks * 10, status[ST_ERR] == 0);
}

// grid (n_cells, n_pop): energy [n_pop][n_cells], virial [n_pop][n_cells][9]
__global__ __launch_bounds__(256) void k_pop_reduce_cells(int n_cells, int n_chunks,
                                                          const int32_t *__restrict__ cell_chunk,
                                                          const double *__restrict__ part,
                                                          double *__restrict__ energy, double *__restrict__ virial,
                                                          const int32_t *__restrict__ status)
{
    if (status[ST_ERR] != 0) return;
    const size_t m = blockIdx.y;
    reduce_cell(blockIdx.x, cell_chunk, part + m * n_chunks * 10, energy + m * n_cells,
                virial + m * n_cells * 9);
}

// Fixed-order block sum of one double (blocks of 256); every thread returns it.
__device__ inline double block_sum256(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// grid (nblk, n_pop): part[m][b] = sum over this block's atoms of |F - F_target|^2
__global__ __launch_bounds__(256) void k_pop_force_err(int n, const float *__restrict__ F,
                                                       const float *__restrict__ tfx, const float *__restrict__ tfy,
                                                       const float *__restrict__ tfz, double *__restrict__ part)
{
    __shared__ double sh[256];
    const size_t m = blockIdx.y;
    const float *fm = F + 3 * m * n;
    double acc = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double dx = (double)fm[i] - tfx[i], dy = (double)fm[n + i] - tfy[i], dz = (double)fm[2 * n + i] - tfz[i];
        acc += dx * dx + dy * dy + dz * dz;
    }
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[m * gridDim.x + blockIdx.x] = s;
}

// One block per member: the loss terms (total, RMSE of the energy per atom,
// of the force components, of the six virial components per atom over the
// cells with a virial target, mean |theta|, RMS theta) into loss[m][6].
__global__ __launch_bounds__(256) void k_pop_loss(int n_cells, int n_atoms, int n_params, int nblk,
                                                  const int64_t *__restrict__ cell_start,
                                                  const double *__restrict__ energy, const double *__restrict__ virial,
                                                  const double *__restrict__ t_energy, const double *__restrict__ t_virial,
                                                  const uint8_t *__restrict__ has_virial,
                                                  const double *__restrict__ fpart, const float *__restrict__ theta,
                                                  double le, double lf, double lv, double l1w, double l2w,
                                                  double *__restrict__ loss)
{
    __shared__ double sh[256];
    const size_t m = blockIdx.x;
    double ae = 0.0, av = 0.0, nv = 0.0, af = 0.0, a1 = 0.0, a2 = 0.0;
    for (int c = threadIdx.x; c < n_cells; c += 256) {
        const double na = (double)(cell_start[c + 1] - cell_start[c]);
        const double de = (energy[m * n_cells + c] - t_energy[c]) / na;
        ae += de * de;
        if (t_virial && (!has_virial || has_virial[c])) {
            nv += 1.0;
            const double *w = virial + (m * n_cells + c) * 9;
            const double *tw = t_virial + (size_t)c * 9;
            const int comp[6] = {0, 4, 8, 1, 5, 6};   // xx yy zz xy yz zx
            for (int q = 0; q < 6; ++q) {
                const double d = (w[comp[q]] - tw[comp[q]]) / na;
                av += d * d;
            }
        }
    }
    for (int k = threadIdx.x; k < nblk; k += 256) af += fpart[m * nblk + k];
    const float *th = theta + m * n_params;
    for (int p = threadIdx.x; p < n_params; p += 256) {
        const double z = th[p];
        a1 += fabs(z);
        a2 += z * z;
    }
    ae = block_sum256(ae, sh);
    av = block_sum256(av, sh);
    nv = block_sum256(nv, sh);
    af = block_sum256(af, sh);
    a1 = block_sum256(a1, sh);
    a2 = block_sum256(a2, sh);
    if (threadIdx.x == 0) {
        const double re = sqrt(ae / n_cells);
        const double rf = sqrt(af / (3.0 * n_atoms));
        const double rv = nv > 0.0 ? sqrt(av / (6.0 * nv)) : 0.0;
        const double r1 = a1 / n_params;
        const double r2 = sqrt(a2 / n_params);
        double *o = loss + m * 6;
        o[0] = le * re + lf * rf + lv * rv + l1w * r1 + l2w * r2;
        o[1] = re;
        o[2] = rf;
        o[3] = rv;
        o[4] = r1;
        o[5] = r2;
    }
}

// SNES: theta_k = mu + sigma * s_k (all [.][n_params], FP32).
__global__ __launch_bounds__(256) void k_snes_sample(int n_pop, int n_params, const float *__restrict__ mu,
                                                     const float *__restrict__ sigma, const float *__restrict__ s,
                                                     float *__restrict__ theta)
{
    const size_t total = (size_t)n_pop * n_params;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (size_t)gridDim.x * 256) {
        const int p = (int)(q % n_params);
        theta[q] = fmaf(sigma[p], s[q], mu[p]);
    }
}

// SNES update (Schaul et al. 2011).  Every block ranks the members by loss
// (lower is better; NaN counts as worst; ties keep the member order), turns
// ranks into utilities, then updates its share of the parameters:
// mu += eta_mu sigma sum_k u_k s_k, sigma *= exp(eta_sigma / 2 sum_k u_k (s_k^2 - 1)),
// sums in FP64 in member order.  n_pop <= 1024.
__global__ __launch_bounds__(256) void k_snes_update(int n_pop, int n_params, const double *__restrict__ loss,
                                                     int loss_stride, const float *__restrict__ s,
                                                     float *__restrict__ mu, float *__restrict__ sigma,
                                                     double eta_mu, double eta_sigma)
{
    __shared__ double u[1024];
    const double lam = (double)n_pop;
    double norm = 0.0;
    for (int r = 1; r <= n_pop; ++r) norm += fmax(0.0, log(lam / 2.0 + 1.0) - log((double)r));
    for (int k = threadIdx.x; k < n_pop; k += 256) {
        double lk = loss[(size_t)k * loss_stride];
        if (isnan(lk)) lk = INFINITY;
        int rank = 0;
        for (int j = 0; j < n_pop; ++j) {
            double lj = loss[(size_t)j * loss_stride];
            if (isnan(lj)) lj = INFINITY;
            rank += (lj < lk) || (lj == lk && j < k);
        }
        u[k] = fmax(0.0, log(lam / 2.0 + 1.0) - log((double)(rank + 1))) / norm - 1.0 / lam;
    }
    __syncthreads();
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n_params; p += gridDim.x * 256) {
        double gm = 0.0, gs = 0.0;
        for (int k = 0; k < n_pop; ++k) {
            const double sk = s[(size_t)k * n_params + p];
            gm += u[k] * sk;
            gs += u[k] * (sk * sk - 1.0);
        }
        const double sg = sigma[p];
        mu[p] = (float)((double)mu[p] + eta_mu * sg * gm);
        sigma[p] = (float)(sg * exp(0.5 * eta_sigma * gs));
    }
}

}  // namespace nep
