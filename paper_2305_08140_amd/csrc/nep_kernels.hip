// NEP-ZBL hot-path kernels for gfx950 (MI355X).
//
// Atom data live in a cell-list ("sorted") order: within every cell, atoms
// are grouped by bin, so that a 64-wide wavefront works on spatially close
// atoms and its neighbour gathers hit the same cache lines.  Positions are
// FP64 structure-of-arrays; every pair vector is formed in FP64 and rounded
// to FP32 before any further arithmetic, so that absolute coordinates of a
// 500 A box never lose precision in the pair geometry.
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
// Forces: F_i = sum_j [dU_i/dr_ij - dU_j/dr_ji].  Because Y_lm(-u) = (-1)^l Y_lm(u)
// and the radial basis depends on |r| only, both terms are the gradient at r_ij
// of ONE function:  G(r) = sum_k (a^i_k + a^j_k) f_k(|r|)
//                        + sum_{n,lm} (B^i_{n,lm} + (-1)^l B^j_{n,lm}) g_n(|r|) Y_lm(r/|r|)
// plus the ZBL term, so the force kernel evaluates one pair gradient per
// neighbour (no second evaluation for the j side) and needs no atomics: every
// atom gathers its own force, deterministically.
// Virial: W = -1/2 sum_i sum_j f_ij (x) r_ij with f_ij the pair's contribution to F_i.
#include "nep_device.h"

namespace nep {

// ------------------------------------------------------------------ helpers

__device__ inline void pair_vector(int32_t e, const PairConsts &pc, int base, double xi, double yi,
                                   double zi, const double *__restrict__ xs,
                                   const double *__restrict__ ys, const double *__restrict__ zs,
                                   const CellGeom *__restrict__ cg, int &j, float &dx, float &dy,
                                   float &dz)
{
    int n0, n1, n2;
    decode_entry(e, pc.jbits, pc.ibits, pc.ioff, j, n0, n1, n2);
    j += base;
    double ddx = xs[j] - xi, ddy = ys[j] - yi, ddz = zs[j] - zi;
    if (n0 | n1 | n2) {
        const double *h = cg->h;
        ddx += n0 * h[0] + n1 * h[3] + n2 * h[6];
        ddy += n0 * h[1] + n1 * h[4] + n2 * h[7];
        ddz += n0 * h[2] + n1 * h[5] + n2 * h[8];
    }
    dx = (float)ddx;
    dy = (float)ddy;
    dz = (float)ddz;
}

// slot of the s-th entry of a list stored front-to-back (nf entries) and
// back-to-front (nb entries) in a column of capacity cap
__device__ inline int list_slot(int s, int nf, int nb, int cap)
{
    return s < nf ? s : s + (cap - nf - nb);
}

__device__ inline float ftanh(float z)
{
    // tanh z = 1 - 2 / (exp(2z) + 1); exp via the hardware base-2 exponential
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * z);   // 2 log2(e) z
    return 1.0f - 2.0f * frcp(e + 1.0f);
}

// ------------------------------------------------------------------ descriptor + network

__global__ __launch_bounds__(256) void k_descriptor(
    PairConsts pc, const double *__restrict__ xs, const double *__restrict__ ys,
    const double *__restrict__ zs, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, float *__restrict__ adj_r, float *__restrict__ adj_a,
    double *__restrict__ e_atom, int32_t *__restrict__ status, int ntiles)
{
    const int tile = xcd_block(ntiles);
    if (tile >= ntiles) return;
    const int t = tile * 256 + threadIdx.x;
    if (t >= pc.n) return;
    if (status[ST_ERR] != 0) return;

    const double xi = xs[t], yi = ys[t], zi = zs[t];
    const CellGeom *cg = cells + cell_of[t];
    const int base = cg->atom_start;
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;

    float csA[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < KB; ++k) s += P[P_CA + n * KB + k];
        csA[n] = s;
    }

    float AR[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) AR[k] = 0.0f;
    float S[NA][NLM];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < NLM; ++lm) S[n][lm] = 0.0f;
    double ezbl = 0.0;
    bool overlap = false;

    // angular list: every entry may be inside both cutoffs
    const int nA = naf + nab;
    for (int s = 0; s < nA; ++s) {
        const int32_t e = nl_ang[(size_t)list_slot(s, naf, nab, pc.capA) * pc.n + t];
        int j;
        float dx, dy, dz;
        pair_vector(e, pc, base, xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_rad2) continue;
        const float r = fsqrt(r2);
        overlap |= (r < 1e-3f);
        {   // radial basis
            const float tt = scaled_minus_one(r, pc.inv_rc_rad, pc.inv_rc_rad_lo);
            float fc;
            cutoff_value(tt, fc);
            float T[KB];
            cheb(fmaf(2.0f * tt, tt, -1.0f), T);
#pragma unroll
            for (int k = 0; k < KB; ++k) AR[k] = fmaf(fc, T[k], AR[k]);
        }
        if (r2 < pc.rc_ang2) {
            const float tt = scaled_minus_one(r, pc.inv_rc_ang, pc.inv_rc_ang_lo);
            float fc;
            cutoff_value(tt, fc);
            float T[KB];
            cheb(fmaf(2.0f * tt, tt, -1.0f), T);
            float g[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float s2 = csA[n];
#pragma unroll
                for (int k = 0; k < KB; ++k) s2 = fmaf(P[P_CA + n * KB + k], T[k], s2);
                g[n] = 0.5f * fc * s2;
            }
            const float rinv = frcp(r);
            float Y[NLM];
            sph(dx * rinv, dy * rinv, dz * rinv, Y);
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int lm = 0; lm < NLM; ++lm) S[n][lm] = fmaf(g[n], Y[lm], S[n][lm]);
        }
        if (r2 < pc.zbl_r2sq) {
            double U, dU;
            zbl_pair((double)r, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
            ezbl += 0.5 * U;
        }
    }
    // radial-only list
    const int nRl = nrf + nrb;
    for (int s = 0; s < nRl; ++s) {
        const int32_t e = nl_rad[(size_t)list_slot(s, nrf, nrb, pc.capR) * pc.n + t];
        int j;
        float dx, dy, dz;
        pair_vector(e, pc, base, xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_rad2) continue;
        const float r = fsqrt(r2);
        const float tt = scaled_minus_one(r, pc.inv_rc_rad, pc.inv_rc_rad_lo);
        float fc;
        cutoff_value(tt, fc);
        float T[KB];
        cheb(fmaf(2.0f * tt, tt, -1.0f), T);
#pragma unroll
        for (int k = 0; k < KB; ++k) AR[k] = fmaf(fc, T[k], AR[k]);
    }
    if (overlap) latch_error(status, -4);

    // descriptor
    float q[DIM];
    {
        float F[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) F[k] = 0.5f * (AR[k] + AR[0]);
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
    // network: forward and backward
    float U = -P[P_B1];
    float dzv[NH];
#pragma unroll
    for (int mu = 0; mu < NH; ++mu) {
        float z = -P[P_B0 + mu];
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) z = fmaf(P[P_W0 + mu * DIM + nu], P[P_QS + nu] * q[nu], z);
        const float th = ftanh(z);
        U = fmaf(P[P_W1 + mu], th, U);
        dzv[mu] = P[P_W1 + mu] * fmaf(-th, th, 1.0f);
    }
    float Fp[DIM];
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) {
        float s = 0.0f;
#pragma unroll
        for (int mu = 0; mu < NH; ++mu) s = fmaf(dzv[mu], P[P_W0 + mu * DIM + nu], s);
        Fp[nu] = s * P[P_QS + nu];
    }
    // adjoints
    float *ar = adj_r + (size_t)t * ADJ_R;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int n = 0; n < NR; ++n) s = fmaf(Fp[n], P[P_CR + n * KB + k], s);
        ar[k] = s;
    }
#pragma unroll
    for (int k = KB; k < ADJ_R; ++k) ar[k] = 0.0f;
    float4 *aa = reinterpret_cast<float4 *>(adj_a + (size_t)t * ADJ_A);
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int v = 0; v < NLM / 4; ++v) {
            float o[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int lm = 4 * v + w;
                const int l = lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
                o[w] = 2.0f * Fp[NR + NA * (l - 1) + n] * S[n][lm];
            }
            aa[n * (NLM / 4) + v] = make_float4(o[0], o[1], o[2], o[3]);
        }
    e_atom[t] = (double)U + ezbl;
}

// ------------------------------------------------------------------ forces + virial

__global__ __launch_bounds__(256) void k_force(
    PairConsts pc, const double *__restrict__ xs, const double *__restrict__ ys,
    const double *__restrict__ zs, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    const float *__restrict__ P, const float *__restrict__ adj_r, const float *__restrict__ adj_a,
    const int32_t *__restrict__ perm, float *__restrict__ fx, float *__restrict__ fy,
    float *__restrict__ fz, float *__restrict__ w_atom, const int32_t *__restrict__ status,
    int ntiles)
{
    const int tile = xcd_block(ntiles);
    if (tile >= ntiles) return;
    const int t = tile * 256 + threadIdx.x;
    if (t >= pc.n) return;
    if (status[ST_ERR] != 0) return;

    const double xi = xs[t], yi = ys[t], zi = zs[t];
    const CellGeom *cg = cells + cell_of[t];
    const int base = cg->atom_start;
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;

    float ai[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) ai[k] = adj_r[(size_t)t * ADJ_R + k];
    float Bi[NA * NLM];
    {
        const float4 *src = reinterpret_cast<const float4 *>(adj_a + (size_t)t * ADJ_A);
#pragma unroll
        for (int v = 0; v < ADJ_A / 4; ++v) {
            const float4 b = src[v];
            Bi[4 * v] = b.x; Bi[4 * v + 1] = b.y; Bi[4 * v + 2] = b.z; Bi[4 * v + 3] = b.w;
        }
    }
    float csA[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < KB; ++k) s += P[P_CA + n * KB + k];
        csA[n] = s;
    }

    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    float W[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = 0.0f;

    // radial part of the pair gradient, plus ZBL; returns dG/dr
    auto radial_dr = [&](int j, float r) -> float {
        const float tt = scaled_minus_one(r, pc.inv_rc_rad, pc.inv_rc_rad_lo);
        float fc, dfc;
        cutoff(tt, pc.inv_rc_rad, fc, dfc);
        const float dxdr = 4.0f * tt * pc.inv_rc_rad;
        float T[KB], dT[KB];
        cheb_d(fmaf(2.0f * tt, tt, -1.0f), T, dT);
        const float *aj = adj_r + (size_t)j * ADJ_R;
        const float4 a0 = reinterpret_cast<const float4 *>(aj)[0];
        const float4 a1 = reinterpret_cast<const float4 *>(aj)[1];
        const float a8 = aj[8];
        const float ah[KB] = {ai[0] + a0.x, ai[1] + a0.y, ai[2] + a0.z, ai[3] + a0.w, ai[4] + a1.x,
                              ai[5] + a1.y, ai[6] + a1.z, ai[7] + a1.w, ai[8] + a8};
        float s0 = 0.0f, s1 = 0.0f, sa = 0.0f;
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            s0 = fmaf(ah[k], T[k], s0);
            s1 = fmaf(ah[k], dT[k], s1);
            sa += ah[k];
        }
        return 0.5f * (dxdr * fc * s1 + dfc * (s0 + sa));
    };

    const int nA = naf + nab;
    for (int s = 0; s < nA; ++s) {
        const int32_t e = nl_ang[(size_t)list_slot(s, naf, nab, pc.capA) * pc.n + t];
        int j;
        float dx, dy, dz;
        pair_vector(e, pc, base, xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_rad2) continue;
        const float r = fsqrt(r2);
        const float rinv = frcp(r);
        float dGdr = radial_dr(j, r);
        if (r2 < pc.zbl_r2sq) {
            double U, dU;
            zbl_pair((double)r, (double)pc.zbl_z, (double)pc.zbl_r1, (double)pc.zbl_r2, U, dU);
            dGdr += (float)dU;
        }
        const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
        float fxp = dGdr * ux, fyp = dGdr * uy, fzp = dGdr * uz;
        if (r2 < pc.rc_ang2) {
            const float tt = scaled_minus_one(r, pc.inv_rc_ang, pc.inv_rc_ang_lo);
            float fc, dfc;
            cutoff(tt, pc.inv_rc_ang, fc, dfc);
            const float dxdr = 4.0f * tt * pc.inv_rc_ang;
            float T[KB], dT[KB];
            cheb_d(fmaf(2.0f * tt, tt, -1.0f), T, dT);
            float g[NA], gp[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float sn = csA[n], sp = 0.0f;
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    sn = fmaf(P[P_CA + n * KB + k], T[k], sn);
                    sp = fmaf(P[P_CA + n * KB + k], dT[k], sp);
                }
                g[n] = 0.5f * fc * sn;
                gp[n] = 0.5f * fmaf(dxdr * fc, sp, dfc * sn);
            }
            float Y[NLM];
            sph(ux, uy, uz, Y);
            const float4 *bj4 = reinterpret_cast<const float4 *>(adj_a + (size_t)j * ADJ_A);
            float Dc[NLM];
            float s1 = 0.0f;
#pragma unroll
            for (int lm = 0; lm < NLM; ++lm) Dc[lm] = 0.0f;
            float Dp[NLM];
#pragma unroll
            for (int lm = 0; lm < NLM; ++lm) Dp[lm] = 0.0f;
#pragma unroll
            for (int n = 0; n < NA; ++n) {
#pragma unroll
                for (int v = 0; v < NLM / 4; ++v) {
                    const float4 b = bj4[n * (NLM / 4) + v];
                    const float bj[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const int lm = 4 * v + w;
                        const bool odd = (lm < 3) || (lm >= 8 && lm < 15);
                        const float bh = odd ? Bi[n * NLM + lm] - bj[w] : Bi[n * NLM + lm] + bj[w];
                        Dc[lm] = fmaf(bh, g[n], Dc[lm]);
                        Dp[lm] = fmaf(bh, gp[n], Dp[lm]);
                    }
                }
            }
#pragma unroll
            for (int lm = 0; lm < NLM; ++lm) s1 = fmaf(Dp[lm], Y[lm], s1);
            float vx, vy, vz;
            sph_grad_contract(ux, uy, uz, Dc, vx, vy, vz);
            const float uv = ux * vx + uy * vy + uz * vz;
            fxp += s1 * ux + (vx - uv * ux) * rinv;
            fyp += s1 * uy + (vy - uv * uy) * rinv;
            fzp += s1 * uz + (vz - uv * uz) * rinv;
        }
        Fx += fxp; Fy += fyp; Fz += fzp;
        W[0] = fmaf(fxp, dx, W[0]); W[1] = fmaf(fxp, dy, W[1]); W[2] = fmaf(fxp, dz, W[2]);
        W[3] = fmaf(fyp, dx, W[3]); W[4] = fmaf(fyp, dy, W[4]); W[5] = fmaf(fyp, dz, W[5]);
        W[6] = fmaf(fzp, dx, W[6]); W[7] = fmaf(fzp, dy, W[7]); W[8] = fmaf(fzp, dz, W[8]);
    }
    const int nRl = nrf + nrb;
    for (int s = 0; s < nRl; ++s) {
        const int32_t e = nl_rad[(size_t)list_slot(s, nrf, nrb, pc.capR) * pc.n + t];
        int j;
        float dx, dy, dz;
        pair_vector(e, pc, base, xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= pc.rc_rad2) continue;
        const float r = fsqrt(r2);
        const float c = radial_dr(j, r) * frcp(r);
        const float fxp = c * dx, fyp = c * dy, fzp = c * dz;
        Fx += fxp; Fy += fyp; Fz += fzp;
        W[0] = fmaf(fxp, dx, W[0]); W[1] = fmaf(fxp, dy, W[1]); W[2] = fmaf(fxp, dz, W[2]);
        W[3] = fmaf(fyp, dx, W[3]); W[4] = fmaf(fyp, dy, W[4]); W[5] = fmaf(fyp, dz, W[5]);
        W[6] = fmaf(fzp, dx, W[6]); W[7] = fmaf(fzp, dy, W[7]); W[8] = fmaf(fzp, dz, W[8]);
    }
    const int i = perm[t];
    fx[i] = Fx;
    fy[i] = Fy;
    fz[i] = Fz;
    float *w = w_atom + (size_t)t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = -0.5f * W[k];
}

// ------------------------------------------------------------------ reductions

// One block per chunk of atoms of a single cell: FP64 sums of the site
// energies and the per-atom virials, written to part[chunk][10].
__global__ __launch_bounds__(256) void k_reduce_chunks(const int32_t *__restrict__ chunk_begin,
                                                       const int32_t *__restrict__ chunk_end,
                                                       const double *__restrict__ e_atom,
                                                       const float *__restrict__ w_atom,
                                                       double *__restrict__ part,
                                                       const int32_t *__restrict__ status)
{
    __shared__ double sh[10][256];
    const int k = blockIdx.x;
    double acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    if (status[ST_ERR] == 0) {
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

// One thread per cell: ordered sum of its chunk partials.
__global__ void k_reduce_cells(int n_cells, const int32_t *__restrict__ cell_chunk,
                               const double *__restrict__ part, double *__restrict__ energy,
                               double *__restrict__ virial, const int32_t *__restrict__ status)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    if (status[ST_ERR] != 0) return;
    double acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    for (int k = cell_chunk[c]; k < cell_chunk[c + 1]; ++k)
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] += part[(size_t)k * 10 + q];
    energy[c] = acc[0];
    if (virial)
#pragma unroll
        for (int q = 0; q < 9; ++q) virial[(size_t)c * 9 + q] = acc[1 + q];
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
    PairConsts pc, const double *__restrict__ xs, const double *__restrict__ ys,
    const double *__restrict__ zs, const int32_t *__restrict__ cell_of,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ nl_ang,
    const int32_t *__restrict__ nl_rad, const uint32_t *__restrict__ ncnt,
    unsigned long long *__restrict__ counts)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nr = 0, na = 0;
    if (t < pc.n) {
        const double xi = xs[t], yi = ys[t], zi = zs[t];
        const CellGeom *cg = cells + cell_of[t];
        const uint32_t cnt = ncnt[t];
        const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff, nrf = (cnt >> 16) & 0xff, nrb = cnt >> 24;
        for (int s = 0; s < naf + nab; ++s) {
            int j;
            float dx, dy, dz;
            pair_vector(nl_ang[(size_t)list_slot(s, naf, nab, pc.capA) * pc.n + t], pc, cg->atom_start,
                        xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
            const float r2 = dx * dx + dy * dy + dz * dz;
            nr += r2 < pc.rc_rad2;
            na += r2 < pc.rc_ang2;
        }
        for (int s = 0; s < nrf + nrb; ++s) {
            int j;
            float dx, dy, dz;
            pair_vector(nl_rad[(size_t)list_slot(s, nrf, nrb, pc.capR) * pc.n + t], pc, cg->atom_start,
                        xi, yi, zi, xs, ys, zs, cg, j, dx, dy, dz);
            nr += (dx * dx + dy * dy + dz * dz) < pc.rc_rad2;
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

}  // namespace nep
