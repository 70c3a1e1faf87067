// Device-side building blocks of the NEP-ZBL kernels (gfx950).
//
// Everything here is single precision except the ZBL pair term, which is
// rare (pairs closer than 2 A) and evaluated in double precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nep {

// ---------------------------------------------------------------- model sizes
// Compiled model: n_max^R = 8 (9 radial components), n_max^A = 4 (5 angular
// radial functions), Chebyshev k = 0..8, l = 1..4, 30 hidden neurons.
constexpr int NR = 9;        // radial descriptor components
constexpr int NA = 5;        // angular radial functions
constexpr int KB = 9;        // Chebyshev basis size (radial and angular)
constexpr int LMAX = 4;
constexpr int NLM = 24;      // (l, m) pairs for l = 1..4
constexpr int DIM = NR + NA * LMAX;   // 29
constexpr int NH = 30;       // hidden neurons

// Packed FP32 parameter block (offsets in floats).
constexpr int P_CR = 0;                  // [NR][KB]
constexpr int P_CA = P_CR + NR * KB;     // [NA][KB]
constexpr int P_QS = P_CA + NA * KB;     // [DIM]
constexpr int P_W0 = P_QS + DIM;         // [NH][DIM]
constexpr int P_B0 = P_W0 + NH * DIM;    // [NH]
constexpr int P_W1 = P_B0 + NH;          // [NH]
constexpr int P_B1 = P_W1 + NH;          // [1]
constexpr int P_SIZE = P_B1 + 1;
// FP64 copy of the angular coefficients and their row sums
constexpr int C64N = NA * KB + NA;
// threads per block of the population descriptor kernel
constexpr int POP_DESC_BS = 64;

// Per-atom record in sorted order, one 64-byte half cache line: the wrapped
// FP64 position (written by the position refresh) and the radial adjoint
// a_k = dU_i/dF_k (written by the descriptor kernel).  A neighbour gather in
// the force kernel touches exactly one record.
struct __attribute__((aligned(64))) AtomRec {
    double x, y, z;
    float a[KB];
    float pad;
};
static_assert(sizeof(AtomRec) == 64, "AtomRec must be 64 bytes");

// The force kernel's record in bin-offset mode (PairConsts::delta): the
// position as 32-bit fixed-point offsets from the corner of the atom's bin
// at the last build (units PairConsts::qs), and the radial adjoints; 48
// bytes, three 16-byte pieces per gather instead of four.  Pair vectors
// formed from two records, d = sum_a o_a bv_a + qs (o_j - o_i) (o the
// neighbour-bin offset), are exact negatives of each other.
struct __attribute__((aligned(16))) AtomRec48 {
    int32_t o[3];
    float a[KB];
};
static_assert(sizeof(AtomRec48) == 48, "AtomRec48 must be 48 bytes");

// Runtime constants shared by the pair kernels.
struct PairConsts {
    float rc_rad, rc_ang;             // cutoffs
    float rc_rad2, rc_ang2;           // squared
    // angular pair gradients: the descriptor kernel stores a slot when
    // r^2 < rc_ang2_write (zero beyond rc_ang2), the force kernel reads the
    // other end's slot when r^2 < rc_ang2_read; write > read by a margin of
    // many ulps, so every slot read was written in the same evaluation
    float rc_ang2_write, rc_ang2_read;
    float inv_rc_rad, inv_rc_ang;     // 1/rc rounded to FP32 ...
    float inv_rc_rad_lo, inv_rc_ang_lo;   // ... and the rounding remainder 1/rc - inv_rc
    float zbl_r1, zbl_r2, zbl_r2sq;
    float zbl_z;                      // nuclear charge
    int capA, capR;                   // list capacities
    int jbits, ibits, ioff;           // neighbour entry encoding
    uint32_t code0;                   // image code of an entry in the cell itself (no shift)
    // an entry names no image iff (code & img_mask) == img_val (either mode)
    uint32_t img_mask, img_val;
    // Bin-offset mode (one periodic cell, every axis binned, at most 2^23
    // atoms): an entry is j | q << jbits | cr << (jbits + 5), q = (o0 + 1) +
    // 3 (o1 + 1) + 9 (o2 + 1) the offset o of j's bin from i's in the 27-bin
    // stencil and cr the axes across whose periodic face that bin lies (the
    // image is n_a = o_a on those axes, 0 on the others); the default
    // model's force records are then AtomRec48 with offsets in units qs.
    int delta;
    double qs, qsinv;
    int n;                            // atoms (list stride)
    // [word][atom]: bit s of word s/32 is set when the s-th entry of the
    // radial list was inside rc_rad at the last descriptor evaluation (the
    // force kernel walks only those entries)
    uint32_t *rmask;
    // [word][atom]: bit s set when the s-th angular-list entry was within
    // the pair-gradient write radius (rc_ang2_write, with a margin) at the
    // last evaluation's first walk; the later angular walks take only those
    uint32_t *amask;
    // [word][atom]: bit s set when the s-th radial-list entry was within
    // rc_cand (rc_rad plus a margin) at the last full radial walk; between
    // full walks, while no atom can have moved by half the margin, the
    // descriptor's radial walk takes only those entries
    uint32_t *cmask;
    float rc_cand;
};

// Reference lattice of the Wigner-Seitz analysis (perfect bcc, cubic
// constant a, n[0] x n[1] x n[2] conventional cells).
struct BccRef {
    double a, inv_a;
    int n[3];
};

struct CellGeom {
    double h[9];       // rows: lattice vectors
    double hinv[9];    // x = s h  =>  s = x hinv
    int nb[3];         // bins per axis (1 for image-loop axes)
    int R[3];          // image range for image-loop axes, 0 for binned axes
    int periodic[3];
    double bv[9];      // rows: bin edge vectors h_a / nb_a
    int bin_offset;    // first global bin of this cell
    int atom_start;    // first atom (caller and sorted order coincide per cell)
    int n_atoms;
    int pad_;
};

// ---------------------------------------------------------------- status word
// status[0]: latched error code (0 = none); status[1], status[2]: required
// angular / radial list lengths seen by the last build; status[3]: nonzero
// while the lists are unusable (the last build ended with an error, so the
// lists may be truncated and the reverse index unwritten).
constexpr int ST_ERR = 0;
constexpr int ST_NEED_A = 1;
constexpr int ST_NEED_R = 2;
constexpr int ST_LBAD = 3;

// velocity-Verlet state (doubles): step length (fs), max |v|^2, max
// displacement^2 since the last build (both as ordered bit patterns of
// non-negative doubles), simulated time, rebuild count.  With the border
// thermostat: max |v|^2 of the border atoms, the factor the next kick applies
// to border velocities first, 2K of the border atoms (eV) after the last
// scaling, the chain positions and velocities (MD_NHC_MAX each) and the
// chain's energy.  MD_STEP_WORDS words are reset at every call; the chain
// state after them persists.
constexpr int MD_DT = 0, MD_VMAX2 = 1, MD_DISP2 = 2, MD_TIME = 3, MD_NREB = 4, MD_VMAX2B = 5, MD_SCALE = 6,
              MD_TWOK = 7;
constexpr int MD_STEP_WORDS = 8;
constexpr int MD_NHC_MAX = 8;
constexpr int MD_XI = 8, MD_VXI = MD_XI + MD_NHC_MAX, MD_ENHC = MD_VXI + MD_NHC_MAX, MD_NBORDER = MD_ENHC + 1;
// bound on any atom's displacement since the last full radial walk (sum of
// the steps' largest displacements), and the current step's largest
// displacement squared
constexpr int MD_CACC = MD_NBORDER + 1, MD_STEP2 = MD_CACC + 1;
// candidate radius of the descriptor's radial walk: rc_rad + CAND_MARGIN;
// between full walks no atom may have moved more than CAND_TRIGGER (below
// half the margin, which keeps every pair that can be inside rc_rad among the
// candidates)
constexpr double CAND_MARGIN = 0.2, CAND_TRIGGER = 0.09;
static_assert(MD_STEP2 < 32, "MD state words");
constexpr int MD_WORDS = 32;

__device__ inline void latch_error(int *status, int code)
{
    atomicCAS(status + ST_ERR, 0, code);
}

// Sum over the 64 lanes of a wavefront, the same total in every lane (xor
// butterfly: a fixed order of additions, so the result is deterministic).
__device__ __forceinline__ float wave_sum64(float v)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Entry check of the kernels that walk the neighbour lists: true if they
// must do nothing, either because an error is latched or because the lists
// are unusable (then NEP_E_STATE is latched, so the call reports an error
// instead of numbers computed on truncated lists).
__device__ inline bool lists_blocked(int *status)
{
    if (status[ST_ERR] != 0) return true;
    if (status[ST_LBAD] != 0) {
        latch_error(status, -7);
        return true;
    }
    return false;
}

// ---------------------------------------------------------------- fast math
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// sin(y) and cos(y) for |y| <= pi/2 from their Taylor series (truncation
// error below 1e-9 there), evaluated in Horner form.
__host__ __device__ inline void sincos_halfpi(float y, float &s, float &c)
{
    const float y2 = y * y;
    float ps = 1.0f / 6227020800.0f;               // 1/13!
    ps = fmaf(ps, y2, -1.0f / 39916800.0f);        // -1/11!
    ps = fmaf(ps, y2, 1.0f / 362880.0f);           // 1/9!
    ps = fmaf(ps, y2, -1.0f / 5040.0f);            // -1/7!
    ps = fmaf(ps, y2, 1.0f / 120.0f);
    ps = fmaf(ps, y2, -1.0f / 6.0f);
    ps = fmaf(ps, y2, 1.0f);
    s = ps * y;
    float pc = 1.0f / 479001600.0f;                // 1/12!
    pc = fmaf(pc, y2, -1.0f / 3628800.0f);         // -1/10!
    pc = fmaf(pc, y2, 1.0f / 40320.0f);            // 1/8!
    pc = fmaf(pc, y2, -1.0f / 720.0f);             // -1/6!
    pc = fmaf(pc, y2, 1.0f / 24.0f);
    pc = fmaf(pc, y2, -0.5f);
    c = fmaf(pc, y2, 1.0f);
}

// tt = r/rc - 1 without the systematic bias that the FP32 rounding of 1/rc
// would add (the Chebyshev argument x = 2 tt^2 - 1 amplifies any bias of x by
// up to k^2 in T_k): 1/rc is carried as inv + inv_lo.
__host__ __device__ inline float scaled_minus_one(float r, float inv, float inv_lo)
{
    return fmaf(r, inv, -1.0f) + r * inv_lo;
}

// Double-precision pieces of the descriptor's pair geometry.
// sin(y) for |y| <= pi/2, Taylor series to y^17 (truncation error < 5e-14).
__host__ __device__ inline double sin_halfpi_d(double y)
{
    const double y2 = y * y;
    double p = 1.0 / 355687428096000.0;            // 1/17!
    p = fma(p, y2, -1.0 / 1307674368000.0);        // -1/15!
    p = fma(p, y2, 1.0 / 6227020800.0);            // 1/13!
    p = fma(p, y2, -1.0 / 39916800.0);             // -1/11!
    p = fma(p, y2, 1.0 / 362880.0);                // 1/9!
    p = fma(p, y2, -1.0 / 5040.0);                 // -1/7!
    p = fma(p, y2, 1.0 / 120.0);
    p = fma(p, y2, -1.0 / 6.0);
    p = fma(p, y2, 1.0);
    return p * y;
}

// fc(r) and T_0..T_8(x), x = 2 (r/rc - 1)^2 - 1, in double precision.
__host__ __device__ inline void basis_d(double r, double inv_rc, double &fc, double T[KB])
{
    const double PI = 3.14159265358979323846;
    const double tt = r * inv_rc - 1.0;
    fc = 0.5 - 0.5 * sin_halfpi_d(PI * (tt + 0.5));
    const double x = 2.0 * tt * tt - 1.0;
    T[0] = 1.0;
    T[1] = x;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = 2; k < KB; ++k) T[k] = fma(x2, T[k - 1], -T[k - 2]);
}

// Smooth cutoff fc(r) = (1 + cos(pi r/rc))/2 and its derivative, for r < rc,
// from tt = r/rc - 1.  With y = pi (tt + 1/2): cos(pi r/rc) = -sin(y),
// sin(pi r/rc) = cos(y); pi is carried as two floats for the same reason.
__host__ __device__ inline void cutoff(float tt, float inv_rc, float &fc, float &dfc)
{
    const float PI_HI = 3.14159274101257324f, PI_LO = -8.74227765734758577e-8f;
    const float u = tt + 0.5f;
    const float y = fmaf(PI_HI, u, PI_LO * u);
    float s, c;
    sincos_halfpi(y, s, c);
    fc = 0.5f - 0.5f * s;
    dfc = -0.5f * PI_HI * inv_rc * c;
}

__host__ __device__ inline void cutoff_value(float tt, float &fc)
{
    float d;
    cutoff(tt, 1.0f, fc, d);
}

// Chebyshev polynomials T_0..T_8 at x (three-term recurrence).
__host__ __device__ inline void cheb(float x, float T[KB])
{
    T[0] = 1.0f;
    T[1] = x;
    const float x2 = 2.0f * x;
#pragma unroll
    for (int k = 2; k < KB; ++k) T[k] = fmaf(x2, T[k - 1], -T[k - 2]);
}

// T_k and dT_k/dx (dT_{k} = 2 T_{k-1} + 2x dT_{k-1} - dT_{k-2}).
__host__ __device__ inline void cheb_d(float x, float T[KB], float dT[KB])
{
    T[0] = 1.0f;
    T[1] = x;
    dT[0] = 0.0f;
    dT[1] = 1.0f;
    const float x2 = 2.0f * x;
#pragma unroll
    for (int k = 2; k < KB; ++k) {
        T[k] = fmaf(x2, T[k - 1], -T[k - 2]);
        dT[k] = fmaf(x2, dT[k - 1], fmaf(2.0f, T[k - 1], -dT[k - 2]));
    }
}

// T_k and dT_k/dx evaluated in double precision from x, rounded to single
// (near x = -1 the recurrences amplify a rounding of x by up to k^2 in T_k
// and k^4 in dT_k, so x must not be rounded before them).
__host__ __device__ inline void cheb_d_from_d(double x, float T[KB], float dT[KB])
{
    double t2 = 1.0, t1 = x, d2 = 0.0, d1 = 1.0;
    T[0] = 1.0f;
    T[1] = (float)x;
    dT[0] = 0.0f;
    dT[1] = 1.0f;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = 2; k < KB; ++k) {
        const double t = fma(x2, t1, -t2);
        const double d = fma(x2, d1, fma(2.0, t1, -d2));
        T[k] = (float)t;
        dT[k] = (float)d;
        t2 = t1; t1 = t; d2 = d1; d1 = d;
    }
}

// ---------------------------------------------------------------- harmonics
// Real spherical harmonics scaled by sqrt(4 pi / (2l+1)), so that
// sum_m Y_lm(u) Y_lm(v) = P_l(u.v) (addition theorem).  Index lm = l^2 - 1 + (m + l).
// Written as polynomials valid on the unit sphere.
#define NEP_S3 1.7320508075688772f
#define NEP_S5 2.2360679774997896f
#define NEP_S6 2.4494897427831781f
#define NEP_S10 3.1622776601683795f
#define NEP_S15 3.8729833462074170f
#define NEP_S35 5.9160797830996160f
#define NEP_S70 8.3666002653407555f

__host__ __device__ inline void sph(float x, float y, float z, float Y[NLM])
{
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    Y[0] = y; Y[1] = z; Y[2] = x;
    Y[3] = NEP_S3 * x * y;
    Y[4] = NEP_S3 * y * z;
    Y[5] = 0.5f * (3.0f * z2 - 1.0f);
    Y[6] = NEP_S3 * x * z;
    Y[7] = 0.5f * NEP_S3 * (x2 - y2);
    Y[8] = 0.25f * NEP_S10 * y * (3.0f * x2 - y2);
    Y[9] = NEP_S15 * x * y * z;
    Y[10] = 0.25f * NEP_S6 * y * (5.0f * z2 - 1.0f);
    Y[11] = 0.5f * z * (5.0f * z2 - 3.0f);
    Y[12] = 0.25f * NEP_S6 * x * (5.0f * z2 - 1.0f);
    Y[13] = 0.5f * NEP_S15 * z * (x2 - y2);
    Y[14] = 0.25f * NEP_S10 * x * (x2 - 3.0f * y2);
    Y[15] = 0.5f * NEP_S35 * x * y * (x2 - y2);
    Y[16] = 0.25f * NEP_S70 * y * z * (3.0f * x2 - y2);
    Y[17] = 0.5f * NEP_S5 * x * y * (7.0f * z2 - 1.0f);
    Y[18] = 0.25f * NEP_S10 * y * z * (7.0f * z2 - 3.0f);
    Y[19] = 0.125f * (35.0f * z2 * z2 - 30.0f * z2 + 3.0f);
    Y[20] = 0.25f * NEP_S10 * x * z * (7.0f * z2 - 3.0f);
    Y[21] = 0.25f * NEP_S5 * (x2 - y2) * (7.0f * z2 - 1.0f);
    Y[22] = 0.25f * NEP_S70 * x * z * (x2 - 3.0f * y2);
    Y[23] = 0.125f * NEP_S35 * (x2 * x2 - 6.0f * x2 * y2 + y2 * y2);
}

// v = sum_lm Dc[lm] * grad_u p_lm(u), the gradient of the polynomials above
// taken with x, y, z independent (the caller projects out the radial part).
// The same harmonics in double precision, one degree l at a time: the 2l+1
// values that sph stores at offsets l*l-1 .. l*l+2l-1, in the same order.
template <int L>
__host__ __device__ inline void sph_degree_d(double x, double y, double z, double *Y)
{
    constexpr double S3 = 1.7320508075688772, S5 = 2.2360679774997896, S6 = 2.4494897427831781;
    constexpr double S10 = 3.1622776601683795, S15 = 3.8729833462074170, S35 = 5.9160797830996160;
    constexpr double S70 = 8.3666002653407555;
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    if constexpr (L == 1) {
        Y[0] = y; Y[1] = z; Y[2] = x;
    } else if constexpr (L == 2) {
        Y[0] = S3 * x * y;
        Y[1] = S3 * y * z;
        Y[2] = 0.5 * (3.0 * z2 - 1.0);
        Y[3] = S3 * x * z;
        Y[4] = 0.5 * S3 * (x2 - y2);
    } else if constexpr (L == 3) {
        Y[0] = 0.25 * S10 * y * (3.0 * x2 - y2);
        Y[1] = S15 * x * y * z;
        Y[2] = 0.25 * S6 * y * (5.0 * z2 - 1.0);
        Y[3] = 0.5 * z * (5.0 * z2 - 3.0);
        Y[4] = 0.25 * S6 * x * (5.0 * z2 - 1.0);
        Y[5] = 0.5 * S15 * z * (x2 - y2);
        Y[6] = 0.25 * S10 * x * (x2 - 3.0 * y2);
    } else {
        static_assert(L == 4, "degrees 1..4");
        Y[0] = 0.5 * S35 * x * y * (x2 - y2);
        Y[1] = 0.25 * S70 * y * z * (3.0 * x2 - y2);
        Y[2] = 0.5 * S5 * x * y * (7.0 * z2 - 1.0);
        Y[3] = 0.25 * S10 * y * z * (7.0 * z2 - 3.0);
        Y[4] = 0.125 * (35.0 * z2 * z2 - 30.0 * z2 + 3.0);
        Y[5] = 0.25 * S10 * x * z * (7.0 * z2 - 3.0);
        Y[6] = 0.25 * S5 * (x2 - y2) * (7.0 * z2 - 1.0);
        Y[7] = 0.25 * S70 * x * z * (x2 - 3.0 * y2);
        Y[8] = 0.125 * S35 * (x2 * x2 - 6.0 * x2 * y2 + y2 * y2);
    }
}

__host__ __device__ inline void sph_grad_contract(float x, float y, float z, const float Dc[NLM],
                                         float &vx, float &vy, float &vz)
{
    // the gradients of the 24 polynomials share a few monomials; each term is
    // (constant x Dc[lm]) times one of them
    const float a3 = 0.25f * NEP_S10, b3 = NEP_S15, c3 = 0.25f * NEP_S6, e3 = 0.5f * NEP_S15;
    const float a4 = 0.5f * NEP_S35, b4 = 0.25f * NEP_S70, c4 = 0.5f * NEP_S5, d4 = 0.25f * NEP_S10;
    const float e4 = 0.25f * NEP_S5, f4 = 0.125f * NEP_S35;
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, xz = x * z, yz = y * z, xyz = xy * z;
    const float dxy = x2 - y2;
    const float t5 = fmaf(5.0f, z2, -1.0f), t7 = fmaf(7.0f, z2, -1.0f), t73 = fmaf(7.0f, z2, -3.0f);
    const float yt7 = y * t7, xt7 = x * t7, zt73 = z * t73, zdxy = z * dxy;
    const float p1 = y * fmaf(3.0f, x2, -y2);   // y (3x^2 - y^2)
    const float p2 = x * fmaf(-3.0f, y2, x2);   // x (x^2 - 3y^2)
    float gx = Dc[2], gy = Dc[0], gz = Dc[1];
    // l = 2
    gx = fmaf(NEP_S3 * Dc[3], y, gx); gx = fmaf(NEP_S3 * Dc[6], z, gx); gx = fmaf(NEP_S3 * Dc[7], x, gx);
    gy = fmaf(NEP_S3 * Dc[3], x, gy); gy = fmaf(NEP_S3 * Dc[4], z, gy); gy = fmaf(-NEP_S3 * Dc[7], y, gy);
    gz = fmaf(NEP_S3 * Dc[4], y, gz); gz = fmaf(NEP_S3 * Dc[6], x, gz); gz = fmaf(3.0f * Dc[5], z, gz);
    // l = 3
    gx = fmaf(6.0f * a3 * Dc[8], xy, gx);  gy = fmaf(3.0f * a3 * Dc[8], dxy, gy);
    gx = fmaf(b3 * Dc[9], yz, gx);         gy = fmaf(b3 * Dc[9], xz, gy);          gz = fmaf(b3 * Dc[9], xy, gz);
    gy = fmaf(c3 * Dc[10], t5, gy);        gz = fmaf(10.0f * c3 * Dc[10], yz, gz);
    gz = fmaf(1.5f * Dc[11], t5, gz);
    gx = fmaf(c3 * Dc[12], t5, gx);        gz = fmaf(10.0f * c3 * Dc[12], xz, gz);
    gx = fmaf(2.0f * e3 * Dc[13], xz, gx); gy = fmaf(-2.0f * e3 * Dc[13], yz, gy); gz = fmaf(e3 * Dc[13], dxy, gz);
    gx = fmaf(3.0f * a3 * Dc[14], dxy, gx); gy = fmaf(-6.0f * a3 * Dc[14], xy, gy);
    // l = 4
    gx = fmaf(a4 * Dc[15], p1, gx);        gy = fmaf(a4 * Dc[15], p2, gy);
    gx = fmaf(6.0f * b4 * Dc[16], xyz, gx); gy = fmaf(3.0f * b4 * Dc[16], zdxy, gy); gz = fmaf(b4 * Dc[16], p1, gz);
    gx = fmaf(c4 * Dc[17], yt7, gx);       gy = fmaf(c4 * Dc[17], xt7, gy);        gz = fmaf(14.0f * c4 * Dc[17], xyz, gz);
    gy = fmaf(d4 * Dc[18], zt73, gy);      gz = fmaf(3.0f * d4 * Dc[18], yt7, gz);
    gz = fmaf(2.5f * Dc[19], zt73, gz);
    gx = fmaf(d4 * Dc[20], zt73, gx);      gz = fmaf(3.0f * d4 * Dc[20], xt7, gz);
    gx = fmaf(2.0f * e4 * Dc[21], xt7, gx); gy = fmaf(-2.0f * e4 * Dc[21], yt7, gy); gz = fmaf(14.0f * e4 * Dc[21], zdxy, gz);
    gx = fmaf(3.0f * b4 * Dc[22], zdxy, gx); gy = fmaf(-6.0f * b4 * Dc[22], xyz, gy); gz = fmaf(b4 * Dc[22], p2, gz);
    gx = fmaf(4.0f * f4 * Dc[23], p2, gx);  gy = fmaf(-4.0f * f4 * Dc[23], p1, gy);
    vx = gx; vy = gy; vz = gz;
}

// The same harmonics without their normalisation: Y_lm = sph_norm(lm) y_lm
// with y_lm polynomials of small integer coefficients.  A caller that folds
// the constants into its coefficients (D'_lm = sph_norm(lm) D_lm) evaluates
// sum_lm D_lm Y_lm as sum_lm D'_lm y_lm and its gradient with fewer products.
__host__ __device__ constexpr float sph_norm(int lm)
{
    return lm < 3 ? 1.0f
         : lm == 3 || lm == 4 || lm == 6 ? NEP_S3
         : lm == 5 ? 0.5f
         : lm == 7 ? 0.5f * NEP_S3
         : lm == 8 || lm == 14 ? 0.25f * NEP_S10
         : lm == 9 ? NEP_S15
         : lm == 10 || lm == 12 ? 0.25f * NEP_S6
         : lm == 11 ? 0.5f
         : lm == 13 ? 0.5f * NEP_S15
         : lm == 15 ? 0.5f * NEP_S35
         : lm == 16 || lm == 22 ? 0.25f * NEP_S70
         : lm == 17 ? 0.5f * NEP_S5
         : lm == 18 || lm == 20 ? 0.25f * NEP_S10
         : lm == 19 ? 0.125f
         : lm == 21 ? 0.25f * NEP_S5
         : 0.125f * NEP_S35;
}

// The unnormalised harmonics of one degree in double precision (the 2l+1
// values y_lm, lm = l*l-1 .. l*l+2l-1, in the order of sph).
template <int L>
__host__ __device__ inline void sph_unnorm_degree_d(double x, double y, double z, double *Y)
{
    if constexpr (L == 1) {
        Y[0] = y; Y[1] = z; Y[2] = x;
    } else if constexpr (L == 2) {
        Y[0] = x * y; Y[1] = y * z; Y[2] = fma(3.0 * z, z, -1.0); Y[3] = x * z; Y[4] = fma(x, x, -y * y);
    } else {
        static_assert(L == 3, "degrees 1..3");
        const double x2 = x * x, y2 = y * y, z2 = z * z, t5 = fma(5.0, z2, -1.0);
        Y[0] = y * fma(3.0, x2, -y2);
        Y[1] = x * y * z;
        Y[2] = y * t5;
        Y[3] = z * (t5 - 2.0);
        Y[4] = x * t5;
        Y[5] = z * (x2 - y2);
        Y[6] = x * fma(-3.0, y2, x2);
    }
}

// Monomials shared by the unnormalised harmonics and their gradients.
struct SphMono {
    float x, y, z, xy, xz, yz, xyz, dxy, t5, t7, t73, p1, p2;
    __host__ __device__ SphMono(float x_, float y_, float z_) : x(x_), y(y_), z(z_)
    {
        const float x2 = x * x, y2 = y * y, z2 = z * z;
        xy = x * y; xz = x * z; yz = y * z; xyz = xy * z;
        dxy = x2 - y2;
        t5 = fmaf(5.0f, z2, -1.0f); t7 = fmaf(7.0f, z2, -1.0f); t73 = fmaf(7.0f, z2, -3.0f);
        p1 = y * fmaf(3.0f, x2, -y2);    // 3x^2 y - y^3
        p2 = x * fmaf(-3.0f, y2, x2);    // x^3 - 3x y^2
    }
};

__host__ __device__ inline void sph_unnorm(const SphMono &m, float y[NLM])
{
    y[0] = m.y; y[1] = m.z; y[2] = m.x;
    y[3] = m.xy; y[4] = m.yz; y[5] = fmaf(3.0f, m.z * m.z, -1.0f); y[6] = m.xz; y[7] = m.dxy;
    y[8] = m.p1; y[9] = m.xyz; y[10] = m.y * m.t5; y[11] = m.z * (m.t5 - 2.0f); y[12] = m.x * m.t5;
    y[13] = m.z * m.dxy; y[14] = m.p2;
    const float z2 = m.z * m.z;
    y[15] = m.xy * m.dxy; y[16] = m.z * m.p1; y[17] = m.xy * m.t7; y[18] = m.yz * m.t73;
    y[19] = fmaf(35.0f * z2, z2, fmaf(-30.0f, z2, 3.0f)); y[20] = m.xz * m.t73; y[21] = m.dxy * m.t7;
    y[22] = m.z * m.p2; y[23] = fmaf(-4.0f * m.xy, m.xy, m.dxy * m.dxy);
}

// v = sum_lm Dc[lm] grad y_lm (x, y, z independent; the caller projects out
// the radial part).
__host__ __device__ inline void sph_unnorm_grad_contract(const SphMono &m, const float Dc[NLM], float &vx,
                                                         float &vy, float &vz)
{
    const float yt7 = m.y * m.t7, xt7 = m.x * m.t7, zt73 = m.z * m.t73, zdxy = m.z * m.dxy;
    float gx = Dc[2], gy = Dc[0], gz = Dc[1];
    // l = 2
    gx = fmaf(Dc[3], m.y, gx); gy = fmaf(Dc[3], m.x, gy);
    gy = fmaf(Dc[4], m.z, gy); gz = fmaf(Dc[4], m.y, gz);
    gz = fmaf(Dc[5], 6.0f * m.z, gz);
    gx = fmaf(Dc[6], m.z, gx); gz = fmaf(Dc[6], m.x, gz);
    gx = fmaf(Dc[7], 2.0f * m.x, gx); gy = fmaf(Dc[7], -2.0f * m.y, gy);
    // l = 3
    const float xy6 = 6.0f * m.xy, dxy3 = 3.0f * m.dxy;
    gx = fmaf(Dc[8], xy6, gx); gy = fmaf(Dc[8], dxy3, gy);
    gx = fmaf(Dc[9], m.yz, gx); gy = fmaf(Dc[9], m.xz, gy); gz = fmaf(Dc[9], m.xy, gz);
    gy = fmaf(Dc[10], m.t5, gy); gz = fmaf(Dc[10], 10.0f * m.yz, gz);
    gz = fmaf(Dc[11], 3.0f * m.t5, gz);
    gx = fmaf(Dc[12], m.t5, gx); gz = fmaf(Dc[12], 10.0f * m.xz, gz);
    gx = fmaf(Dc[13], 2.0f * m.xz, gx); gy = fmaf(Dc[13], -2.0f * m.yz, gy); gz = fmaf(Dc[13], m.dxy, gz);
    gx = fmaf(Dc[14], dxy3, gx); gy = fmaf(Dc[14], -xy6, gy);
    // l = 4
    const float xyz6 = 6.0f * m.xyz, zdxy3 = 3.0f * zdxy;
    gx = fmaf(Dc[15], m.p1, gx); gy = fmaf(Dc[15], m.p2, gy);
    gx = fmaf(Dc[16], xyz6, gx); gy = fmaf(Dc[16], zdxy3, gy); gz = fmaf(Dc[16], m.p1, gz);
    gx = fmaf(Dc[17], yt7, gx); gy = fmaf(Dc[17], xt7, gy); gz = fmaf(Dc[17], 14.0f * m.xyz, gz);
    gy = fmaf(Dc[18], zt73, gy); gz = fmaf(Dc[18], 3.0f * yt7, gz);
    gz = fmaf(Dc[19], 20.0f * zt73, gz);
    gx = fmaf(Dc[20], zt73, gx); gz = fmaf(Dc[20], 3.0f * xt7, gz);
    gx = fmaf(Dc[21], 2.0f * xt7, gx); gy = fmaf(Dc[21], -2.0f * yt7, gy); gz = fmaf(Dc[21], 14.0f * zdxy, gz);
    gx = fmaf(Dc[22], zdxy3, gx); gy = fmaf(Dc[22], -xyz6, gy); gz = fmaf(Dc[22], m.p2, gz);
    gx = fmaf(Dc[23], 4.0f * m.p2, gx); gy = fmaf(Dc[23], -4.0f * m.p1, gy);
    vx = gx; vy = gy; vz = gz;
}

// ---------------------------------------------------------------- ZBL
// Eqs. 2-4 of the paper with the Tersoff switch between r1 and r2, double
// precision.  Returns U and dU/dr for r < r2.
__host__ __device__ inline void zbl_pair(double r, double Z, double r1, double r2, double &U, double &dU)
{
    const double KE = 14.399645478425668;          // e^2 / (4 pi eps0), eV A
    const double a = 0.46848 / (2.0 * pow(Z, 0.23));
    const double inva = 1.0 / a;
    const double c0 = 0.32825, c1 = 0.09219, c2 = 0.58110;
    const double e0 = 2.54931, e1 = 0.29182, e2 = 0.59231;
    const double t0 = c0 * exp(-e0 * r * inva);
    const double t1 = c1 * exp(-e1 * r * inva);
    const double t2 = c2 * exp(-e2 * r * inva);
    const double phi = t0 + t1 + t2;
    const double dphi = -(e0 * t0 + e1 * t1 + e2 * t2) * inva;
    double ft = 1.0, dft = 0.0;
    if (r >= r1) {
        const double w = 3.14159265358979323846 / (r2 - r1);
        ft = 0.5 * (1.0 + cos(w * (r - r1)));
        dft = -0.5 * w * sin(w * (r - r1));
    }
    const double k = KE * Z * Z;
    const double rinv = 1.0 / r;
    U = k * rinv * phi * ft;
    dU = k * rinv * (dphi * ft + phi * dft - phi * ft * rinv);
}

// Bin-offset mode: the entry code of a neighbour in the bin at stencil offset
// q = (o0 + 1) + 3 (o1 + 1) + 9 (o2 + 1), seen through the image m (nonzero
// only on the axes whose periodic face that bin lies across).
__host__ __device__ inline uint32_t delta_code(int q, const int m[3])
{
    return (uint32_t)q | ((uint32_t)((m[0] != 0) | ((m[1] != 0) << 1) | ((m[2] != 0) << 2)) << 5);
}

// ---------------------------------------------------------------- neighbours
__host__ __device__ inline void decode_entry(int32_t e, int jbits, int ibits, int ioff, int &j, int &n0,
                                    int &n1, int &n2)
{
    const uint32_t u = (uint32_t)e;
    j = (int)(u & ((1u << jbits) - 1u));
    const uint32_t code = u >> jbits;
    const uint32_t m = (1u << ibits) - 1u;
    n0 = (int)(code & m) - ioff;
    n1 = (int)((code >> ibits) & m) - ioff;
    n2 = (int)(code >> (2 * ibits)) - ioff;
}

// XCD-aware block order: the hardware dispatches workgroups round-robin over
// the 8 XCDs, so launched block b runs on XCD b % 8.  Mapping it to logical
// tile (b % 8) * per + b / 8 gives every XCD one contiguous run of tiles, so
// spatially adjacent atom tiles share one L2.  The grid must be launched with
// 8 * per blocks (per = ceil(tiles / 8)); logical tiles >= tiles do nothing.
// Batcher's odd-even merge sort of 32 keys, ascending (191 compare-exchange
// steps); every index is a compile-time constant once the loops are
// unrolled, so on the GPU the keys stay in registers.
__host__ __device__ inline void sort32(uint32_t a[32])
{
#pragma unroll
    for (int p = 1; p < 32; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < 32; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < 32 && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const uint32_t x = a[i + j], y = a[i + j + k];
                        a[i + j] = x < y ? x : y;
                        a[i + j + k] = x < y ? y : x;
                    }
}

__device__ inline int xcd_block(int ntiles)
{
    const int b = blockIdx.x;
    const int per = (ntiles + 7) / 8;
    return (b % 8) * per + b / 8;
}


// ---------------------------------------------------------------- bin blocks
// The aligned 2 x 2 x 2 blocks of a cell's bin grid (8 consecutive Morton
// codes) and their halo, the bins within one bin of a block: halo
// coordinates d = 0..3 per axis name bin 2 B - 1 + d of block B.
__host__ __device__ inline int halo_index(int d0, int d1, int d2) { return (d2 * 4 + d1) * 4 + d0; }
constexpr int LB_BS = 256;   // threads per block of the list build by bin blocks

__host__ __device__ inline uint32_t pack_block(int b0, int b1, int b2)
{
    return (uint32_t)b0 | ((uint32_t)b1 << 10) | ((uint32_t)b2 << 20);
}

__host__ __device__ inline void unpack_block(uint32_t p, int b[3])
{
    b[0] = (int)(p & 1023u);
    b[1] = (int)((p >> 10) & 1023u);
    b[2] = (int)(p >> 20);
}

}  // namespace nep
