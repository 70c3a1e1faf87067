// Neighbour-list walking and pair geometry shared by the kernel files:
// list slot order, multiply-free slot walks, the software pipeline over a
// list, FP64 pair vectors (exactly antisymmetric) and distances.
#pragma once
#include "nep_device.h"

namespace nep {

// slot of the s-th entry of a list stored front-to-back (nf entries) and
// back-to-front (nb entries) in a column of capacity cap
__host__ __device__ inline int list_slot(int s, int nf, int nb, int cap)
{
    return s < nf ? s : s + (cap - nf - nb);
}

// The same slots walked in order as element offsets slot * n + t of a
// [slot][atom] array, with one 64-bit add per entry instead of a multiply:
//   for (ListWalk w(t, n, nf, nb, cap); w.s < nf + nb; w.next()) ... a[w.off] ...
struct ListWalk {
    size_t off, n, jump;
    int s, nf;
    __host__ __device__ ListWalk(int t, int n_, int nf_, int nb, int cap)
        : off(0), n((size_t)n_), jump((size_t)(cap - nf_ - nb) * (size_t)n_), s(0), nf(nf_)
    {
        off = (size_t)t + (nf_ == 0 ? jump : 0);
    }
    __host__ __device__ void next()
    {
        ++s;
        off += n + (s == nf ? jump : 0);
    }
};

__device__ inline float ftanh(float z)
{
    // tanh z = 1 - 2 / (exp(2z) + 1); exp via the hardware base-2 exponential
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * z);   // 2 log2(e) z
    return 1.0f - 2.0f * frcp(e + 1.0f);
}

// ------------------------------------------------------------------ descriptor + network

// The image shift n.h of a list entry added to a pair vector.  Entries in the
// cell itself (all but those across a periodic face) carry the code code0,
// or in bin-offset mode no crossing bits, and are recognised by one
// comparison before the code is decoded.
__device__ __forceinline__ void add_image(int32_t e, const PairConsts &pc, const CellGeom *__restrict__ cg,
                                          double &dx, double &dy, double &dz)
{
    const uint32_t code = (uint32_t)e >> pc.jbits;
    if ((code & pc.img_mask) == pc.img_val) return;
    int n0, n1, n2;
    if (pc.delta) {
        const uint32_t cr = code >> 5;
        const int q = (int)(code & 31u);
        n0 = (cr & 1u) ? q % 3 - 1 : 0;
        n1 = (cr & 2u) ? (q / 3) % 3 - 1 : 0;
        n2 = (cr & 4u) ? q / 9 - 1 : 0;
    } else {
        const uint32_t m = (1u << pc.ibits) - 1u;
        n0 = (int)(code & m) - pc.ioff;
        n1 = (int)((code >> pc.ibits) & m) - pc.ioff;
        n2 = (int)(code >> (2 * pc.ibits)) - pc.ioff;
    }
    const double *h = cg->h;
    dx += n0 * h[0] + n1 * h[3] + n2 * h[6];
    dy += n0 * h[1] + n1 * h[4] + n2 * h[7];
    dz += n0 * h[2] + n1 * h[5] + n2 * h[8];
}


// Bin-offset mode: the 27 vectors o0 b0 + o1 b1 + o2 b2 of the neighbour-bin
// offsets o in {-1, 0, 1}^3 (b_a the bin edge vectors, index
// q = (o0+1) + 3 (o1+1) + 9 (o2+1)), staged in LDS by every thread of the
// block, 4 doubles per entry (two aligned LDS reads).  Entry 26 - q is the
// exact negative of entry q (products and sums negate exactly), so pair
// vectors formed from the table stay antisymmetric.  Ends with a barrier:
// call it before any thread of the block can leave.
constexpr int BIN_TAB = 27 * 4;
__device__ __forceinline__ void stage_bin_vectors(const CellGeom *__restrict__ cg, double *__restrict__ tab)
{
    for (int q = (int)threadIdx.x; q < 27; q += (int)blockDim.x) {
        const double o0 = q % 3 - 1, o1 = (q / 3) % 3 - 1, o2 = q / 9 - 1;
        const double *bv = cg->bv;
#pragma unroll
        for (int d = 0; d < 3; ++d) tab[4 * q + d] = o0 * bv[d] + o1 * bv[3 + d] + o2 * bv[6 + d];
        tab[4 * q + 3] = 0.0;
    }
    __syncthreads();
}

// Pair vector in double precision, computed so that the vector seen from the
// other end of the pair is its exact negative: (x_j - x_i) first, then the
// image shift n.h (which is exactly negated for -n).
__device__ inline void pair_vector_d(int32_t e, const PairConsts &pc, int base, double xi, double yi,
                                     double zi, const double4 *__restrict__ xq,
                                     const CellGeom *__restrict__ cg, int &j, double &dx, double &dy,
                                     double &dz)
{
    j = (int)((uint32_t)e & ((1u << pc.jbits) - 1u)) + base;
    const double4 pj = xq[j];
    dx = pj.x - xi;
    dy = pj.y - yi;
    dz = pj.z - zi;
    add_image(e, pc, cg, dx, dy, dz);
}

// The same pair vector from a neighbour position already gathered.
__device__ inline void pair_vector_p(int32_t e, const PairConsts &pc, double px, double py, double pz, double xi,
                                     double yi, double zi, const CellGeom *__restrict__ cg, double &dx, double &dy,
                                     double &dz)
{
    dx = px - xi;
    dy = py - yi;
    dz = pz - zi;
    add_image(e, pc, cg, dx, dy, dz);
}

// Software pipeline over one atom's list: entries are loaded two neighbours
// ahead and the neighbour's position one ahead, so the dependent gathers of
// the next neighbours overlap the arithmetic of the current one.
//   for (NeighbourPipe q(...); q.s < q.count;) { q.pop(...); ... }
struct NeighbourPipe {
    ListWalk w;
    int count, s;
    int32_t e_cur, e_nx;
    double x_cur, y_cur, z_cur;
    __device__ NeighbourPipe(const int32_t *__restrict__ nl, const double4 *__restrict__ xq, int base,
                             uint32_t jmask, int t, int n, int nf, int nb, int cap)
        : w(t, n, nf, nb, cap), count(nf + nb), s(0), e_cur(0), e_nx(0), x_cur(0.0), y_cur(0.0), z_cur(0.0)
    {
        if (count > 0) {
            e_cur = nl[w.off];
            const double4 *q = xq + ((int)((uint32_t)e_cur & jmask) + base);
            x_cur = q->x; y_cur = q->y; z_cur = q->z;
        }
        w.next();
        if (w.s < count) e_nx = nl[w.off];
    }
    __device__ void pop(const int32_t *__restrict__ nl, const double4 *__restrict__ xq, int base, uint32_t jmask,
                        int32_t &e, double &px, double &py, double &pz)
    {
        e = e_cur; px = x_cur; py = y_cur; pz = z_cur;
        if (s + 1 < count) {
            e_cur = e_nx;
            const double4 *q = xq + ((int)((uint32_t)e_cur & jmask) + base);
            x_cur = q->x; y_cur = q->y; z_cur = q->z;
            w.next();
            if (w.s < count) e_nx = nl[w.off];
        }
        ++s;
    }
};

// Inside-cutoff bits of a list walked in order: bit s of word s/32 for entry
// s, each word stored once to mask[word * n + t] when complete.
struct MaskWriter {
    uint32_t word = 0;
    __device__ void add(uint32_t *__restrict__ mask, size_t n, int t, int s, int count, bool inside)
    {
        word |= (uint32_t)inside << (s & 31);
        if ((s & 31) == 31 || s + 1 == count) {
            mask[(size_t)(s >> 5) * n + t] = word;
            word = 0;
        }
    }
};

// The same bits when only some entries are visited (in increasing order):
// set(s) marks entry s, and every word up to the last is stored once.
struct SparseMaskWriter {
    uint32_t *__restrict__ mask;
    size_t n;
    int t, nw, w;
    uint32_t bits;
    __device__ SparseMaskWriter(uint32_t *__restrict__ m, int n_, int t_, int count)
        : mask(m), n((size_t)n_), t(t_), nw((count + 31) >> 5), w(0), bits(0)
    {
    }
    __device__ void set(int s)
    {
        const int ws = s >> 5;
        while (w < ws) {
            mask[(size_t)w * n + t] = bits;
            bits = 0;
            ++w;
        }
        bits |= 1u << (s & 31);
    }
    __device__ void finish()
    {
        while (w < nw) {
            mask[(size_t)w * n + t] = bits;
            bits = 0;
            ++w;
        }
    }
};

// The set bits of those words in order: next() returns the next entry index
// inside the cutoff, or -1.
struct MaskWalk {
    const uint32_t *__restrict__ mask;
    size_t n;
    int t, nw, w;
    uint32_t bits;
    __device__ MaskWalk(const uint32_t *__restrict__ m, int n_, int t_, int count)
        : mask(m), n((size_t)n_), t(t_), nw((count + 31) >> 5), w(0), bits(0)
    {
        if (nw > 0) bits = mask[(size_t)t];
    }
    __device__ int next()
    {
        while (bits == 0) {
            if (++w >= nw) return -1;
            bits = mask[(size_t)w * n + t];
        }
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        return (w << 5) + b;
    }
};

// The software pipeline of NeighbourPipe over the entries a MaskWalk yields
// (entry index s, slot offset off(s) = slot * n + t).
//   for (MaskPipe q(...); q.valid();) { q.pop(..., s); ... }
struct MaskPipe {
    MaskWalk mw;
    size_t n;
    int t, nf, nb, cap;
    int s_cur, s_nx;
    int32_t e_cur, e_nx;
    double x_cur, y_cur, z_cur;
    __device__ size_t off(int s) const { return (size_t)list_slot(s, nf, nb, cap) * n + t; }
    __device__ MaskPipe(const uint32_t *__restrict__ mask, const int32_t *__restrict__ nl,
                        const double4 *__restrict__ xq, int base, uint32_t jmask, int t_, int n_, int nf_, int nb_,
                        int cap_)
        : mw(mask, n_, t_, nf_ + nb_), n((size_t)n_), t(t_), nf(nf_), nb(nb_), cap(cap_), e_cur(0), e_nx(0),
          x_cur(0.0), y_cur(0.0), z_cur(0.0)
    {
        s_cur = mw.next();
        if (s_cur >= 0) {
            e_cur = nl[off(s_cur)];
            const double4 *q = xq + ((int)((uint32_t)e_cur & jmask) + base);
            x_cur = q->x; y_cur = q->y; z_cur = q->z;
        }
        s_nx = mw.next();
        if (s_nx >= 0) e_nx = nl[off(s_nx)];
    }
    __device__ bool valid() const { return s_cur >= 0; }
    __device__ void pop(const int32_t *__restrict__ nl, const double4 *__restrict__ xq, int base, uint32_t jmask,
                        int32_t &e, double &px, double &py, double &pz, int &s)
    {
        e = e_cur; px = x_cur; py = y_cur; pz = z_cur; s = s_cur;
        s_cur = s_nx;
        if (s_cur >= 0) {
            e_cur = e_nx;
            const double4 *q = xq + ((int)((uint32_t)e_cur & jmask) + base);
            x_cur = q->x; y_cur = q->y; z_cur = q->z;
            s_nx = mw.next();
            if (s_nx >= 0) e_nx = nl[off(s_nx)];
        }
    }
};

// |r| in double precision from r^2: FP32 square root refined by one
// Newton step (relative error ~1e-15).
__device__ inline double dist_d(double r2)
{
    const float rf = fsqrt((float)r2);
    const double rd = (double)rf;
    return rd + fma(-rd, rd, r2) * (double)(0.5f * frcp(rf));
}

}  // namespace nep
