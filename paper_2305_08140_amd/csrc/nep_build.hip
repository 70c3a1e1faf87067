// Cell list, neighbour lists and velocity-Verlet kernels (gfx950).
//
// Cell list: every cell of the batch gets its own bin grid.  Along an axis
// whose perpendicular width is at least 3 (rc + skin) the cell is cut into
// nb >= 3 bins of width >= rc + skin and the search visits the bins b-1..b+1
// (with periodic wrap); a narrower periodic axis gets one bin and the search
// loops over the explicit images -R..R, R = ceil((rc + skin) / width), which
// covers every image within reach (small cells see several images of the same
// atom and their own images).  Atoms are counting-sorted by bin (stable in the
// caller's index), and their wrapped FP64 positions are stored in that order.
//
// Neighbour lists: per atom two fixed-capacity columns (stored transposed,
// [slot][atom], so that a wavefront reads them coalesced):
//   angular list   r < rc_ang + skin:  r < rc_ang filled from the front,
//                                      the skin shell from the back
//   radial list    rc_ang + skin <= r < rc_rad + skin: r < rc_rad from the
//                                      front, the skin shell from the back
// so that the pair loops meet the inside-cutoff entries first and in the
// same order on all lanes (little divergence).  With the 3 x 3 x 3 bin search
// the bins are visited in the order their atoms are stored, so each part of a
// list is ascending in the neighbour's index: neighbouring atoms of a
// wavefront then gather nearby records at the same slot, which shares cache
// lines between lanes (3.5 % off the descriptor kernel, 2.5 % off the force
// kernel at 8.2 M atoms).  An entry packs the neighbour's index within its
// cell (jbits bits) with the image n in 3 fields of ibits.
#include "nep_device.h"

namespace nep {

// ------------------------------------------------------------------ binning

__device__ inline int pack_wrap(int w0, int w1, int w2)
{
    return ((w0 + 512) & 1023) | (((w1 + 512) & 1023) << 10) | (((w2 + 512) & 1023) << 20);
}

__device__ inline void unpack_wrap(int p, int &w0, int &w1, int &w2)
{
    w0 = (p & 1023) - 512;
    w1 = ((p >> 10) & 1023) - 512;
    w2 = ((p >> 20) & 1023) - 512;
}

__global__ void k_fill_i32(int n, int32_t *__restrict__ a, int32_t v, const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// Per atom (caller order): bin, wrap count, bin histogram, reference position.
// Bins are numbered along a Morton curve within each cell (bin_rank maps the
// x-fastest linear bin index to that order), so that a run of consecutive
// sorted atoms occupies a compact 3D region and its neighbour halo fits L2.
__global__ void k_bin_assign(int n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, const int32_t *__restrict__ cell_of,
                             const CellGeom *__restrict__ cells, int32_t *__restrict__ bin_of,
                             int32_t *__restrict__ wrap, int32_t *__restrict__ bin_count,
                             double *__restrict__ xref, const int32_t *__restrict__ bin_rank,
                             int32_t *__restrict__ status, const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CellGeom &cg = cells[cell_of[i]];
    const double p[3] = {x[i], y[i], z[i]};
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) {
        latch_error(status, -5);
        bin_of[i] = cg.bin_offset;
        wrap[i] = pack_wrap(0, 0, 0);
        atomicAdd(bin_count + cg.bin_offset, 1);
        return;
    }
    int w[3], b[3];
    for (int a = 0; a < 3; ++a) {
        double s = p[0] * cg.hinv[a] + p[1] * cg.hinv[3 + a] + p[2] * cg.hinv[6 + a];
        w[a] = 0;
        if (cg.periodic[a]) {
            const double fl = floor(s);
            w[a] = (int)fl;
            s -= fl;
        }
        int bb = (int)floor(s * cg.nb[a]);
        bb = bb < 0 ? 0 : (bb >= cg.nb[a] ? cg.nb[a] - 1 : bb);
        b[a] = bb;
        if (w[a] < -511 || w[a] > 511) latch_error(status, -1);
    }
    const int lin = (b[2] * cg.nb[1] + b[1]) * cg.nb[0] + b[0];
    const int gb = cg.bin_offset + bin_rank[cg.bin_offset + lin];
    bin_of[i] = gb;
    wrap[i] = pack_wrap(w[0], w[1], w[2]);
    atomicAdd(bin_count + gb, 1);
    xref[i] = p[0];
    xref[(size_t)n + i] = p[1];
    xref[2 * (size_t)n + i] = p[2];
}

// Exclusive scan, three phases: 2048-element block scans, a serial scan of
// the block sums (one block, in chunks), and the block offsets added back.
__global__ __launch_bounds__(256) void k_scan_blocks(int n, const int32_t *__restrict__ in,
                                                     int32_t *__restrict__ out,
                                                     int32_t *__restrict__ sums,
                                                     const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    __shared__ int32_t sh[256];
    const int base = blockIdx.x * 2048 + threadIdx.x * 8;
    int32_t v[8], s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = sh[threadIdx.x] - s;   // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void k_scan_sums(int nb, int32_t *__restrict__ sums,
                                                   const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    __shared__ int32_t sh[256];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 256) {
        const int k = c0 + threadIdx.x;
        const int32_t v = k < nb ? sums[k] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < nb) sums[k] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += sh[255];
        __syncthreads();
    }
}

__global__ void k_scan_add(int n, int32_t *__restrict__ out, const int32_t *__restrict__ sums,
                           const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] += sums[t / 2048];
}

// Scatter atoms into their bins (arbitrary order within a bin).
__global__ void k_bin_scatter(int n, const int32_t *__restrict__ bin_of,
                              const int32_t *__restrict__ bin_start, int32_t *__restrict__ fill,
                              int32_t *__restrict__ tmp, const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = bin_of[i];
    const int slot = atomicAdd(fill + b, 1);
    tmp[bin_start[b] + slot] = i;
}

// Stable order within each bin: an atom's rank is the number of atoms of its
// bin with a smaller caller index.  Also records the sorted atom's local bin.
__global__ void k_bin_rank(int n, const int32_t *__restrict__ bin_of,
                           const int32_t *__restrict__ bin_start, const int32_t *__restrict__ tmp,
                           const int32_t *__restrict__ cell_of, const CellGeom *__restrict__ cells,
                           int32_t *__restrict__ perm, int32_t *__restrict__ bin_sorted,
                           const int32_t *__restrict__ bin_lin, const int32_t *__restrict__ flag)
{
    if (flag && *flag == 0) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = tmp[p];
    const int b = bin_of[i];
    const int b0 = bin_start[b], b1 = bin_start[b + 1];
    int rank = 0;
    for (int q = b0; q < b1; ++q) rank += tmp[q] < i;
    perm[b0 + rank] = i;
    bin_sorted[b0 + rank] = bin_lin[b];   // x-fastest linear index of the bin within its cell
}

// Wrapped positions in sorted order: xq[t] = x[perm[t]] - w . h, 32-byte
// records (four atoms per 128-byte line).  Runs at every evaluation (and
// in a build, when `flag` is non-null and set); non-finite positions latch
// NEP_E_NONFINITE.  With xf set (the paper-size model in bin-offset mode,
// one cell) also the 16-byte fixed-point form its walks gather: offsets
// from the corner of the atom's bin of the last build in units 1/qsinv (an
// offset beyond the 32-bit range means the atom left its bin by far more
// than the skin: error -9).
__global__ void k_sort_positions(int n, const int32_t *__restrict__ perm,
                                 const double *__restrict__ x, const double *__restrict__ y,
                                 const double *__restrict__ z, const int32_t *__restrict__ wrap,
                                 const int32_t *__restrict__ cell_of,
                                 const CellGeom *__restrict__ cells, double4 *__restrict__ xq,
                                 int32_t *__restrict__ status, const int32_t *__restrict__ flag,
                                 const int32_t *__restrict__ bin_sorted, double qsinv, int4 *__restrict__ xf)
{
    if (flag && *flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = perm[t];
    int w0, w1, w2;
    unpack_wrap(wrap[i], w0, w1, w2);
    const double *h = cells[cell_of[t]].h;
    const double px = x[i], py = y[i], pz = z[i];
    if (!isfinite(px) || !isfinite(py) || !isfinite(pz)) latch_error(status, -5);
    const double wx = px - (w0 * h[0] + w1 * h[3] + w2 * h[6]);
    const double wy = py - (w0 * h[1] + w1 * h[4] + w2 * h[7]);
    const double wz = pz - (w0 * h[2] + w1 * h[5] + w2 * h[8]);
    xq[t] = make_double4(wx, wy, wz, 0.0);
    if (xf) {
        const CellGeom &cg = cells[0];
        const int lbin = bin_sorted[t];
        const int b0 = lbin % cg.nb[0], b1 = (lbin / cg.nb[0]) % cg.nb[1], b2 = lbin / (cg.nb[0] * cg.nb[1]);
        const double *bv = cg.bv;
        const double d[3] = {wx - (b0 * bv[0] + b1 * bv[3] + b2 * bv[6]), wy - (b0 * bv[1] + b1 * bv[4] + b2 * bv[7]),
                             wz - (b0 * bv[2] + b1 * bv[5] + b2 * bv[8])};
        int o[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = rint(d[k] * qsinv);
            if (!(fabs(v) < 2147483000.0)) latch_error(status, -9);
            o[k] = (int)fmin(fmax(v, -2147483000.0), 2147483000.0);
        }
        xf[t] = make_int4(o[0], o[1], o[2], 0);
    }
}

// One atom's list build: the candidates of each visited bin are offered in
// turn, and the entries are written to the front (inside the cutoff at build
// time) or the back (skin shell) of the atom's angular or radial column.
struct ListBuilder {
    const PairConsts &pc;
    double lA2, lR2, cA2, cR2;
    int t, atom_start;
    double xi, yi, zi;
    int32_t *nl_ang, *nl_rad;
    int32_t *status;
    uint64_t cntA = 0, cntR = 0;   // front | back << 32 (kept in registers)
    __device__ ListBuilder(const PairConsts &pc_, double lA2_, double lR2_, double cA2_, double cR2_, int t_,
                           int atom_start_, double4 pi, int32_t *nl_ang_, int32_t *nl_rad_, int32_t *status_)
        : pc(pc_), lA2(lA2_), lR2(lR2_), cA2(cA2_), cR2(cR2_), t(t_), atom_start(atom_start_), xi(pi.x), yi(pi.y),
          zi(pi.z), nl_ang(nl_ang_), nl_rad(nl_rad_), status(status_)
    {
    }
    // squared distance to a candidate at pu seen through the image shift:
    // (x_u - x_i) + shift, exactly the negative of the vector seen from u
    __device__ __forceinline__ double dist2(const double4 &pu, double sx, double sy, double sz) const
    {
        const double dx = (pu.x - xi) + sx, dy = (pu.y - yi) + sy, dz = (pu.z - zi) + sz;
        return dx * dx + dy * dy + dz * dz;
    }
    // candidate u (sorted index) at position pu, seen through the image
    // shift (sx, sy, sz) whose entry code is `code`
    __device__ __forceinline__ void offer(int u, const double4 &pu, double sx, double sy, double sz, uint32_t code)
    {
        const double r2 = dist2(pu, sx, sy, sz);
        if (r2 >= lR2) return;
        const uint32_t jl = (uint32_t)(u - atom_start);
        const int32_t e = (int32_t)(jl | (code << pc.jbits));
        if (jl >= (1u << pc.jbits)) latch_error(status, -1);
        const bool ang = r2 < lA2;
        const bool front = r2 < (ang ? cA2 : cR2);
        const uint64_t cnt = ang ? cntA : cntR;
        const int f = (int)(cnt & 0xffffffffu), b = (int)(cnt >> 32), cap = ang ? pc.capA : pc.capR;
        if (f + b < cap) (ang ? nl_ang : nl_rad)[(size_t)(front ? f : cap - 1 - b) * pc.n + t] = e;
        const uint64_t inc = front ? 1ull : (1ull << 32);
        cntA += ang ? inc : 0ull;
        cntR += ang ? 0ull : inc;
    }
    // the entry code of a neighbour in the bin at stencil offset q (bin-offset
    // mode) or seen through the image m (otherwise)
    __device__ uint32_t entry_code(int q, const int m[3]) const
    {
        return pc.delta ? delta_code(q, m) : image_code(m);
    }
    __device__ uint32_t image_code(const int m[3]) const
    {
        return (uint32_t)(m[0] + pc.ioff) | ((uint32_t)(m[1] + pc.ioff) << pc.ibits) |
               ((uint32_t)(m[2] + pc.ioff) << (2 * pc.ibits));
    }
    // counts (clamped to the capacities after an overflow, which is latched
    // with the lengths needed)
    __device__ void finish(uint32_t *ncnt)
    {
        int naf = (int)(cntA & 0xffffffffu), nab = (int)(cntA >> 32);
        int nrf = (int)(cntR & 0xffffffffu), nrb = (int)(cntR >> 32);
        const int nA = naf + nab, nR = nrf + nrb;
        if (nA > pc.capA || nR > pc.capR) {
            latch_error(status, -3);
            if (nA > pc.capA) { naf = naf < pc.capA ? naf : pc.capA; nab = pc.capA - naf; }
            if (nR > pc.capR) { nrf = nrf < pc.capR ? nrf : pc.capR; nrb = pc.capR - nrf; }
        }
        atomicMax(status + ST_NEED_A, nA);
        atomicMax(status + ST_NEED_R, nR);
        ncnt[t] = (uint32_t)naf | ((uint32_t)nab << 8) | ((uint32_t)nrf << 16) | ((uint32_t)nrb << 24);
    }
};

// Neighbour lists of every sorted atom (see the file comment for the layout).
__global__ __launch_bounds__(256) void k_build_lists(
    PairConsts pc, double lA2, double lR2, double cA2, double cR2, const double4 *__restrict__ xq,
    const int32_t *__restrict__ cell_of, const CellGeom *__restrict__ cells,
    const int32_t *__restrict__ bin_sorted, const int32_t *__restrict__ bin_start,
    const int32_t *__restrict__ bin_rank,
    int32_t *__restrict__ nl_ang, int32_t *__restrict__ nl_rad, uint32_t *__restrict__ ncnt,
    int32_t *__restrict__ status, const int32_t *__restrict__ flag, int sorted_scan)
{
    if (flag && *flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pc.n) return;
    const CellGeom &cg = cells[cell_of[t]];
    ListBuilder lb(pc, lA2, lR2, cA2, cR2, t, cg.atom_start, xq[t], nl_ang, nl_rad, status);
    const int lbin = bin_sorted[t];
    const int bc[3] = {lbin % cg.nb[0], (lbin / cg.nb[0]) % cg.nb[1], lbin / (cg.nb[0] * cg.nb[1])};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (cg.R[a] > 0) { lo[a] = -cg.R[a]; hi[a] = cg.R[a]; }
        else { lo[a] = -1; hi[a] = 1; }
    }
    // bin of offset o from this atom's bin: global bin index (or -1 past an
    // open face) and the image m it lies in
    auto bin_at = [&](int o0, int o1, int o2, int m[3]) __attribute__((always_inline)) -> int {
        const int o[3] = {o0, o1, o2};
        int bb[3];
        bool out = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (cg.R[a] > 0) { bb[a] = 0; m[a] = o[a]; }
            else {
                int b = bc[a] + o[a];
                m[a] = 0;
                if (cg.periodic[a]) {
                    if (b < 0) { b += cg.nb[a]; m[a] = -1; }
                    else if (b >= cg.nb[a]) { b -= cg.nb[a]; m[a] = 1; }
                } else if (b < 0 || b >= cg.nb[a]) out = true;
                bb[a] = b;
            }
        }
        if (out) return -1;
        return cg.bin_offset + bin_rank[cg.bin_offset + (bb[2] * cg.nb[1] + bb[1]) * cg.nb[0] + bb[0]];
    };
    auto scan_bin = [&](int gb, int q, const int m[3]) __attribute__((always_inline)) {
        const double sx = m[0] * cg.h[0] + m[1] * cg.h[3] + m[2] * cg.h[6];
        const double sy = m[0] * cg.h[1] + m[1] * cg.h[4] + m[2] * cg.h[7];
        const double sz = m[0] * cg.h[2] + m[1] * cg.h[5] + m[2] * cg.h[8];
        const bool self_image = (m[0] | m[1] | m[2]) == 0;
        const uint32_t code = lb.entry_code(q, m);
        for (int u = bin_start[gb]; u < bin_start[gb + 1]; ++u) {
            if (u == t && self_image) continue;
            lb.offer(u, xq[u], sx, sy, sz, code);
        }
    };
    if (sorted_scan && cg.R[0] == 0 && cg.R[1] == 0 && cg.R[2] == 0) {
        // the 3 x 3 x 3 neighbour bins in the order their atoms are stored,
        // so that every list is ascending in the neighbour index and the
        // lists of nearby atoms gather nearby records at equal slots.  Keys
        // (bin << 5 | offset) sorted by an odd-even merge network in registers.
        uint32_t key[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            key[q] = 0xffffffffu;
            if (q < 27) {
                int m[3];
                const int gb = bin_at(q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1, m);
                if (gb >= 0) key[q] = ((uint32_t)gb << 5) | (uint32_t)q;
            }
        }
        sort32(key);
        for (int k = 0; k < 27; ++k) {
            const uint32_t kq = key[0];
#pragma unroll
            for (int q = 0; q < 31; ++q) key[q] = key[q + 1];
            if (kq == 0xffffffffu) break;
            const int q = (int)(kq & 31u);
            int m[3];
            const int gb = bin_at(q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1, m);
            scan_bin(gb, q, m);
        }
    } else {
        for (int o2 = lo[2]; o2 <= hi[2]; ++o2)
            for (int o1 = lo[1]; o1 <= hi[1]; ++o1)
                for (int o0 = lo[0]; o0 <= hi[0]; ++o0) {
                    int m[3];
                    const int gb = bin_at(o0, o1, o2, m);
                    // (the stencil offset names the bin only with every axis binned)
                    if (gb >= 0) scan_bin(gb, (o0 + 1) + 3 * (o1 + 1) + 9 * (o2 + 1), m);
                }
    }
    lb.finish(ncnt);
}

// The same lists for one large binned cell (at least 4 bins along every
// periodic axis), built by bin blocks: a workgroup takes the aligned
// 2 x 2 x 2 block of bins k (8 consecutive Morton codes, so its atoms are one
// contiguous run), copies the positions of the block's halo (the bins within
// one bin of it, up to 4 x 4 x 4, each a contiguous run) into LDS once, and
// every atom of the block then scans its 27 neighbour bins there instead of
// gathering each candidate from memory (~600 candidates per atom, 22 atoms
// per bin at the bcc density).  Bins are visited in storage order and every
// candidate goes through the same ListBuilder as above, so the lists are
// identical to k_build_lists's.  A block whose halo exceeds the LDS copy
// gathers from memory.
constexpr int LB_CAP = 1600;     // halo positions per block in LDS (51 KB)
__global__ __launch_bounds__(LB_BS) void k_build_lists_blocks(
    PairConsts pc, double lA2, double lR2, double cA2, double cR2, const double4 *__restrict__ xq,
    const CellGeom *__restrict__ cells, const int32_t *__restrict__ bin_sorted,
    const int32_t *__restrict__ bin_start, const int32_t *__restrict__ bin_rank,
    const uint32_t *__restrict__ blk_coord, int nblocks, int32_t *__restrict__ nl_ang,
    int32_t *__restrict__ nl_rad, uint32_t *__restrict__ ncnt, int32_t *__restrict__ status,
    const int32_t *__restrict__ flag)
{
    __shared__ double4 pos[LB_CAP];
    __shared__ int s_off[65], s_gst[64], s_gb[64], s_a[2];
    if (flag && *flag == 0) return;
    const int k = xcd_block(nblocks);
    if (k >= nblocks) return;
    const int tid = threadIdx.x;
    const CellGeom &cg = cells[0];
    int B[3];
    unpack_block(blk_coord[k], B);
    if (tid < 64) {
        // halo bin hb = tid at halo coordinates d (bin 2 B - 1 + d): absent
        // beyond an open face and past the far side of a block one bin wide
        const int hb = tid;
        const int d[3] = {hb & 3, (hb >> 2) & 3, hb >> 4};
        bool present = true, own = true;
        int bb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int width = min(2, cg.nb[a] - 2 * B[a]);
            if (d[a] > width + 1) present = false;
            if (d[a] < 1 || d[a] > width) own = false;
            int u = 2 * B[a] - 1 + d[a];
            if (cg.periodic[a]) u = u < 0 ? u + cg.nb[a] : (u >= cg.nb[a] ? u - cg.nb[a] : u);
            else if (u < 0 || u >= cg.nb[a]) present = false;
            bb[a] = u;
        }
        int cnt = 0, gst = 0, gb = -1;
        if (present) {
            gb = cg.bin_offset + bin_rank[cg.bin_offset + (bb[2] * cg.nb[1] + bb[1]) * cg.nb[0] + bb[0]];
            gst = bin_start[gb];
            cnt = bin_start[gb + 1] - gst;
        }
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (hb >= o) incl += v;
        }
        int a0 = own ? gst : INT32_MAX, a1 = own ? gst + cnt : INT32_MIN;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a0 = min(a0, __shfl_xor(a0, o));
            a1 = max(a1, __shfl_xor(a1, o));
        }
        s_off[hb] = incl - cnt;
        s_gst[hb] = gst;
        s_gb[hb] = gb;
        if (hb == 63) s_off[64] = incl;
        if (hb == 0) { s_a[0] = a0 <= a1 ? a0 : 0; s_a[1] = a0 <= a1 ? a1 : 0; }
    }
    __syncthreads();
    const int total = s_off[64];
    const bool staged = total <= LB_CAP;
    if (staged) {
        for (int r = tid; r < total; r += LB_BS) {
            // halo bin holding record r: the last hb with s_off[hb] <= r
            int lo = 0, hi = 64;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= r) lo = mid;
                else hi = mid;
            }
            pos[r] = xq[s_gst[lo] + (r - s_off[lo])];
        }
    }
    __syncthreads();
    // Bins out of reach: along a periodic axis of a cell with a diagonal h,
    // a neighbour bin's atoms lie beyond the shared face (up to the rounding
    // of the binning, covered by eps), so an atom at distance p from its own
    // bin's lower face is at least p (offset -1) or w - p (offset +1) from
    // them; a bin whose nearest point is outside the list cutoff holds no
    // entry and is skipped (the lists are unchanged).
    const bool diag = cg.h[1] == 0.0 && cg.h[2] == 0.0 && cg.h[3] == 0.0 && cg.h[5] == 0.0 && cg.h[6] == 0.0 &&
                      cg.h[7] == 0.0;
    double bw[3];
    bool prune[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bw[a] = cg.h[4 * a] / cg.nb[a];
        prune[a] = diag && cg.periodic[a];
    }
    for (int t = s_a[0] + tid; t < s_a[1]; t += LB_BS) {
        const double4 pt = xq[t];
        ListBuilder lb(pc, lA2, lR2, cA2, cR2, t, cg.atom_start, pt, nl_ang, nl_rad, status);
        const int lbin = bin_sorted[t];
        const int bc[3] = {lbin % cg.nb[0], (lbin / cg.nb[0]) % cg.nb[1], lbin / (cg.nb[0] * cg.nb[1])};
        // distances to the lower and upper faces of the own bin (0 where no
        // pruning applies)
        double dlo[3], dhi[3];
        {
            const double pa[3] = {pt.x, pt.y, pt.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double eps = 1e-9 * cg.h[4 * a];
                const double p = pa[a] - bc[a] * bw[a];
                dlo[a] = prune[a] ? fmax(p - eps, 0.0) : 0.0;
                dhi[a] = prune[a] ? fmax(bw[a] - p - eps, 0.0) : 0.0;
            }
        }
        // the 27 neighbour bins in storage order (keys gb << 5 | offset)
        uint32_t key[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            key[q] = 0xffffffffu;
            if (q < 27) {
                const int o[3] = {q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1};
                const int hb = halo_index(bc[0] - 2 * B[0] + 1 + o[0], bc[1] - 2 * B[1] + 1 + o[1],
                                          bc[2] - 2 * B[2] + 1 + o[2]);
                if (s_gb[hb] >= 0) key[q] = ((uint32_t)s_gb[hb] << 5) | (uint32_t)q;
            }
        }
        sort32(key);
        for (int kk = 0; kk < 27; ++kk) {
            const uint32_t kq = key[0];
#pragma unroll
            for (int q = 0; q < 31; ++q) key[q] = key[q + 1];
            if (kq == 0xffffffffu) break;
            const int q = (int)(kq & 31u);
            const int o[3] = {q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1};
            {
                double d2 = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double d = o[a] < 0 ? dlo[a] : (o[a] > 0 ? dhi[a] : 0.0);
                    d2 = fma(d, d, d2);
                }
                if (d2 >= lR2) continue;
            }
            int m[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int u = bc[a] + o[a];
                m[a] = cg.periodic[a] ? (u < 0 ? -1 : (u >= cg.nb[a] ? 1 : 0)) : 0;
            }
            const int hb = halo_index(bc[0] - 2 * B[0] + 1 + o[0], bc[1] - 2 * B[1] + 1 + o[1],
                                      bc[2] - 2 * B[2] + 1 + o[2]);
            const double sx = m[0] * cg.h[0] + m[1] * cg.h[3] + m[2] * cg.h[6];
            const double sy = m[0] * cg.h[1] + m[1] * cg.h[4] + m[2] * cg.h[7];
            const double sz = m[0] * cg.h[2] + m[1] * cg.h[5] + m[2] * cg.h[8];
            const bool self_image = (m[0] | m[1] | m[2]) == 0;
            const uint32_t code = lb.entry_code(q, m);
            const int r0 = s_off[hb], r1 = s_off[hb + 1], u0 = s_gst[hb] - r0;
            // (two loops, so that the LDS one issues no memory loads)
            if (staged) {
                for (int r = r0; r < r1; ++r) {
                    const int u = u0 + r;
                    if (u == t && self_image) continue;
                    lb.offer(u, pos[r], sx, sy, sz, code);
                }
            } else {
                for (int r = r0; r < r1; ++r) {
                    const int u = u0 + r;
                    if (u == t && self_image) continue;
                    lb.offer(u, xq[u], sx, sy, sz, code);
                }
            }
        }
        lb.finish(ncnt);
    }
}

// Reverse index of the angular lists: for entry (t, slot) naming atom j with
// image n, the slot of j's list that names t with image -n (255 if absent,
// which symmetric lists never produce).  sorted_scan: the lists of binned
// cells were built in storage order (as k_build_lists with that flag).
__global__ __launch_bounds__(256) void k_build_reverse(PairConsts pc, const int32_t *__restrict__ cell_of,
                                                       const CellGeom *__restrict__ cells,
                                                       const int32_t *__restrict__ nl_ang,
                                                       const uint32_t *__restrict__ ncnt,
                                                       uint8_t *__restrict__ rev, int32_t *__restrict__ status,
                                                       const int32_t *__restrict__ flag, int sorted_scan)
{
    if (flag && *flag == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pc.n) return;
    if (status[ST_ERR] != 0) return;
    const CellGeom &cg = cells[cell_of[t]];
    const int base = cg.atom_start;
    const bool sorted = sorted_scan && cg.R[0] == 0 && cg.R[1] == 0 && cg.R[2] == 0;
    const uint32_t cnt = ncnt[t];
    const int naf = cnt & 0xff, nab = (cnt >> 8) & 0xff;
    const uint32_t jmask = (1u << pc.jbits) - 1u, imask = (1u << pc.ibits) - 1u;
    const uint32_t tl = (uint32_t)(t - base);
    for (int s = 0; s < naf + nab; ++s) {
        const int slot = s < naf ? s : s + (pc.capA - naf - nab);
        const uint32_t e = (uint32_t)nl_ang[(size_t)slot * pc.n + t];
        const int j = (int)(e & jmask) + base;
        const uint32_t code = e >> pc.jbits;
        uint32_t want;
        if (pc.delta) {
            // the partner's bin offset is the negated one (q -> 26 - q), the
            // same faces crossed
            want = tl | (((26u - (code & 31u)) | (code & ~31u)) << pc.jbits);
        } else {
            const int n0 = (int)(code & imask) - pc.ioff, n1 = (int)((code >> pc.ibits) & imask) - pc.ioff,
                      n2 = (int)(code >> (2 * pc.ibits)) - pc.ioff;
            want = tl | (((uint32_t)(-n0 + pc.ioff) | ((uint32_t)(-n1 + pc.ioff) << pc.ibits) |
                          ((uint32_t)(-n2 + pc.ioff) << (2 * pc.ibits))) << pc.jbits);
        }
        const uint32_t cj = ncnt[j];
        const int jf = cj & 0xff, jb = (cj >> 8) & 0xff;
        // both ends classify the pair from the same r^2 (exactly negated FP64
        // pair vectors), so a front entry's partner is in j's front part and
        // a back entry's in j's back part; the other part is searched only if
        // that fails (after a capacity overflow, for instance)
        const int f0 = 0, f1 = jf, b0 = pc.capA - jb, b1 = pc.capA;
        const bool front = s < naf;
        int found = 255;
        if (sorted) {
            // a list built in storage order holds each neighbour once per
            // part, ascending in its index (the front part in slot order, the
            // back part in reverse slot order): bisect on the index field
            const int q0 = front ? f0 : b0, q1 = front ? f1 : b1;
            int lo = 0, hi = q1 - q0;        // rank in ascending index order
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int sq = front ? q0 + mid : q1 - 1 - mid;
                if (((uint32_t)nl_ang[(size_t)sq * pc.n + j] & jmask) < tl) lo = mid + 1;
                else hi = mid;
            }
            const int sq = front ? q0 + lo : q1 - 1 - lo;
            if (lo < q1 - q0 && (uint32_t)nl_ang[(size_t)sq * pc.n + j] == want) found = sq;
        }
        for (int pass = 0; pass < 2 && found == 255; ++pass) {
            const bool in_front = (pass == 0) == front;
            const int q0 = in_front ? f0 : b0, q1 = in_front ? f1 : b1;
            for (int sq = q0; sq < q1; ++sq)
                if ((uint32_t)nl_ang[(size_t)sq * pc.n + j] == want) { found = sq; break; }
        }
        rev[(size_t)slot * pc.n + t] = (uint8_t)found;
    }
}

// ------------------------------------------------------------------ velocity Verlet

// Block maximum of a non-negative double, one atomicMax per block on its
// bit pattern (non-negative doubles order like their unsigned bit patterns).
__device__ inline void block_max_atomic(double v, double *dst)
{
    __shared__ double sh[4];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
        atomicMax(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)__double_as_longlong(m));
    }
}

// Block sum of a double in a fixed order (waves by shuffles, then the four
// wave sums in order); thread 0 stores it to dst.  Blocks of 256 threads.
__device__ inline void block_sum_store(double v, double *dst)
{
    __shared__ double sh[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        *dst = t;
    }
}

// v += dt/2 F/m ; x += dt v ; track the largest displacement since the last
// build.  With a border set, the velocities of border atoms are first scaled
// by md[MD_SCALE] (the thermostat's factors since the last kick).
// Grid-stride loop over atoms (blocks of 256 threads).
__global__ __launch_bounds__(256) void k_kick_drift(int n, double *__restrict__ x, double *__restrict__ y,
                                                    double *__restrict__ z, double *__restrict__ vx,
                                                    double *__restrict__ vy, double *__restrict__ vz,
                                                    const float *__restrict__ fx, const float *__restrict__ fy,
                                                    const float *__restrict__ fz, double acc_per_mass,
                                                    const double *__restrict__ xref, const uint8_t *__restrict__ border,
                                                    double *__restrict__ md, int32_t *__restrict__ status)
{
    double dmax = 0.0, smax = 0.0;
    if (status[ST_ERR] == 0) {
        const double dt = md[MD_DT];
        const double c = 0.5 * dt * acc_per_mass;
        const double scale = border ? md[MD_SCALE] : 1.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            double u0 = vx[i], u1 = vy[i], u2 = vz[i];
            if (border && border[i]) { u0 *= scale; u1 *= scale; u2 *= scale; }
            const double v0 = u0 + c * fx[i], v1 = u1 + c * fy[i], v2 = u2 + c * fz[i];
            vx[i] = v0; vy[i] = v1; vz[i] = v2;
            const double p0 = x[i] + dt * v0, p1 = y[i] + dt * v1, p2 = z[i] + dt * v2;
            x[i] = p0; y[i] = p1; z[i] = p2;
            const double e0 = p0 - xref[i], e1 = p1 - xref[(size_t)n + i], e2 = p2 - xref[2 * (size_t)n + i];
            double d2 = e0 * e0 + e1 * e1 + e2 * e2;
            if (!isfinite(d2)) { latch_error(status, -5); d2 = 0.0; }
            dmax = fmax(dmax, d2);
            const double s2 = dt * dt * (v0 * v0 + v1 * v1 + v2 * v2);
            if (isfinite(s2)) smax = fmax(smax, s2);
        }
    }
    block_max_atomic(dmax, md + MD_DISP2);
    __syncthreads();
    block_max_atomic(smax, md + MD_STEP2);
}

// The radial walk's candidate bound after a drift: the largest step of this
// drift is added to the bound on any atom's displacement since the last full
// radial walk; the next evaluation walks in full (and restarts the bound)
// after a rebuild or once the bound reaches half the candidate margin.
__global__ void k_cand_update(double half_margin, double *__restrict__ md, const int32_t *__restrict__ rebuilt,
                              int32_t *__restrict__ cflag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = md[MD_CACC] + sqrt(md[MD_STEP2]);
    md[MD_STEP2] = 0.0;
    const int full = *rebuilt != 0 || !(acc < half_margin);
    if (full) acc = 0.0;
    md[MD_CACC] = acc;
    *cflag = full;
}

// The bound's start value: 0 right after a full radial walk, huge when the
// candidate mask is not known to match the positions.
__global__ void k_cand_set(double *__restrict__ md, double acc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    md[MD_CACC] = acc;
    md[MD_STEP2] = 0.0;
}

// Largest |v|^2 (of the non-border atoms when a border set is given; then
// also the border maximum and the border sum of |v|^2, for the thermostat).
struct VelStats {
    double vmax = 0.0, vmax_b = 0.0, sum_b = 0.0;
    __device__ void add(double v2, bool b)
    {
        if (b) { vmax_b = fmax(vmax_b, v2); sum_b += v2; }
        else vmax = fmax(vmax, v2);
    }
    // block results: maxima into md, the border sum into ke_part[blockIdx.x]
    __device__ void store(bool has_border, double *__restrict__ ke_part, double *__restrict__ md) const
    {
        block_max_atomic(vmax, md + MD_VMAX2);
        if (has_border) {
            __syncthreads();
            block_max_atomic(vmax_b, md + MD_VMAX2B);
            __syncthreads();
            block_sum_store(sum_b, ke_part + blockIdx.x);
        }
    }
};

// v += dt/2 F/m ; track max |v|^2 for the next step length.
__global__ __launch_bounds__(256) void k_kick(int n, double *__restrict__ vx, double *__restrict__ vy,
                                              double *__restrict__ vz, const float *__restrict__ fx,
                                              const float *__restrict__ fy, const float *__restrict__ fz,
                                              double acc_per_mass, const uint8_t *__restrict__ border,
                                              double *__restrict__ ke_part, double *__restrict__ md,
                                              const int32_t *__restrict__ status)
{
    VelStats vs;
    if (status[ST_ERR] == 0) {
        const double c = 0.5 * md[MD_DT] * acc_per_mass;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const double v0 = vx[i] + c * fx[i], v1 = vy[i] + c * fy[i], v2 = vz[i] + c * fz[i];
            vx[i] = v0; vy[i] = v1; vz[i] = v2;
            vs.add(v0 * v0 + v1 * v1 + v2 * v2, border && border[i]);
        }
    }
    vs.store(border != nullptr, ke_part, md);
}

// max |v|^2 of the current velocities (and the border statistics).
__global__ __launch_bounds__(256) void k_vmax(int n, const double *__restrict__ vx, const double *__restrict__ vy,
                                              const double *__restrict__ vz, const uint8_t *__restrict__ border,
                                              double *__restrict__ ke_part, double *__restrict__ md)
{
    VelStats vs;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        vs.add(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i], border && border[i]);
    vs.store(border != nullptr, ke_part, md);
}

// Step length for the next step: dt = min(dt_max, max_disp / max|v|) (Sec. II.B).
__global__ void k_dt_update(double dt_max, double max_disp, double dt_min, double *__restrict__ md,
                            int32_t *__restrict__ status, int advance_time)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (advance_time) md[MD_TIME] += md[MD_DT];
    const double vmax = sqrt(md[MD_VMAX2]);
    double dt = dt_max;
    if (max_disp > 0.0 && vmax > 0.0) dt = fmin(dt_max, max_disp / vmax);
    if (!(dt >= dt_min)) latch_error(status, -6);
    md[MD_DT] = dt;
    md[MD_VMAX2] = 0.0;
    md[MD_VMAX2B] = 0.0;
}

// Rebuild decision: an atom moved more than skin/2 since the last build.
__global__ void k_rebuild_flag(double half_skin2, double *__restrict__ md, int32_t *__restrict__ flag,
                               const int32_t *__restrict__ status)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    // unusable lists (a build that ended with an error) are rebuilt too
    const int r = md[MD_DISP2] > half_skin2 || status[ST_LBAD] != 0;
    *flag = r;
    if (r) md[MD_NREB] += 1.0;
    md[MD_DISP2] = 0.0;
}

// End of a list build: the lists are usable if no error was latched while
// they were built (an overflow truncates them and skips the reverse index).
// Skipped with the rest of the build when *flag is 0.
__global__ void k_lists_commit(int32_t *__restrict__ status, const int32_t *__restrict__ flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (flag && *flag == 0) return;
    status[ST_LBAD] = status[ST_ERR] != 0 ? 1 : 0;
}

// Largest displacement since the last build (for the rebuild decision at a
// chunk start, when positions may have been changed by the caller).
__global__ __launch_bounds__(256) void k_disp(int n, const double *__restrict__ x, const double *__restrict__ y,
                                              const double *__restrict__ z, const double *__restrict__ xref,
                                              double *__restrict__ md)
{
    double dmax = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double e0 = x[i] - xref[i], e1 = y[i] - xref[(size_t)n + i], e2 = z[i] - xref[2 * (size_t)n + i];
        double d2 = e0 * e0 + e1 * e1 + e2 * e2;
        if (!isfinite(d2)) d2 = 1e300;
        dmax = fmax(dmax, d2);
    }
    block_max_atomic(dmax, md + MD_DISP2);
}

__global__ void k_set_flag(int32_t *__restrict__ flag, int32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = v;
}

// Cell index of every atom from the cell offsets (binary search).
__global__ void k_cell_of(int n, int n_cells, const int64_t *__restrict__ cell_start,
                          int32_t *__restrict__ cell_of)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_cells;   // cell_start[lo] <= i < cell_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cell_start[mid] <= i) lo = mid;
        else hi = mid;
    }
    cell_of[i] = lo;
}

}  // namespace nep
