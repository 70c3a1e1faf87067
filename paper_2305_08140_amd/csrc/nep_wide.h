// The paper-size model (Sec. III.A: Chebyshev expansion orders n_max^R = 15
// and n_max^A = 10, l_max = 4, 100 hidden neurons; cutoffs as the default
// model): 16 radial functions on 16 Chebyshev terms, 11 angular functions on
// 11 terms, 60 descriptor components.  Its 11 x 24 angular sums do not fit
// one lane's registers, so the evaluation runs in phases with the sums and
// descriptors staged in HBM, [component][atom] (coalesced per wavefront):
//   k_w_radial    radial sums and descriptors, ZBL half energies
//   k_w_angular   angular sums of one group of WGA channels per launch
//                 (l <= 3 in FP64, l = 4 in FP32, as in the default model)
//   k_w_network   network forward and backward per atom, site energy, the
//                 atom's record (position + 16 radial adjoints, 96 bytes;
//                 80 with a fixed-point position in bin-offset mode)
//   k_w_grad      dU_i/dr_ij of every angular slot, channel group by group
//   k_w_force     radial + ZBL pair forces, angular assembly, virial
// and, for the parameter gradient, k_w_param_grad after the first three.
#pragma once
#include "nep_device.h"

namespace nep {

constexpr int WR = 16, WKR = 16;         // radial functions, radial Chebyshev terms
constexpr int WA = 11, WKA = 11;         // angular functions, angular Chebyshev terms
constexpr int WH = 100;                  // hidden neurons
constexpr int WDIM = WR + WA * LMAX;     // 60
constexpr int WGA = 4;                   // angular channels per launch of the angular sums
constexpr int WNGA = (WA + WGA - 1) / WGA;  // 3 launches (4, 4, 3)
// default threads per block (one atom per lane; nep_autotune may pick 64, 128
// or 256 for a system size): the descriptor phases in 64-thread blocks (a
// block retires with its slowest wave; 24.7 -> 24.3 ms at 8,192,000 atoms),
// the force kernel in 256-thread blocks (11.2 -> 10.7 ms)
constexpr int WBS = 64, WBS_F = 256;
constexpr int WN_BS = 256;               // threads per block of the matrix-core network
constexpr int WG = 3;                    // angular channels per group of the gradient walk
constexpr int WNG = (WA + WG - 1) / WG;  // 4 groups (3, 3, 3, 2)

// parameter block (floats): c_rad [WR][WKR], c_ang [WA][WKA], q_scale [WDIM],
// w0 [WH][WDIM], b0 [WH], w1 [WH], b1
constexpr int W_CR = 0;
constexpr int W_CA = W_CR + WR * WKR;
constexpr int W_QS = W_CA + WA * WKA;
constexpr int W_W0 = W_QS + WDIM;
constexpr int W_B0 = W_W0 + WH * WDIM;
constexpr int W_W1 = W_B0 + WH;
constexpr int W_B1 = W_W1 + WH;
constexpr int W_SIZE = W_B1 + 1;
// double copy of the angular coefficients and their row sums
constexpr int W_C64 = WA * WKA + WA;
// trainable parameters, in the order of the gradient: c_rad, c_ang, w0, b0, w1, b1
constexpr int W_NPARAM = WR * WKR + WA * WKA + WH * WDIM + WH + WH + 1;

// the force kernel's per-neighbour record: 88 bytes padded to 96, six
// 16-byte pieces per gather (a 128-byte stride would cost eight, and
// power-of-two strides gather more slowly)
struct __attribute__((aligned(16))) WAtomRec {
    double x, y, z;
    float a[WKR];
    float pad[2];
};
static_assert(sizeof(WAtomRec) == 96, "WAtomRec must be 96 bytes");

// bin-offset mode (one periodic cell binned along every axis): the position
// as fixed-point offsets from the corner of the atom's bin, 76 bytes padded
// to 80, five 16-byte pieces per gather
struct __attribute__((aligned(16))) WAtomRec80 {
    int32_t o[3];
    float a[WKR];
    float pad;
};
static_assert(sizeof(WAtomRec80) == 80, "WAtomRec80 must be 80 bytes");

__global__ void k_w_params64(const float *P, double *C64);
__global__ void k_w_pop_params(const float *theta, const float *base, float *P, double *C64);
template <int BS, bool D16>
__global__ void k_w_radial(PairConsts pc, const double4 *xq, const int4 *xf, const int32_t *cell_of,
                           const CellGeom *cells, const int32_t *nl_ang, const int32_t *nl_rad,
                           const uint32_t *ncnt, const float *P, float *Q, double *e_atom, int32_t *status,
                           const int32_t *cflag);
template <int BS, bool D16>
__global__ void k_w_angular(PairConsts pc, const double4 *xq, const int4 *xf, const int32_t *cell_of,
                            const CellGeom *cells, const int32_t *nl_ang, const uint32_t *ncnt, const double *C64,
                            int group, float *S, float *Q);
template <int BS>
__global__ void k_w_network(int n, const double4 *xq, const float *P, const float *Q, WAtomRec *xw, float *FpA,
                            double *e_atom, const CellGeom *cells, const int32_t *bin_sorted, double qsinv,
                            int32_t *status);
template <bool BF16>
__global__ void k_w_network_mfma(int n_atoms, int ntiles, const double4 *xq, const float *P, const float *Q,
                                 WAtomRec *xw, float *FpA, double *e_atom, const CellGeom *cells,
                                 const int32_t *bin_sorted, double qsinv, int32_t *status);
template <int BS, bool D16>
__global__ void k_w_grad(PairConsts pc, const double4 *xq, const int4 *xf, const int32_t *cell_of,
                         const CellGeom *cells, const int32_t *nl_ang, const uint32_t *ncnt, const float *P,
                         const double *C64, const float *S, const float *FpA, float4 *pair_grad, float4 *f_own,
                         float *w_atom);
template <int BS, bool D80>
__global__ void k_w_force(PairConsts pc, const WAtomRec *xw, const int32_t *cell_of, const CellGeom *cells,
                          const int32_t *nl_ang, const int32_t *nl_rad, const uint32_t *ncnt, const uint8_t *rev,
                          const float4 *pair_grad, const float4 *f_own, const int32_t *perm, float *fx, float *fy,
                          float *fz, float *w_atom, int32_t *status);
__global__ void k_w_param_grad(PairConsts pc, const double4 *xq, const int32_t *cell_of, const CellGeom *cells,
                               const int32_t *nl_ang, const int32_t *nl_rad, const uint32_t *ncnt, const float *P,
                               const float *Q, const float *S, const float *FpA, const double *gE, double *part,
                               int32_t *status, int ntiles);

}  // namespace nep
