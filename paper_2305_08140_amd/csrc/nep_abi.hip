// Host side of the C ABI declared in include/nep.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "nep.h"
#include "nep_device.h"
#include "nep_wide.h"

namespace nep {
// kernels (nep_kernels.hip)
template <int BS, bool PE, int NNMODE>
__global__ void k_descriptor(PairConsts, const double4 *, AtomRec *, const int32_t *, const CellGeom *, const int32_t *,
                             const int32_t *, const uint32_t *, const float *, const double *, float4 *, float4 *,
                             float *, double *, int32_t *, int, const int32_t *, const int32_t *);
template <int BS, bool PE, bool D48>
__global__ void k_force(PairConsts, const AtomRec *, const int32_t *, const CellGeom *, const int32_t *,
                        const int32_t *, const uint32_t *, const uint8_t *, const float4 *, const float4 *,
                        const int32_t *, float *, float *, float *, float *, int32_t *, int);
__global__ void k_reduce_chunks(const int32_t *, const int32_t *, const double *, const float *, double *,
                                const int32_t *);
__global__ void k_reduce_cells(int, const int32_t *, const double *, double *, double *, const int32_t *);
__global__ void k_energy_atom_out(int, const int32_t *, const double *, float *);
__global__ void k_param_grad(PairConsts, const double4 *, const int32_t *, const CellGeom *, const int32_t *,
                             const int32_t *, const uint32_t *, const float *, const double *, const double *,
                             double *, int32_t *, int);
__global__ void k_params64(const float *, double *);
__global__ void k_param_reduce(int, int, const double *, double *);
__global__ void k_grad_pos(int, const int32_t *, const double *, const float *, const float *, const float *,
                           double *, double *, double *);
__global__ void k_grad_cell(const CellGeom *, const double *, const double *, const double *, const float *,
                            const float *, const float *, const double *, const double *, double *);
__global__ void k_count_inside(PairConsts, const double4 *, const int32_t *,
                               const CellGeom *, const int32_t *, const int32_t *, const uint32_t *,
                               unsigned long long *);
__global__ void k_pop_params(const float *, const float *, float *, double *);
__global__ void k_pop_descriptor(PairConsts, const double4 *, AtomRec *, const int32_t *, const CellGeom *,
                                 const int32_t *, const int32_t *, const uint32_t *, const float *, const double *,
                                 float4 *, float4 *, float *, double *, int32_t *, int, int);
__global__ void k_pop_force(PairConsts, const AtomRec *, const int32_t *, const CellGeom *, const int32_t *,
                            const int32_t *, const uint32_t *, const uint8_t *, const float4 *, const float4 *,
                            const int32_t *, float *, float *, int32_t *, int, int);
__global__ void k_pop_reduce_chunks(int, int, const int32_t *, const int32_t *, const double *, const float *,
                                    double *, const int32_t *);
__global__ void k_pop_reduce_cells(int, int, const int32_t *, const double *, double *, double *,
                                   const int32_t *);
__global__ void k_pop_force_err(int, const float *, const float *, const float *, const float *, double *);
__global__ void k_pop_loss(int, int, int, int, const int64_t *, const double *, const double *, const double *,
                           const double *, const uint8_t *, const double *, const float *, double, double, double,
                           double, double, double *);
__global__ void k_snes_sample(int, int, const float *, const float *, const float *, float *);
__global__ void k_snes_update(int, int, const double *, int, const float *, float *, float *, double, double);
// kernels (nep_defects.hip)
__global__ void k_ws_fill(int, int32_t *, int32_t);
__global__ void k_ws_assign(int, const double *, const double *, const double *, BccRef, int32_t *, int32_t *,
                            int32_t *);
__global__ void k_ws_collect(int, const int32_t *, int, int32_t *, int32_t *, int32_t *);
__global__ void k_ws_sort(int, const int32_t *, int32_t *, const int32_t *, int32_t *);
__global__ void k_ws_label_init(int, int32_t *);
__global__ void k_ws_label_step(int, const int32_t *, double, BccRef, int32_t *, int32_t *);
__global__ void k_ws_cluster_sizes(int, const int32_t *, const int32_t *, int32_t *);
// kernels (nep_build.hip)
__global__ void k_fill_i32(int, int32_t *, int32_t, const int32_t *);
__global__ void k_bin_assign(int, const double *, const double *, const double *, const int32_t *,
                             const CellGeom *, int32_t *, int32_t *, int32_t *, double *, const int32_t *,
                             int32_t *, const int32_t *);
__global__ void k_scan_blocks(int, const int32_t *, int32_t *, int32_t *, const int32_t *);
__global__ void k_scan_sums(int, int32_t *, const int32_t *);
__global__ void k_scan_add(int, int32_t *, const int32_t *, const int32_t *);
__global__ void k_bin_scatter(int, const int32_t *, const int32_t *, int32_t *, int32_t *, const int32_t *);
__global__ void k_bin_rank(int, const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                           const CellGeom *, int32_t *, int32_t *, const int32_t *, const int32_t *);
__global__ void k_sort_positions(int, const int32_t *, const double *, const double *, const double *,
                                 const int32_t *, const int32_t *, const CellGeom *, double4 *, int32_t *,
                                 const int32_t *, const int32_t *, double, int4 *);
__global__ void k_build_lists(PairConsts, double, double, double, double, const double4 *, const int32_t *,
                              const CellGeom *, const int32_t *, const int32_t *, const int32_t *, int32_t *,
                              int32_t *, uint32_t *, int32_t *, const int32_t *, int);
__global__ void k_build_reverse(PairConsts, const int32_t *, const CellGeom *, const int32_t *,
                                const uint32_t *, uint8_t *, int32_t *, const int32_t *, int);
__global__ void k_build_lists_blocks(PairConsts, double, double, double, double, const double4 *, const CellGeom *,
                                     const int32_t *, const int32_t *, const int32_t *, const uint32_t *, int,
                                     int32_t *, int32_t *, uint32_t *, int32_t *, const int32_t *);
__global__ void k_kick_drift(int, double *, double *, double *, double *, double *, double *, const float *,
                             const float *, const float *, double, const double *, const uint8_t *, double *,
                             int32_t *);
__global__ void k_kick(int, double *, double *, double *, const float *, const float *, const float *, double,
                       const uint8_t *, double *, double *, const int32_t *);
__global__ void k_vmax(int, const double *, const double *, const double *, const uint8_t *, double *, double *);
__global__ void k_dt_update(double, double, double, double *, int32_t *, int);
__global__ void k_rebuild_flag(double, double *, int32_t *, const int32_t *);
__global__ void k_lists_commit(int32_t *, const int32_t *);
__global__ void k_disp(int, const double *, const double *, const double *, const double *, double *);
__global__ void k_set_flag(int32_t *, int32_t);
__global__ void k_cand_update(double, double *, const int32_t *, int32_t *);
__global__ void k_cand_set(double *, double);
__global__ void k_cell_of(int, int, const int64_t *, int32_t *);
// kernels (nep_thermostat.hip)
__global__ void k_border_mask(int, const double *, const double *, const double *, double, double, double, int,
                              double, uint8_t *, int32_t *);
__global__ void k_scale_border(int, double *, double *, double *, const uint8_t *, const double *);
__global__ void k_nhc(const double *, int, double, int, double, double, double, double, double, const int32_t *,
                      double *, int32_t *, int);
}  // namespace nep

using namespace nep;

// (eV / u) -> (A / fs)^2, i.e. an acceleration F/m in eV/(u A) to A/fs^2
// (e = 1.602176634e-19 C, u = 1.66053906660e-27 kg).
static const double ACC_EV_U_A = 9.6485332156653280e-3;
// Boltzmann constant, eV/K (CODATA 2018)
static const double K_B_EV = 8.617333262e-5;

#define HIP_TRY(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return NEP_E_HIP;     \
    } while (0)

// Launch shapes used until the autotuner has run for a size bucket: 64-thread
// tiles for the descriptor (a block retires with its slowest wave, and the
// per-atom neighbour counts vary; 9.37 -> 9.03 ms at 8,192,000 atoms against
// 256-thread tiles), 256-thread tiles for the force kernel.
static const int DEFAULT_SHAPE_DESC = 0, DEFAULT_SHAPE_FORCE = 2;

struct nep_ctx {
    nep_hparams hp;
    nep_config cfg;
    int device = 0;
    float *params = nullptr;
    // per-atom storage (capacity cfg.max_atoms)
    AtomRec *xp = nullptr;       // [N] sorted wrapped positions and radial adjoints
    double4 *xq = nullptr;       // [N] sorted wrapped positions, compact copy
    double *c64 = nullptr;       // angular coefficients and their row sums, double precision
    // the paper-size model (nep_wide.h): staged sums, descriptors, adjoints, records
    bool wide = false;
    float *w_S = nullptr, *w_Q = nullptr, *w_FpA = nullptr;
    WAtomRec *xw = nullptr;
    int4 *xf = nullptr;          // bin-offset mode: fixed-point positions for the radial phase
    double *xref = nullptr;      // [3][N] caller-order positions at the last build
    int32_t *perm = nullptr, *bin_of = nullptr, *wrap = nullptr, *cell_of = nullptr, *tmp = nullptr,
            *bin_sorted = nullptr;
    uint32_t *ncnt = nullptr;
    int32_t *nl_ang = nullptr, *nl_rad = nullptr;
    float *w_atom = nullptr;
    float4 *pair_grad = nullptr;  // [capA][N] dU_i/dr_ij of every angular list slot
    float4 *f_own = nullptr;      // [N] sum_j dU_i/dr_ij (angular)
    uint8_t *rev = nullptr;       // [capA][N] reverse slot index
    uint32_t *rmask = nullptr;    // [ceil(capR/32)][N] radial entries inside rc_rad
    uint32_t *amask = nullptr;    // [ceil(capA/32)][N] angular entries within the write radius
    uint32_t *cmask = nullptr;    // [ceil(capR/32)][N] radial entries within the candidate radius
    int32_t *cflag = nullptr;     // next evaluation's radial walk: 1 full, 0 candidates only
    double *e_atom = nullptr;
    // per-cell storage
    CellGeom *cells = nullptr;
    int64_t *cell_start_d = nullptr;
    int32_t *chunk_begin = nullptr, *chunk_end = nullptr, *cell_chunk = nullptr;
    double *part = nullptr;
    int n_chunks = 0, chunk_cap = 0;
    // bins
    int32_t *bin_count = nullptr, *bin_start = nullptr, *bin_fill = nullptr, *scan_sums = nullptr;
    int32_t *bin_rank = nullptr, *bin_lin = nullptr;   // Morton order of the bins of every cell
    int64_t bin_cap = 0;
    int n_bins = 0;
    // status and md state
    int32_t *status = nullptr;       // [8]
    int32_t *flag = nullptr;         // rebuild flag
    double *md = nullptr;            // [MD_WORDS]
    // border thermostat: one byte per atom, block partials of the border
    // |v|^2, the border count, and what the set was selected with
    uint8_t *border = nullptr;
    double *ke_part = nullptr;       // [MAX_STREAM_BLOCKS]
    int32_t *n_border = nullptr;
    bool border_valid = false;
    int th_chain = 0, th_axes = 0;
    double th_border = 0.0;
    // population evaluation (SNES): per-member parameters and evaluation
    // buffers for up to pop_cap members at the context's capacity
    int pop_cap = 0;
    int64_t pop_chunk_cap = 0;
    float *pop_P = nullptr;
    double *pop_c64 = nullptr;
    AtomRec *pop_xp = nullptr;
    float4 *pop_pg = nullptr, *pop_fown = nullptr;
    float *pop_w = nullptr, *pop_F = nullptr;
    double *pop_e = nullptr, *pop_E = nullptr, *pop_W = nullptr, *pop_part = nullptr, *pop_fpart = nullptr;
    unsigned long long *counts = nullptr;
    double *pg_part = nullptr;       // parameter-gradient block partials
    int pg_blocks = 0;
    // list build by bin blocks (one binned cell): the blocks in Morton order
    // of their coordinates (packed), 0 when the system is not eligible
    int lb_blocks = 0;
    int64_t lb_cap = 0;
    uint32_t *blk_coord = nullptr;
    // launch shapes of the two evaluation kernels (index into SHAPES), per
    // size bucket floor(log2 n_atoms) once the autotuner has run
    int shape_desc = DEFAULT_SHAPE_DESC, shape_force = DEFAULT_SHAPE_FORCE;
    int nn_mode = 0;                 // hidden layer: 0 FP32 vector ALU, 1 BF16 / 2 FP32 matrix cores
    int tuned_desc[32], tuned_force[32];
    // captured evaluation graph and the arguments it was captured with
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uintptr_t> graph_key;
    int32_t *h_status = nullptr;     // pinned
    double *h_md = nullptr;          // pinned
    unsigned long long *h_counts = nullptr;
    // state of the last build
    bool built = false;
    int64_t built_n = -1;
    int built_cells = -1;
    std::vector<double> built_h;
    std::vector<int64_t> built_start;
    int pbc[3] = {1, 1, 1};
    PairConsts pc;
    // incremented by every setup_system: the captured graph holds the pair
    // constants and per-cell tables of the setup it was captured under
    uint64_t setup_gen = 0;
    std::vector<CellGeom> geom;
};

static int grid_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }
// the fixed-point positions the position refresh writes for the paper-size
// model's walks in bin-offset mode (none otherwise)
static int4 *wide_xf(const nep_ctx *c) { return c->wide && c->pc.delta ? c->xf : nullptr; }


static int bucket_of(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n && b < 31) ++b;
    return b;
}

static int xcd_grid(int tiles) { return 8 * ((tiles + 7) / 8); }
// grid of the streaming (grid-stride) kernels: enough blocks to fill the chip
static const int MAX_STREAM_BLOCKS = 2048;
static int stream_grid(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, MAX_STREAM_BLOCKS); }

static void inv3(const double *h, double *hi)
{
    const double a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], k = h[7], l = h[8];
    const double det = a * (e * l - f * k) - b * (d * l - f * g) + c * (d * k - e * g);
    hi[0] = (e * l - f * k) / det; hi[1] = (c * k - b * l) / det; hi[2] = (b * f - c * e) / det;
    hi[3] = (f * g - d * l) / det; hi[4] = (a * l - c * g) / det; hi[5] = (c * d - a * f) / det;
    hi[6] = (d * k - e * g) / det; hi[7] = (b * g - a * k) / det; hi[8] = (a * e - b * d) / det;
}

static constexpr int N_PARAMS = NR * KB + NA * KB + NH * DIM + NH + NH + 1;

// Allocation-free backward: the parameter-gradient block partials live in a
// file-scope device array instead of the context.  It holds the partials of
// the widest launch the backward makes (PG_MAX_BLOCKS rows of the larger
// model's parameter count, W_NPARAM doubles: 53.9 MB), so every system a
// context of either model accepts fits, with the same rows as nep_backward.
// Each device keeps its own copy until the process ends; host code reaches
// it only through the address resolved per device below, never through the
// name.
static constexpr int PG_MAX_BLOCKS = 1024;
static constexpr int PG_MAX_PARAMS = N_PARAMS > W_NPARAM ? N_PARAMS : W_NPARAM;
static __device__ __align__(256) double scratch[(size_t)PG_MAX_BLOCKS * PG_MAX_PARAMS];
static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The scratch address on `dev`, resolved once per device; the first call for
// a device must run with that device current (nep_create does it).
static int scratch_address(int dev, double **p)
{
    *p = nullptr;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return NEP_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return NEP_E_HIP;
        if (cur != dev) return NEP_E_ARG;
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return NEP_E_HIP;
        g_scratch_ptr[dev] = (double *)q;
    }
    *p = g_scratch_ptr[dev];
    return NEP_OK;
}

extern "C" {

const char *nep_strerror(int code)
{
    switch (code) {
    case NEP_OK: return "ok";
    case NEP_E_ARG: return "invalid argument";
    case NEP_E_HIP: return "HIP runtime error";
    case NEP_E_NEIGH_OVERFLOW: return "neighbour list capacity exceeded";
    case NEP_E_OVERLAP: return "overlapping atoms (distance below 1e-3 A)";
    case NEP_E_NONFINITE: return "non-finite position or velocity";
    case NEP_E_DT_UNDERFLOW: return "adaptive time step below dt_min";
    case NEP_E_STATE: return "neighbour lists not built for this system";
    case NEP_E_UNSUPPORTED: return "hyperparameters not supported by the compiled kernels";
    case NEP_E_INTERNAL: return "internal consistency check failed (asymmetric neighbour lists)";
    case NEP_E_CAPACITY: return "more defect sites than the arrays hold";
    default: return "unknown error";
    }
}

static void free_population(nep_ctx *c)
{
    void *bufs[] = {c->pop_P, c->pop_c64, c->pop_xp, c->pop_pg, c->pop_fown, c->pop_w, c->pop_F,
                    c->pop_e, c->pop_E, c->pop_W, c->pop_part, c->pop_fpart};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    c->pop_P = nullptr; c->pop_c64 = nullptr; c->pop_xp = nullptr; c->pop_pg = c->pop_fown = nullptr;
    c->pop_w = c->pop_F = nullptr;
    c->pop_e = c->pop_E = c->pop_W = c->pop_part = c->pop_fpart = nullptr;
    c->pop_cap = 0;
}

void nep_destroy(nep_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_population(c);
    void *bufs[] = {c->params, c->c64, c->w_S, c->w_Q, c->w_FpA, c->xw, c->xf, c->xp, c->xq, c->xref, c->bin_rank, c->bin_lin, c->perm, c->bin_of, c->wrap, c->cell_of, c->tmp,
                    c->bin_sorted, c->ncnt, c->nl_ang, c->nl_rad, c->pair_grad, c->f_own, c->rev,
                    c->w_atom,
                    c->e_atom, c->cells, c->cell_start_d, c->chunk_begin, c->chunk_end, c->cell_chunk,
                    c->part, c->bin_count, c->bin_start, c->bin_fill, c->scan_sums, c->status, c->flag,
                    c->md, c->counts, c->pg_part, c->border, c->ke_part, c->n_border, c->rmask, c->amask, c->cmask, c->cflag,
                    c->blk_coord};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->h_md) (void)hipHostFree(c->h_md);
    if (c->h_counts) (void)hipHostFree(c->h_counts);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    delete c;
}

int nep_create(const nep_hparams *hp, const nep_config *cfg, nep_ctx **out)
{
    if (!out) return NEP_E_ARG;
    *out = nullptr;
    if (!hp || !cfg) return NEP_E_ARG;
    const bool small = hp->n_rad == NR && hp->n_ang == NA && hp->k_rad == KB && hp->k_ang == KB &&
                       hp->l_max == LMAX && hp->n_hidden == NH;
    const bool wide = hp->n_rad == WR && hp->n_ang == WA && hp->k_rad == WKR && hp->k_ang == WKA &&
                      hp->l_max == LMAX && hp->n_hidden == WH;
    if (!small && !wide) return NEP_E_UNSUPPORTED;
    if (!(hp->rc_rad > 0 && hp->rc_ang > 0 && hp->rc_ang <= hp->rc_rad && hp->zbl_r1 >= 0 &&
          hp->zbl_r2 > hp->zbl_r1 && hp->zbl_r2 <= hp->rc_ang && hp->Z > 0))
        return NEP_E_ARG;
    if (cfg->max_atoms <= 0 || cfg->max_atoms > (1LL << 26) || cfg->max_cells <= 0 ||
        cfg->max_neigh_ang <= 0 || cfg->max_neigh_ang > 255 || cfg->max_neigh_rad <= 0 ||
        cfg->max_neigh_rad > 255 || !(cfg->skin >= 0.0))
        return NEP_E_ARG;
    nep_ctx *c = new nep_ctx();
    for (int k = 0; k < 32; ++k) c->tuned_desc[k] = c->tuned_force[k] = -1;
    c->hp = *hp;
    c->cfg = *cfg;
    c->wide = wide;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return NEP_E_HIP; }
    {
        // the allocation-free backward's scratch address on this device
        double *sp = nullptr;
        const int src = scratch_address(c->device, &sp);
        if (src != NEP_OK) { delete c; return src; }
    }
    const size_t N = (size_t)cfg->max_atoms;
    bool ok = true;
    auto A = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes > 0 ? bytes : 16) != hipSuccess) ok = false;
    };
    const size_t p_size = wide ? W_SIZE : P_SIZE;
    A((void **)&c->params, p_size * sizeof(float));
    A((void **)&c->c64, (wide ? W_C64 : NA * KB + NA) * sizeof(double));
    if (wide) {
        A((void **)&c->xw, N * sizeof(WAtomRec));
        A((void **)&c->xf, N * sizeof(int4));
        A((void **)&c->w_S, N * WA * NLM * sizeof(float));
        A((void **)&c->w_Q, N * WDIM * sizeof(float));
        A((void **)&c->w_FpA, N * WA * LMAX * sizeof(float));
    }
    A((void **)&c->xp, N * sizeof(AtomRec));
    A((void **)&c->xq, N * sizeof(double4));
    A((void **)&c->xref, 3 * N * sizeof(double));
    A((void **)&c->perm, N * 4);
    A((void **)&c->bin_of, N * 4);
    A((void **)&c->wrap, N * 4);
    A((void **)&c->cell_of, N * 4);
    A((void **)&c->tmp, N * 4);
    A((void **)&c->bin_sorted, N * 4);
    A((void **)&c->ncnt, N * 4);
    A((void **)&c->nl_ang, N * cfg->max_neigh_ang * 4);
    A((void **)&c->nl_rad, N * cfg->max_neigh_rad * 4);
    A((void **)&c->pair_grad, N * cfg->max_neigh_ang * sizeof(float4));
    A((void **)&c->f_own, N * sizeof(float4));
    A((void **)&c->rev, N * cfg->max_neigh_ang);
    A((void **)&c->rmask, N * ((cfg->max_neigh_rad + 31) / 32) * 4);
    A((void **)&c->cmask, N * ((cfg->max_neigh_rad + 31) / 32) * 4);
    A((void **)&c->cflag, 4);
    A((void **)&c->amask, N * ((cfg->max_neigh_ang + 31) / 32) * 4);
    A((void **)&c->w_atom, N * 9 * 4);
    A((void **)&c->e_atom, N * 8);
    A((void **)&c->cells, (size_t)cfg->max_cells * sizeof(CellGeom));
    A((void **)&c->cell_start_d, ((size_t)cfg->max_cells + 1) * 8);
    A((void **)&c->status, 8 * 4);
    A((void **)&c->flag, 4);
    A((void **)&c->md, MD_WORDS * 8);
    A((void **)&c->border, N);
    A((void **)&c->ke_part, MAX_STREAM_BLOCKS * 8);
    A((void **)&c->n_border, 4);
    A((void **)&c->counts, 2 * 8);
    if (ok && hipHostMalloc((void **)&c->h_status, 8 * 4, hipHostMallocDefault) != hipSuccess) ok = false;
    if (ok && hipHostMalloc((void **)&c->h_md, MD_WORDS * 8, hipHostMallocDefault) != hipSuccess) ok = false;
    if (ok && hipHostMalloc((void **)&c->h_counts, 2 * 8, hipHostMallocDefault) != hipSuccess) ok = false;
    if (ok && hipMemset(c->status, 0, 8 * 4) != hipSuccess) ok = false;
    if (ok && hipMemset(c->md, 0, MD_WORDS * 8) != hipSuccess) ok = false;
    if (ok && hipMemset(c->params, 0, p_size * sizeof(float)) != hipSuccess) ok = false;
    // index arrays start in range, so that no kernel can ever see garbage indices
    if (ok && hipMemset(c->perm, 0, N * 4) != hipSuccess) ok = false;
    if (ok && hipMemset(c->ncnt, 0, N * 4) != hipSuccess) ok = false;
    if (ok && hipMemset(c->cell_of, 0, N * 4) != hipSuccess) ok = false;
    // reverse slots start as "absent"; no list is usable before a build
    if (ok && hipMemset(c->rev, 0xff, N * cfg->max_neigh_ang) != hipSuccess) ok = false;
    if (ok && hipMemset(c->status + ST_LBAD, 0xff, 4) != hipSuccess) ok = false;
    if (ok && hipDeviceSynchronize() != hipSuccess) ok = false;
    if (!ok) { nep_destroy(c); return NEP_E_HIP; }
    *out = c;
    return NEP_OK;
}

int nep_set_weights(nep_ctx *c, const nep_weights *w, int32_t on_device, void *stream)
{
    if (!c || !w || !w->c_rad || !w->c_ang || !w->q_scale || !w->w0 || !w->b0 || !w->w1) return NEP_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    struct Part { const float *src; int off, n; };
    const Part small_parts[] = {
        {w->c_rad, P_CR, NR * KB}, {w->c_ang, P_CA, NA * KB}, {w->q_scale, P_QS, DIM},
        {w->w0, P_W0, NH * DIM},   {w->b0, P_B0, NH},         {w->w1, P_W1, NH}};
    const Part wide_parts[] = {
        {w->c_rad, W_CR, WR * WKR}, {w->c_ang, W_CA, WA * WKA}, {w->q_scale, W_QS, WDIM},
        {w->w0, W_W0, WH * WDIM},   {w->b0, W_B0, WH},          {w->w1, W_W1, WH}};
    const Part *parts = c->wide ? wide_parts : small_parts;
    for (int k = 0; k < 6; ++k) {
        const Part &p = parts[k];
        if (on_device) HIP_TRY(hipMemcpyAsync(c->params + p.off, p.src, p.n * 4, kind, s));
        else HIP_TRY(hipMemcpy(c->params + p.off, p.src, p.n * 4, kind));
    }
    const int b1_off = c->wide ? W_B1 : P_B1;
    if (on_device) {
        // b1 is a host scalar even when the arrays live on the device
        HIP_TRY(hipMemcpyAsync(c->params + b1_off, &w->b1, 4, hipMemcpyHostToDevice, s));
    } else {
        HIP_TRY(hipMemcpy(c->params + b1_off, &w->b1, 4, hipMemcpyHostToDevice));
    }
    if (c->wide) k_w_params64<<<1, 128, 0, s>>>(c->params, c->c64);
    else k_params64<<<1, 64, 0, s>>>(c->params, c->c64);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return NEP_OK;
}

static int check_system(const nep_ctx *c, const nep_system *s, bool need_vel)
{
    if (!s || !s->x || !s->y || !s->z || !s->h) return NEP_E_ARG;
    if (s->n_atoms <= 0 || s->n_atoms > c->cfg.max_atoms) return NEP_E_ARG;
    const int nc = s->cell_start ? s->n_cells : 1;
    if (nc <= 0 || nc > c->cfg.max_cells) return NEP_E_ARG;
    if (s->cell_start) {
        if (s->cell_start[0] != 0 || s->cell_start[nc] != s->n_atoms) return NEP_E_ARG;
        for (int k = 0; k < nc; ++k)
            if (s->cell_start[k + 1] <= s->cell_start[k]) return NEP_E_ARG;
    }
    if (need_vel && (!s->vx || !s->vy || !s->vz || !(s->mass > 0))) return NEP_E_ARG;
    return NEP_OK;
}

static bool same_system(const nep_ctx *c, const nep_system *s)
{
    const int nc = s->cell_start ? s->n_cells : 1;
    if (!c->built || c->built_n != s->n_atoms || c->built_cells != nc) return false;
    for (int a = 0; a < 3; ++a)
        if (c->pbc[a] != (s->pbc[a] ? 1 : 0)) return false;
    if (memcmp(c->built_h.data(), s->h, (size_t)nc * 9 * sizeof(double)) != 0) return false;
    if (s->cell_start && memcmp(c->built_start.data(), s->cell_start, (size_t)(nc + 1) * 8) != 0) return false;
    return true;
}

// Geometry, bins and reduction chunks of a new system (host decisions).
static int setup_system(nep_ctx *c, const nep_system *s, hipStream_t st)
{
    c->border_valid = false;
    ++c->setup_gen;
    const int nc = s->cell_start ? s->n_cells : 1;
    const int64_t n = s->n_atoms;
    std::vector<int64_t> start(nc + 1);
    if (s->cell_start) for (int k = 0; k <= nc; ++k) start[k] = s->cell_start[k];
    else { start[0] = 0; start[1] = n; }
    const double lcut = c->hp.rc_rad + c->cfg.skin;
    c->geom.assign(nc, CellGeom());
    int64_t nbins = 0;
    bool small_images = false;
    int64_t max_cell_atoms = 0;
    for (int k = 0; k < nc; ++k) {
        CellGeom &g = c->geom[k];
        memset(&g, 0, sizeof g);
        memcpy(g.h, s->h + 9 * k, 9 * sizeof(double));
        inv3(g.h, g.hinv);
        if (!std::isfinite(g.hinv[0]) || !std::isfinite(g.hinv[4]) || !std::isfinite(g.hinv[8])) return NEP_E_ARG;
        for (int a = 0; a < 3; ++a) {
            const double q = g.hinv[0 * 3 + a] * g.hinv[0 * 3 + a] + g.hinv[1 * 3 + a] * g.hinv[1 * 3 + a] +
                             g.hinv[2 * 3 + a] * g.hinv[2 * 3 + a];
            const double width = 1.0 / std::sqrt(q);
            g.periodic[a] = s->pbc[a] ? 1 : 0;
            int nb = (int)std::floor(width / lcut);
            if (g.periodic[a]) {
                if (nb >= 3) { g.nb[a] = nb; g.R[a] = 0; }
                else {
                    g.nb[a] = 1;
                    g.R[a] = (int)std::ceil(lcut / width);
                    if (g.R[a] > 1) small_images = true;
                    if (g.R[a] > 7) return NEP_E_ARG;   // cell thinner than (rc + skin) / 7
                }
            } else {
                g.nb[a] = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
                g.R[a] = 0;
            }
        }
        const int64_t cb = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
        if (cb > (1 << 28)) return NEP_E_ARG;
        g.bin_offset = (int)nbins;
        nbins += cb;
        g.atom_start = (int)start[k];
        g.n_atoms = (int)(start[k + 1] - start[k]);
        max_cell_atoms = std::max<int64_t>(max_cell_atoms, g.n_atoms);
    }
    if (nbins > (1LL << 30)) return NEP_E_ARG;
    PairConsts &pc = c->pc;
    pc.rc_rad = (float)c->hp.rc_rad;
    pc.rc_ang = (float)c->hp.rc_ang;
    pc.rc_rad2 = pc.rc_rad * pc.rc_rad;
    pc.rc_ang2 = pc.rc_ang * pc.rc_ang;
    pc.rc_ang2_write = pc.rc_ang2 * (1.0f + 0x1p-16f);
    pc.rc_ang2_read = pc.rc_ang2 * (1.0f + 0x1p-17f);
    pc.inv_rc_rad = (float)(1.0 / c->hp.rc_rad);
    pc.inv_rc_ang = (float)(1.0 / c->hp.rc_ang);
    pc.inv_rc_rad_lo = (float)(1.0 / c->hp.rc_rad - (double)pc.inv_rc_rad);
    pc.inv_rc_ang_lo = (float)(1.0 / c->hp.rc_ang - (double)pc.inv_rc_ang);
    pc.zbl_r1 = (float)c->hp.zbl_r1;
    pc.zbl_r2 = (float)c->hp.zbl_r2;
    pc.zbl_r2sq = pc.zbl_r2 * pc.zbl_r2;
    pc.zbl_z = (float)c->hp.Z;
    pc.capA = c->cfg.max_neigh_ang;
    pc.capR = c->cfg.max_neigh_rad;
    if (small_images) { pc.ibits = 4; pc.ioff = 8; pc.jbits = 20; }
    else { pc.ibits = 2; pc.ioff = 1; pc.jbits = 26; }
    pc.code0 = (uint32_t)pc.ioff | ((uint32_t)pc.ioff << pc.ibits) | ((uint32_t)pc.ioff << (2 * pc.ibits));
    // bin edge vectors; bin-offset mode for one periodic cell binned along
    // every axis with at most 2^23 atoms (23 index bits + 5 offset + 3 face)
    for (int k = 0; k < nc; ++k)
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) c->geom[k].bv[3 * a + d] = c->geom[k].h[3 * a + d] / c->geom[k].nb[a];
    {
        const CellGeom &g = c->geom[0];
        bool delta = nc == 1 && n <= (1LL << 23);
        for (int a = 0; a < 3; ++a) delta = delta && g.periodic[a] && g.R[a] == 0;
        pc.delta = delta ? 1 : 0;
        pc.qs = pc.qsinv = 1.0;
        if (delta) {
            pc.jbits = 23;
            // fixed-point unit of the force records' offsets: an atom lies in
            // its bin (sum of the edge vectors) give or take half the skin
            // until the next build; 1 A more for safety
            double range = 0.0;
            for (int d = 0; d < 3; ++d)
                range = std::max(range, std::fabs(g.bv[d]) + std::fabs(g.bv[3 + d]) + std::fabs(g.bv[6 + d]));
            range += c->cfg.skin + 1.0;
            const int kq = (int)std::floor(std::log2(2147483000.0 / range));
            pc.qs = std::ldexp(1.0, -kq);
            pc.qsinv = std::ldexp(1.0, kq);
        }
    }
    if (max_cell_atoms > (1LL << pc.jbits)) return NEP_E_ARG;
    // no-image test: the crossing bits clear, or the code of the cell itself
    pc.img_mask = pc.delta ? ~31u : 0xffffffffu;
    pc.img_val = pc.delta ? 0u : pc.code0;
    pc.n = (int)n;
    pc.rmask = c->rmask;
    pc.cmask = c->cmask;
    pc.rc_cand = (float)(c->hp.rc_rad + CAND_MARGIN);
    pc.amask = c->amask;

    // bins
    if (nbins + 1 > c->bin_cap) {
        int32_t *old_bufs[] = {c->bin_count, c->bin_start, c->bin_fill, c->scan_sums, c->bin_rank, c->bin_lin};
        for (int32_t *p : old_bufs)
            if (p) (void)hipFree(p);
        c->bin_count = c->bin_start = c->bin_fill = c->scan_sums = c->bin_rank = c->bin_lin = nullptr;
        c->bin_cap = 0;
        const int64_t cap = nbins + 1;
        HIP_TRY(hipMalloc(&c->bin_count, cap * 4));
        HIP_TRY(hipMalloc(&c->bin_start, cap * 4));
        HIP_TRY(hipMalloc(&c->bin_fill, cap * 4));
        HIP_TRY(hipMalloc(&c->scan_sums, ((cap + 2047) / 2048 + 1) * 4));
        HIP_TRY(hipMalloc(&c->bin_rank, cap * 4));
        HIP_TRY(hipMalloc(&c->bin_lin, cap * 4));
        c->bin_cap = cap;
    }
    c->n_bins = (int)nbins;
    // Morton order of every cell's bins: rank[lin] and its inverse lin[rank]
    std::vector<int32_t> rank(nbins), lin_of(nbins);
    {
        auto spread = [](uint64_t v) {   // interleave the low 21 bits with two zero bits
            v &= 0x1fffff;
            v = (v | v << 32) & 0x1f00000000ffffULL;
            v = (v | v << 16) & 0x1f0000ff0000ffULL;
            v = (v | v << 8) & 0x100f00f00f00f00fULL;
            v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
            v = (v | v << 2) & 0x1249249249249249ULL;
            return v;
        };
        std::vector<std::pair<uint64_t, int32_t>> key;
        for (int k = 0; k < nc; ++k) {
            const CellGeom &g = c->geom[k];
            const int cb = g.nb[0] * g.nb[1] * g.nb[2];
            key.resize(cb);
            for (int l = 0; l < cb; ++l) {
                const int b0 = l % g.nb[0], b1 = (l / g.nb[0]) % g.nb[1], b2 = l / (g.nb[0] * g.nb[1]);
                key[l] = {spread(b0) | spread(b1) << 1 | spread(b2) << 2, l};
            }
            std::sort(key.begin(), key.end());
            for (int r = 0; r < cb; ++r) {
                rank[g.bin_offset + key[r].second] = r;
                lin_of[g.bin_offset + r] = key[r].second;
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(c->bin_rank, rank.data(), nbins * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->bin_lin, lin_of.data(), nbins * 4, hipMemcpyHostToDevice, st));

    // reduction chunks: contiguous sorted-atom ranges that never span two cells
    const int CH = 4096;
    std::vector<int32_t> cb, ce, cc(nc + 1);
    for (int k = 0; k < nc; ++k) {
        cc[k] = (int32_t)cb.size();
        for (int64_t a = start[k]; a < start[k + 1]; a += CH) {
            cb.push_back((int32_t)a);
            ce.push_back((int32_t)std::min<int64_t>(a + CH, start[k + 1]));
        }
    }
    cc[nc] = (int32_t)cb.size();
    const int nch = (int)cb.size();
    if (nch > c->chunk_cap) {
        if (c->chunk_begin) {
            (void)hipFree(c->chunk_begin);
            (void)hipFree(c->chunk_end);
            (void)hipFree(c->part);
        }
        c->chunk_begin = c->chunk_end = nullptr;
        c->part = nullptr;
        HIP_TRY(hipMalloc(&c->chunk_begin, nch * 4));
        HIP_TRY(hipMalloc(&c->chunk_end, nch * 4));
        HIP_TRY(hipMalloc(&c->part, (size_t)nch * 10 * 8));
        c->chunk_cap = nch;
    }
    if (!c->cell_chunk) HIP_TRY(hipMalloc(&c->cell_chunk, ((size_t)c->cfg.max_cells + 1) * 4));
    c->n_chunks = nch;
    HIP_TRY(hipMemcpyAsync(c->chunk_begin, cb.data(), nch * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->chunk_end, ce.data(), nch * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->cell_chunk, cc.data(), (nc + 1) * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->cells, c->geom.data(), nc * sizeof(CellGeom), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->cell_start_d, start.data(), (nc + 1) * 8, hipMemcpyHostToDevice, st));
    // bin blocks of the list build: one cell binned along every axis (its
    // halo bins are then distinct), bin keys within the sort's 27 bits
    c->lb_blocks = 0;
    if (nc == 1 && nbins < (1 << 27)) {
        const CellGeom &g = c->geom[0];
        bool ok = true;
        for (int a = 0; a < 3; ++a)
            if (g.R[a] != 0 || g.nb[a] > 2046) ok = false;
        if (ok) {
            int nk[3];
            for (int a = 0; a < 3; ++a) nk[a] = (g.nb[a] + 1) / 2;
            const int64_t nblk = (int64_t)nk[0] * nk[1] * nk[2];
            auto spread = [](uint64_t v) {   // interleave the low 21 bits with two zero bits
                v &= 0x1fffff;
                v = (v | v << 32) & 0x1f00000000ffffULL;
                v = (v | v << 16) & 0x1f0000ff0000ffULL;
                v = (v | v << 8) & 0x100f00f00f00f00fULL;
                v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
                v = (v | v << 2) & 0x1249249249249249ULL;
                return v;
            };
            std::vector<std::pair<uint64_t, uint32_t>> key(nblk);
            for (int64_t l = 0; l < nblk; ++l) {
                const int b0 = (int)(l % nk[0]), b1 = (int)((l / nk[0]) % nk[1]);
                const int b2 = (int)(l / ((int64_t)nk[0] * nk[1]));
                key[l] = {spread(b0) | spread(b1) << 1 | spread(b2) << 2, pack_block(b0, b1, b2)};
            }
            std::sort(key.begin(), key.end());
            std::vector<uint32_t> coord(nblk);
            for (int64_t r = 0; r < nblk; ++r) coord[r] = key[r].second;
            if (nblk > c->lb_cap) {
                if (c->blk_coord) (void)hipFree(c->blk_coord);
                c->blk_coord = nullptr;
                c->lb_cap = 0;
                HIP_TRY(hipMalloc(&c->blk_coord, nblk * 4));
                c->lb_cap = nblk;
            }
            HIP_TRY(hipMemcpyAsync(c->blk_coord, coord.data(), nblk * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
            c->lb_blocks = (int)nblk;
        }
    }
    // cell index of every atom
    k_cell_of<<<grid_for(n, 256), 256, 0, st>>>((int)n, nc, c->cell_start_d, c->cell_of);
    HIP_TRY(hipGetLastError());
    // the host vectors above are released on return: wait for the copies
    HIP_TRY(hipStreamSynchronize(st));

    {
        const int b = bucket_of(n);
        c->shape_desc = c->tuned_desc[b] >= 0 ? c->tuned_desc[b] : DEFAULT_SHAPE_DESC;
        c->shape_force = c->tuned_force[b] >= 0 ? c->tuned_force[b] : DEFAULT_SHAPE_FORCE;
    }
    c->built_n = n;
    c->built_cells = nc;
    c->built_h.assign(s->h, s->h + 9 * nc);
    c->built_start = start;
    for (int a = 0; a < 3; ++a) c->pbc[a] = s->pbc[a] ? 1 : 0;
    return NEP_OK;
}

// Launch the list build on `st`; with `flag` non-NULL every kernel returns
// at once unless *flag is set on the device.
static int launch_build(nep_ctx *c, const nep_system *s, hipStream_t st, const int32_t *flag)
{
    const int n = (int)s->n_atoms;
    const int nb1 = c->n_bins + 1;
    k_fill_i32<<<grid_for(nb1, 256), 256, 0, st>>>(nb1, c->bin_count, 0, flag);
    k_fill_i32<<<grid_for(nb1, 256), 256, 0, st>>>(nb1, c->bin_fill, 0, flag);
    k_bin_assign<<<grid_for(n, 256), 256, 0, st>>>(n, s->x, s->y, s->z, c->cell_of, c->cells, c->bin_of,
                                                   c->wrap, c->bin_count, c->xref, c->bin_rank, c->status, flag);
    const int nblk = grid_for(nb1, 2048);
    k_scan_blocks<<<nblk, 256, 0, st>>>(nb1, c->bin_count, c->bin_start, c->scan_sums, flag);
    k_scan_sums<<<1, 256, 0, st>>>(nblk, c->scan_sums, flag);
    k_scan_add<<<grid_for(nb1, 256), 256, 0, st>>>(nb1, c->bin_start, c->scan_sums, flag);
    k_bin_scatter<<<grid_for(n, 256), 256, 0, st>>>(n, c->bin_of, c->bin_start, c->bin_fill, c->tmp, flag);
    k_bin_rank<<<grid_for(n, 256), 256, 0, st>>>(n, c->bin_of, c->bin_start, c->tmp, c->cell_of, c->cells,
                                                 c->perm, c->bin_sorted, c->bin_lin, flag);
    // sorted positions for the list build (skipped with the rest of the
    // build when the flag says no rebuild; every evaluation refreshes them)
    k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of,
                                                       c->cells, c->xq, c->status, flag,
                                                       c->bin_sorted, c->pc.qsinv, wide_xf(c));
    const double lA = c->hp.rc_ang + c->cfg.skin, lR = c->hp.rc_rad + c->cfg.skin;
    if (c->lb_blocks > 0)
        k_build_lists_blocks<<<xcd_grid(c->lb_blocks), LB_BS, 0, st>>>(
            c->pc, lA * lA, lR * lR, c->hp.rc_ang * c->hp.rc_ang, c->hp.rc_rad * c->hp.rc_rad, c->xq, c->cells,
            c->bin_sorted, c->bin_start, c->bin_rank, c->blk_coord, c->lb_blocks, c->nl_ang, c->nl_rad, c->ncnt,
            c->status, flag);
    else
        k_build_lists<<<grid_for(n, 256), 256, 0, st>>>(
            c->pc, lA * lA, lR * lR, c->hp.rc_ang * c->hp.rc_ang, c->hp.rc_rad * c->hp.rc_rad, c->xq, c->cell_of,
            c->cells, c->bin_sorted, c->bin_start, c->bin_rank, c->nl_ang, c->nl_rad, c->ncnt, c->status, flag,
            c->n_bins < (1 << 27) ? 1 : 0);
    k_build_reverse<<<grid_for(n, 256), 256, 0, st>>>(c->pc, c->cell_of, c->cells, c->nl_ang, c->ncnt, c->rev,
                                                      c->status, flag, c->n_bins < (1 << 27) ? 1 : 0);
    // the lists are usable only if the build latched no error
    k_lists_commit<<<1, 64, 0, st>>>(c->status, flag);
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

int nep_update_neighbors(nep_ctx *c, const nep_system *s, void *stream)
{
    if (!c) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if (!c->built || !same_system(c, s)) return nep_build_neighbors(c, s, stream);
    // the rebuild decision on the device: the largest displacement since the
    // last build against skin/2 (unusable lists are rebuilt as well); the
    // build's launches skip their work when the flag says no
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)s->n_atoms;
    const double half_skin2 = 0.25 * c->cfg.skin * c->cfg.skin;
    k_disp<<<stream_grid(n), 256, 0, st>>>(n, s->x, s->y, s->z, c->xref, c->md);
    k_rebuild_flag<<<1, 64, 0, st>>>(half_skin2, c->md, c->flag, c->status);
    return launch_build(c, s, st, c->flag);
}

int nep_build_neighbors(nep_ctx *c, const nep_system *s, void *stream)
{
    if (!c) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!same_system(c, s)) {
        c->built = false;
        rc = setup_system(c, s, st);
        if (rc) return rc;
    }
    HIP_TRY(hipMemsetAsync(c->status + ST_NEED_A, 0, 2 * 4, st));
    rc = launch_build(c, s, st, nullptr);
    if (rc) return rc;
    c->built = true;
    return NEP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ launch shapes
struct Shape {
    int bs;
    bool persistent;
};
static const Shape SHAPES[6] = {{64, false}, {128, false}, {256, false}, {64, true}, {128, true}, {256, true}};
static const int N_SHAPES = 6;

template <int BS, bool PE, int NNMODE>
static void launch_desc_t(nep_ctx *c, hipStream_t st)
{
    const int n = c->pc.n, tiles = (n + BS - 1) / BS;
    int grid = xcd_grid(tiles);
    if (PE) {
        int per_cu = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_descriptor<BS, PE, NNMODE>, BS, 0);
        grid = std::max(1, std::min(tiles, 256 * std::max(per_cu, 1)));
    }
    k_descriptor<BS, PE, NNMODE><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xp, c->cell_of, c->cells, c->nl_ang, c->nl_rad,
                                                      c->ncnt, c->params, c->c64, c->pair_grad, c->f_own, c->w_atom,
                                                      c->e_atom, c->status, tiles, c->cflag, c->bin_sorted);
}

template <int BS, bool PE>
static void launch_desc_m(nep_ctx *c, hipStream_t st)
{
    if (c->nn_mode == 1) launch_desc_t<BS, PE, 1>(c, st);
    else if (c->nn_mode == 2) launch_desc_t<BS, PE, 2>(c, st);
    else launch_desc_t<BS, PE, 0>(c, st);
}

template <int BS, bool PE>
static void launch_force_t(nep_ctx *c, const nep_efv *o, hipStream_t st)
{
    const int n = c->pc.n, tiles = (n + BS - 1) / BS;
    int grid = xcd_grid(tiles);
    if (PE) {
        int per_cu = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force<BS, PE, false>, BS, 0);
        grid = std::max(1, std::min(tiles, 256 * std::max(per_cu, 1)));
    }
    // the descriptor kernel wrote 48-byte records in bin-offset mode
    if (c->pc.delta)
        k_force<BS, PE, true><<<grid, BS, 0, st>>>(c->pc, c->xp, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                                   c->rev, c->pair_grad, c->f_own, c->perm, o->fx, o->fy, o->fz,
                                                   c->w_atom, c->status, tiles);
    else
        k_force<BS, PE, false><<<grid, BS, 0, st>>>(c->pc, c->xp, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                                    c->rev, c->pair_grad, c->f_own, c->perm, o->fx, o->fy, o->fz,
                                                    c->w_atom, c->status, tiles);
}

static void launch_desc(nep_ctx *c, int shape, hipStream_t st)
{
    switch (shape) {
    case 0: launch_desc_m<64, false>(c, st); break;
    case 1: launch_desc_m<128, false>(c, st); break;
    case 3: launch_desc_m<64, true>(c, st); break;
    case 4: launch_desc_m<128, true>(c, st); break;
    case 5: launch_desc_m<256, true>(c, st); break;
    default: launch_desc_m<256, false>(c, st); break;
    }
}

static void launch_force(nep_ctx *c, int shape, const nep_efv *o, hipStream_t st)
{
    switch (shape) {
    case 0: launch_force_t<64, false>(c, o, st); break;
    case 1: launch_force_t<128, false>(c, o, st); break;
    case 3: launch_force_t<64, true>(c, o, st); break;
    case 4: launch_force_t<128, true>(c, o, st); break;
    case 5: launch_force_t<256, true>(c, o, st); break;
    default: launch_force_t<256, false>(c, o, st); break;
    }
}

// The paper-size model's descriptor phases and force kernel (nep_wide.h), in
// blocks of BS threads (shapes 0, 1, 2: 64, 128, 256; the persistent shapes
// of the default model's kernels do not exist here): the staged sums,
// descriptors and network adjoints ...
template <int BS>
static void launch_wide_sums_t(nep_ctx *c, hipStream_t st)
{
    const int n = c->pc.n, grid = xcd_grid((n + BS - 1) / BS);
    if (c->pc.delta) {
        // bin-offset mode: the walks gather the 16-byte fixed-point positions
        // the position refresh wrote
        k_w_radial<BS, true><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang,
                                                  c->nl_rad, c->ncnt, c->params, c->w_Q, c->e_atom, c->status,
                                                  c->cflag);
    } else {
        k_w_radial<BS, false><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang,
                                                   c->nl_rad, c->ncnt, c->params, c->w_Q, c->e_atom, c->status,
                                                   c->cflag);
    }
    for (int g = 0; g < WNGA; ++g) {
        if (c->pc.delta)
            k_w_angular<BS, true><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang, c->ncnt,
                                                       c->c64, g, c->w_S, c->w_Q);
        else
            k_w_angular<BS, false><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang,
                                                        c->ncnt, c->c64, g, c->w_S, c->w_Q);
    }
    // bin-offset mode: the records carry fixed-point positions (WAtomRec80)
    const int32_t *bs = c->pc.delta ? c->bin_sorted : nullptr;
    if (c->nn_mode != 0) {
        // the hidden layer on the matrix cores (FP32 or BF16 operands): a
        // persistent grid, three blocks of four wavefronts per CU
        const int ntiles = (n + 63) / 64;
        const int blocks = std::max(1, std::min((ntiles + 3) / 4, 3 * 256));
        if (c->nn_mode == 2)
            k_w_network_mfma<false><<<blocks, WN_BS, 0, st>>>(n, ntiles, c->xq, c->params, c->w_Q, c->xw, c->w_FpA,
                                                              c->e_atom, c->cells, bs, c->pc.qsinv, c->status);
        else
            k_w_network_mfma<true><<<blocks, WN_BS, 0, st>>>(n, ntiles, c->xq, c->params, c->w_Q, c->xw, c->w_FpA,
                                                             c->e_atom, c->cells, bs, c->pc.qsinv, c->status);
    } else {
        k_w_network<BS><<<grid, BS, 0, st>>>(n, c->xq, c->params, c->w_Q, c->xw, c->w_FpA, c->e_atom, c->cells, bs,
                                             c->pc.qsinv, c->status);
    }
}

// ... then the pair gradients
template <int BS>
static void launch_wide_desc_t(nep_ctx *c, hipStream_t st)
{
    const int n = c->pc.n, grid = xcd_grid((n + BS - 1) / BS);
    launch_wide_sums_t<BS>(c, st);
    if (c->pc.delta)
        k_w_grad<BS, true><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang, c->ncnt,
                                                c->params, c->c64, c->w_S, c->w_FpA, c->pair_grad, c->f_own,
                                                c->w_atom);
    else
        k_w_grad<BS, false><<<grid, BS, 0, st>>>(c->pc, c->xq, c->xf, c->cell_of, c->cells, c->nl_ang, c->ncnt,
                                                 c->params, c->c64, c->w_S, c->w_FpA, c->pair_grad, c->f_own,
                                                 c->w_atom);
}

template <int BS>
static void launch_wide_force_t(nep_ctx *c, const nep_efv *o, hipStream_t st)
{
    const int n = c->pc.n, grid = xcd_grid((n + BS - 1) / BS);
    if (c->pc.delta)
        k_w_force<BS, true><<<grid, BS, 0, st>>>(c->pc, c->xw, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                                 c->rev, c->pair_grad, c->f_own, c->perm, o->fx, o->fy, o->fz,
                                                 c->w_atom, c->status);
    else
        k_w_force<BS, false><<<grid, BS, 0, st>>>(c->pc, c->xw, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                                  c->rev, c->pair_grad, c->f_own, c->perm, o->fx, o->fy, o->fz,
                                                  c->w_atom, c->status);
}

static const int N_WIDE_SHAPES = 3;

static void launch_wide_sums(nep_ctx *c, hipStream_t st)
{
    if (c->shape_desc == 1) launch_wide_sums_t<128>(c, st);
    else if (c->shape_desc == 2) launch_wide_sums_t<256>(c, st);
    else launch_wide_sums_t<64>(c, st);
}

static void launch_wide_desc(nep_ctx *c, int shape, hipStream_t st)
{
    if (shape == 1) launch_wide_desc_t<128>(c, st);
    else if (shape == 2) launch_wide_desc_t<256>(c, st);
    else launch_wide_desc_t<64>(c, st);
}

static void launch_wide_force(nep_ctx *c, int shape, const nep_efv *o, hipStream_t st)
{
    if (shape == 0) launch_wide_force_t<64>(c, o, st);
    else if (shape == 1) launch_wide_force_t<128>(c, o, st);
    else launch_wide_force_t<256>(c, o, st);
}

extern "C" {

static void launch_desc_any(nep_ctx *c, hipStream_t st)
{
    if (c->wide) launch_wide_desc(c, c->shape_desc, st);
    else launch_desc(c, c->shape_desc, st);
}

static void launch_force_any(nep_ctx *c, const nep_efv *o, hipStream_t st)
{
    if (c->wide) launch_wide_force(c, c->shape_force, o, st);
    else launch_force(c, c->shape_force, o, st);
}

// One evaluation: sorted positions, descriptor + network, forces, reductions.
// ev (may be NULL): three events recorded on st before the descriptor
// kernel(s), between them and the force kernel, and after it.
// One evaluation.  md_step: inside the MD loop, where k_cand_update has
// decided whether the descriptor's radial walk goes over every entry or only
// over the candidates of the last full walk; any other evaluation walks in
// full (and writes the candidate mask).
static int launch_efv(nep_ctx *c, const nep_system *s, nep_efv *o, hipStream_t st, bool refresh_positions,
                      hipEvent_t *ev = nullptr, bool md_step = false)
{
    const int n = (int)s->n_atoms;
    if (!md_step) k_set_flag<<<1, 64, 0, st>>>(c->cflag, 1);
    if (refresh_positions)
        k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of,
                                                           c->cells, c->xq, c->status, nullptr,
                                                           c->bin_sorted, c->pc.qsinv, wide_xf(c));
    if (ev) HIP_TRY(hipEventRecord(ev[0], st));
    launch_desc_any(c, st);
    if (ev) HIP_TRY(hipEventRecord(ev[1], st));
    launch_force_any(c, o, st);
    if (ev) HIP_TRY(hipEventRecord(ev[2], st));
    k_reduce_chunks<<<c->n_chunks, 256, 0, st>>>(c->chunk_begin, c->chunk_end, c->e_atom, c->w_atom, c->part,
                                                 c->status);
    k_reduce_cells<<<c->built_cells, 256, 0, st>>>(c->built_cells, c->cell_chunk, c->part,
                                                                o->energy, o->virial, c->status);
    if (o->energy_atom)
        k_energy_atom_out<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, c->e_atom, o->energy_atom);
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

static int check_out(const nep_efv *o)
{
    if (!o || !o->energy || !o->fx || !o->fy || !o->fz) return NEP_E_ARG;
    return NEP_OK;
}

int nep_compute_efv(nep_ctx *c, const nep_system *s, nep_efv *o, void *stream)
{
    if (!c) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if (!same_system(c, s)) return NEP_E_STATE;
    return launch_efv(c, s, o, (hipStream_t)stream, true);
}

int nep_time_efv(nep_ctx *c, const nep_system *s, nep_efv *o, int32_t reps, double *ms, void *stream)
{
    if (!c || !ms || reps <= 0) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if (!same_system(c, s)) return NEP_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)s->n_atoms;
    hipEvent_t ev[5];
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    double acc[4] = {0, 0, 0, 0};
    k_set_flag<<<1, 64, 0, st>>>(c->cflag, 1);   // full radial walks
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(hipEventRecord(ev[0], st));
        k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of,
                                                           c->cells, c->xq, c->status, nullptr,
                                                           c->bin_sorted, c->pc.qsinv, wide_xf(c));
        HIP_TRY(hipEventRecord(ev[1], st));
        launch_desc_any(c, st);
        HIP_TRY(hipEventRecord(ev[2], st));
        launch_force_any(c, o, st);
        HIP_TRY(hipEventRecord(ev[3], st));
        k_reduce_chunks<<<c->n_chunks, 256, 0, st>>>(c->chunk_begin, c->chunk_end, c->e_atom, c->w_atom,
                                                     c->part, c->status);
        k_reduce_cells<<<c->built_cells, 256, 0, st>>>(c->built_cells, c->cell_chunk, c->part,
                                                                    o->energy, o->virial, c->status);
        HIP_TRY(hipEventRecord(ev[4], st));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventSynchronize(ev[4]));
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            acc[k] += t;
        }
    }
    for (auto &e : ev) HIP_TRY(hipEventDestroy(e));
    for (int k = 0; k < 4; ++k) ms[k] = acc[k] / reps;
    return NEP_OK;
}


int nep_set_precision(nep_ctx *c, int32_t mode)
{
    if (!c || mode < 0 || mode > 2) return NEP_E_ARG;
    c->nn_mode = mode;
    return NEP_OK;
}

int nep_num_params(const nep_ctx *c)
{
    if (!c) return NEP_E_ARG;
    if (c->wide) return W_NPARAM;
    return N_PARAMS;
}

static int backward_checks(nep_ctx *c, const nep_system *s, const nep_efv *o, const double *gE,
                           const double *grad_params, const double *gx, const double *gy, const double *gz,
                           const double *gh)
{
    if (!c || !gE || !grad_params) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if ((gx || gy || gz) && !(gx && gy && gz)) return NEP_E_ARG;
    if (gh && !o->virial) return NEP_E_ARG;
    if (!same_system(c, s)) return NEP_E_STATE;
    return NEP_OK;
}

// The backward's launches, with `part` holding at least `blocks` partial rows.
static int backward_launch(nep_ctx *c, const nep_system *s, const nep_efv *o, const double *gE,
                           double *grad_params, double *gx, double *gy, double *gz, double *gh, double *part,
                           int blocks, int tiles, hipStream_t st)
{
    const int n = (int)s->n_atoms;
    k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of,
                                                       c->cells, c->xq, c->status, nullptr,
                                                       c->bin_sorted, c->pc.qsinv, wide_xf(c));
    if (c->wide) {
        // the staged sums, descriptors and adjoints of these positions (a
        // full radial walk, as in any evaluation outside the MD loop)
        k_set_flag<<<1, 64, 0, st>>>(c->cflag, 1);
        launch_wide_sums(c, st);
        k_w_param_grad<<<blocks, 64, 0, st>>>(c->pc, c->xq, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                              c->params, c->w_Q, c->w_S, c->w_FpA, gE, part, c->status, tiles);
    } else {
        k_param_grad<<<blocks, 64, 0, st>>>(c->pc, c->xq, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt,
                                            c->params, c->c64, gE, part, c->status, tiles);
    }
    const int np = nep_num_params(c);
    k_param_reduce<<<(np + 31) / 32, 256, 0, st>>>(blocks, np, part, grad_params);
    if (gx) k_grad_pos<<<grid_for(n, 256), 256, 0, st>>>(n, c->cell_of, gE, o->fx, o->fy, o->fz, gx, gy, gz);
    if (gh)
        k_grad_cell<<<c->built_cells, 256, 0, st>>>(c->cells, s->x, s->y, s->z, o->fx, o->fy, o->fz, o->virial,
                                                    gE, gh);
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

int nep_backward(nep_ctx *c, const nep_system *s, const nep_efv *o, const double *gE, double *grad_params,
                 double *gx, double *gy, double *gz, double *gh, void *stream)
{
    int rc = backward_checks(c, s, o, gE, grad_params, gx, gy, gz, gh);
    if (rc) return rc;
    const int tiles = (int)((s->n_atoms + 63) / 64);
    const int blocks = std::min(tiles, PG_MAX_BLOCKS);
    if (blocks > c->pg_blocks) {
        if (c->pg_part) (void)hipFree(c->pg_part);
        c->pg_part = nullptr;
        HIP_TRY(hipMalloc(&c->pg_part, (size_t)blocks * nep_num_params(c) * sizeof(double)));
        c->pg_blocks = blocks;
    }
    return backward_launch(c, s, o, gE, grad_params, gx, gy, gz, gh, c->pg_part, blocks, tiles,
                           (hipStream_t)stream);
}

int nep_backward_noalloc(nep_ctx *c, const nep_system *s, const nep_efv *o, const double *gE,
                         double *grad_params, double *gx, double *gy, double *gz, double *gh, void *stream)
{
    int rc = backward_checks(c, s, o, gE, grad_params, gx, gy, gz, gh);
    if (rc) return rc;
    const int tiles = (int)((s->n_atoms + 63) / 64);
    const int blocks = std::min(tiles, PG_MAX_BLOCKS);
    if ((size_t)blocks * nep_num_params(c) > (size_t)PG_MAX_BLOCKS * PG_MAX_PARAMS) return NEP_E_CAPACITY;
    double *part = nullptr;
    if ((rc = scratch_address(c->device, &part))) return rc;
    // every block zeroes its own rows before adding to them, so the rows a
    // previous call left behind need no clearing
    return backward_launch(c, s, o, gE, grad_params, gx, gy, gz, gh, part, blocks, tiles, (hipStream_t)stream);
}

int nep_autotune(nep_ctx *c, const nep_system *s, nep_efv *o, int32_t reps, int32_t *shape_out, void *stream)
{
    if (!c || reps <= 0) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if (!same_system(c, s)) return NEP_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)s->n_atoms;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    k_set_flag<<<1, 64, 0, st>>>(c->cflag, 1);   // full radial walks
    k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of,
                                                       c->cells, c->xq, c->status, nullptr,
                                                       c->bin_sorted, c->pc.qsinv, wide_xf(c));
    auto time_it = [&](auto &&launch) -> float {
        launch();   // warm-up
        HIP_TRY(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) launch();
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        return ms;
    };
    // the paper-size model's phases come in the three non-persistent shapes
    const int n_shapes = c->wide ? N_WIDE_SHAPES : N_SHAPES;
    auto desc = [&](int k) {
        if (c->wide) launch_wide_desc(c, k, st);
        else launch_desc(c, k, st);
    };
    auto force = [&](int k) {
        if (c->wide) launch_wide_force(c, k, o, st);
        else launch_force(c, k, o, st);
    };
    int best_d = 2, best_f = 2;
    float t_best = 1e30f;
    for (int k = 0; k < n_shapes; ++k) {
        const float t = time_it([&] { desc(k); });
        if (t < t_best) { t_best = t; best_d = k; }
    }
    desc(best_d);
    t_best = 1e30f;
    for (int k = 0; k < n_shapes; ++k) {
        const float t = time_it([&] { force(k); });
        if (t < t_best) { t_best = t; best_f = k; }
    }
    HIP_TRY(hipEventDestroy(e0));
    HIP_TRY(hipEventDestroy(e1));
    HIP_TRY(hipGetLastError());
    const int b = bucket_of(n);
    c->tuned_desc[b] = c->shape_desc = best_d;
    c->tuned_force[b] = c->shape_force = best_f;
    if (shape_out) { shape_out[0] = best_d; shape_out[1] = best_f; }
    return NEP_OK;
}

int nep_compute_efv_graph(nep_ctx *c, const nep_system *s, nep_efv *o, void *stream)
{
    if (!c || !stream) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if (!same_system(c, s)) return NEP_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<uintptr_t> key = {
        (uintptr_t)s->n_atoms, (uintptr_t)s->x, (uintptr_t)s->y, (uintptr_t)s->z, (uintptr_t)o->energy,
        (uintptr_t)o->fx, (uintptr_t)o->fy, (uintptr_t)o->fz, (uintptr_t)o->virial, (uintptr_t)o->energy_atom,
        (uintptr_t)c->shape_desc, (uintptr_t)c->shape_force, (uintptr_t)c->n_chunks, (uintptr_t)c->built_cells,
        (uintptr_t)c->nn_mode, (uintptr_t)c->setup_gen};
    if (!c->graph_exec || key != c->graph_key) {
        if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int lrc = launch_efv(c, s, o, st, true);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (lrc != NEP_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return lrc != NEP_OK ? lrc : NEP_E_HIP;
        }
        c->graph = g;
        HIP_TRY(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
        c->graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(c->graph_exec, st));
    return NEP_OK;
}

int nep_status(nep_ctx *c, void *stream)
{
    if (!c) return NEP_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(c->h_status, c->status, 8 * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int code = c->h_status[ST_ERR];
    if (code != 0) {
        const int32_t zero = 0;
        HIP_TRY(hipMemcpy(c->status + ST_ERR, &zero, 4, hipMemcpyHostToDevice));
    }
    return code;
}

int nep_required_neighbors(nep_ctx *c, int32_t *ang, int32_t *rad)
{
    if (!c || !ang || !rad) return NEP_E_ARG;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c->h_status, c->status, 8 * 4, hipMemcpyDeviceToHost));
    *ang = c->h_status[ST_NEED_A];
    *rad = c->h_status[ST_NEED_R];
    return NEP_OK;
}

int nep_mean_neighbors(nep_ctx *c, void *stream, double *mean_rad, double *mean_ang)
{
    if (!c || !mean_rad || !mean_ang || !c->built) return NEP_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(c->counts, 0, 16, st));
    const int n = c->pc.n;
    k_count_inside<<<grid_for(n, 256), 256, 0, st>>>(c->pc, c->xq, c->cell_of, c->cells,
                                                     c->nl_ang, c->nl_rad, c->ncnt, c->counts);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->h_counts, c->counts, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *mean_rad = (double)c->h_counts[0] / n;
    *mean_ang = (double)c->h_counts[1] / n;
    return NEP_OK;
}

int nep_step_verlet(nep_ctx *c, nep_system *s, const nep_md *md, int32_t n_steps, nep_efv *o,
                    nep_md_stats *stats, void *stream)
{
    if (!c || !md || n_steps < 0) return NEP_E_ARG;
    int rc = check_system(c, s, true);
    if (rc) return rc;
    if ((rc = check_out(o))) return rc;
    if (!(md->dt_max > 0) || !(md->max_disp >= 0) || !(md->dt_min >= 0)) return NEP_E_ARG;
    const bool thermo = md->thermo_chain != 0;
    if (thermo) {
        if (md->thermo_chain < 0 || md->thermo_chain > MD_NHC_MAX || !(md->thermo_T > 0) ||
            !(md->thermo_tau > 0) || !(md->thermo_border >= 0) || md->thermo_axes < 1 || md->thermo_axes > 7)
            return NEP_E_ARG;
        if ((s->cell_start ? s->n_cells : 1) != 1) return NEP_E_UNSUPPORTED;
        const double *h = s->h;
        if (h[1] != 0 || h[2] != 0 || h[3] != 0 || h[5] != 0 || h[6] != 0 || h[7] != 0 || !(h[0] > 0) ||
            !(h[4] > 0) || !(h[8] > 0))
            return NEP_E_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)s->n_atoms;
    const double acc = ACC_EV_U_A / s->mass;
    const double half_skin2 = 0.25 * c->cfg.skin * c->cfg.skin;
    const int sg = stream_grid(n);

    // reset the step state (the pinned staging buffer is idle: the previous
    // chunk synchronised before reading it); the chain state is kept
    for (int k = 0; k < MD_WORDS; ++k) c->h_md[k] = 0.0;
    HIP_TRY(hipMemcpyAsync(c->md, c->h_md, MD_STEP_WORDS * 8, hipMemcpyHostToDevice, st));
    // lists valid for the current positions?
    bool fresh = false;
    if (!same_system(c, s)) {
        c->built = false;
        if ((rc = setup_system(c, s, st))) return rc;
        if ((rc = launch_build(c, s, st, nullptr))) return rc;
        c->built = true;
        fresh = true;
    } else {
        k_disp<<<sg, 256, 0, st>>>(n, s->x, s->y, s->z, c->xref, c->md);
        k_rebuild_flag<<<1, 64, 0, st>>>(half_skin2, c->md, c->flag, c->status);
        if ((rc = launch_build(c, s, st, c->flag))) return rc;
    }
    const bool initial = !md->forces_valid || fresh;
    if (initial) {
        if ((rc = launch_efv(c, s, o, st, true))) return rc;
    }
    // the candidate bound starts from that full walk, or forces one at the
    // first step (the positions may have changed since the last call)
    k_cand_set<<<1, 64, 0, st>>>(c->md, initial ? 0.0 : 1e30);
    // border set and chain at rest, from the positions at this call's start
    const bool th = thermo && n_steps > 0;
    if (th && (md->thermo_reset || !c->border_valid || c->th_chain != md->thermo_chain ||
               c->th_axes != md->thermo_axes || c->th_border != md->thermo_border)) {
        HIP_TRY(hipMemcpyAsync(c->md + MD_STEP_WORDS, c->h_md + MD_STEP_WORDS, (MD_WORDS - MD_STEP_WORDS) * 8,
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(c->n_border, 0, 4, st));
        k_border_mask<<<sg, 256, 0, st>>>(n, s->x, s->y, s->z, s->h[0], s->h[4], s->h[8], md->thermo_axes,
                                          md->thermo_border, c->border, c->n_border);
        c->border_valid = true;
        c->th_chain = md->thermo_chain;
        c->th_axes = md->thermo_axes;
        c->th_border = md->thermo_border;
    }
    const uint8_t *bd = th ? c->border : nullptr;
    const double mass_conv = s->mass / ACC_EV_U_A;   // 2K (eV) = mass_conv * sum |v|^2
    const double kT = K_B_EV * md->thermo_T;
    auto chain = [&](int phase) {
        k_nhc<<<1, 256, 0, st>>>(c->ke_part, sg, mass_conv, md->thermo_chain, kT, md->thermo_tau, md->dt_max,
                                 md->max_disp, md->dt_min, c->n_border, c->md, c->status, phase);
    };
    // first step length (and first chain half step) from the initial velocities
    k_vmax<<<sg, 256, 0, st>>>(n, s->vx, s->vy, s->vz, bd, c->ke_part, c->md);
    if (th) chain(0);
    else k_dt_update<<<1, 64, 0, st>>>(md->dt_max, md->max_disp, md->dt_min, c->md, c->status, 0);
    // the rebuild counter counts rebuilds inside the chunk only
    HIP_TRY(hipMemsetAsync(c->md + MD_NREB, 0, 8, st));
    // kernel timing: three events per step for the first MAX_TIMED steps
    const int MAX_TIMED = 4096;
    const int n_timed = md->time_kernels ? std::min(n_steps, MAX_TIMED) : 0;
    std::vector<hipEvent_t> ev(3 * (size_t)n_timed);
    auto free_events = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto &e : ev) {
        e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) { free_events(); return NEP_E_HIP; }
    }
    for (int k = 0; k < n_steps; ++k) {
        k_kick_drift<<<sg, 256, 0, st>>>(n, s->x, s->y, s->z, s->vx, s->vy, s->vz, o->fx, o->fy, o->fz, acc,
                                         c->xref, bd, c->md, c->status);
        k_rebuild_flag<<<1, 64, 0, st>>>(half_skin2, c->md, c->flag, c->status);
        k_cand_update<<<1, 64, 0, st>>>(CAND_TRIGGER, c->md, c->flag, c->cflag);
        if ((rc = launch_build(c, s, st, c->flag))) { free_events(); return rc; }
        if ((rc = launch_efv(c, s, o, st, true, k < n_timed ? &ev[3 * (size_t)k] : nullptr, true))) {
            free_events();
            return rc;
        }
        k_kick<<<sg, 256, 0, st>>>(n, s->vx, s->vy, s->vz, o->fx, o->fy, o->fz, acc, bd, c->ke_part, c->md,
                                   c->status);
        if (th) chain(k + 1 < n_steps ? 1 : 2);
        else k_dt_update<<<1, 64, 0, st>>>(md->dt_max, md->max_disp, md->dt_min, c->md, c->status, 1);
    }
    if (th) k_scale_border<<<sg, 256, 0, st>>>(n, s->vx, s->vy, s->vz, c->border, c->md);
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(c->h_md, c->md, MD_WORDS * 8, hipMemcpyDeviceToHost, st) ||
        hipMemcpyAsync(c->h_status, c->status, 8 * 4, hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st) != hipSuccess) {
        free_events();
        return NEP_E_HIP;
    }
    double ms_d = 0.0, ms_f = 0.0;
    for (int k = 0; k < n_timed; ++k) {
        float a = 0.0f, b = 0.0f;
        if (hipEventElapsedTime(&a, ev[3 * (size_t)k], ev[3 * (size_t)k + 1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[3 * (size_t)k + 1], ev[3 * (size_t)k + 2]) != hipSuccess) {
            free_events();
            return NEP_E_HIP;
        }
        ms_d += a;
        ms_f += b;
    }
    free_events();
    if (stats) {
        stats->n_rebuilds = (int64_t)c->h_md[MD_NREB];
        stats->dt_last = c->h_md[MD_DT];
        stats->time = c->h_md[MD_TIME];
        stats->n_border = th ? (int64_t)c->h_md[MD_NBORDER] : 0;
        stats->thermo_energy = th ? c->h_md[MD_ENHC] : 0.0;
        stats->border_temperature =
            stats->n_border > 0 ? c->h_md[MD_TWOK] / (3.0 * (double)stats->n_border * K_B_EV) : 0.0;
        stats->n_timed_steps = n_timed;
        stats->ms_descriptor = n_timed > 0 ? ms_d / n_timed : 0.0;
        stats->ms_force = n_timed > 0 ? ms_f / n_timed : 0.0;
    }
    const int code = c->h_status[ST_ERR];
    if (code != 0) {
        const int32_t zero = 0;
        HIP_TRY(hipMemcpy(c->status + ST_ERR, &zero, 4, hipMemcpyHostToDevice));
    }
    return code;
}


// ---------------------------------------------------------------- defects

// Minimum-label propagation until no label changes (at most d_n rounds:
// every round that changes something lowers some label).
static int ws_cluster(int d_n, const int32_t *sites, double cut2, const BccRef &r, int32_t *label,
                      int32_t *flag_d, int32_t *flag_h, hipStream_t st)
{
    if (d_n == 0) return NEP_OK;
    const int g = (d_n + 255) / 256;
    k_ws_label_init<<<g, 256, 0, st>>>(d_n, label);
    for (int it = 0; it <= d_n; ++it) {
        k_ws_fill<<<1, 64, 0, st>>>(1, flag_d, 0);
        k_ws_label_step<<<g, 256, 0, st>>>(d_n, sites, cut2, r, label, flag_d);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(flag_h, flag_d, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (*flag_h == 0) return NEP_OK;
    }
    return NEP_E_INTERNAL;
}

int nep_wigner_seitz(const nep_system *s, const nep_bcc_ref *ref, int32_t *occ, int32_t *site_of_atom,
                     int32_t cap, int32_t *vac_sites, int32_t *vac_label, int32_t *int_sites, int32_t *int_mult,
                     int32_t *int_label, int32_t *work, nep_defects *out, void *stream)
{
    if (!s || !ref || !occ || !work || !out || !s->x || !s->y || !s->z || !s->h) return NEP_E_ARG;
    if (cap < 0 || (cap > 0 && (!vac_sites || !vac_label || !int_sites || !int_mult || !int_label))) return NEP_E_ARG;
    if (s->cell_start && s->n_cells != 1) return NEP_E_ARG;
    if (s->n_atoms <= 0 || s->n_atoms > (1LL << 30) || !(ref->a > 0.0)) return NEP_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (ref->n[a] <= 0 || ref->n[a] > (1 << 10)) return NEP_E_ARG;
    if (2LL * ref->n[0] * ref->n[1] * ref->n[2] > (1LL << 30)) return NEP_E_ARG;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double want = a == b ? ref->n[a] * ref->a : 0.0;
            if (fabs(s->h[3 * a + b] - want) > 1e-9 * ref->n[a] * ref->a) return NEP_E_ARG;
        }
    hipStream_t st = (hipStream_t)stream;
    BccRef r;
    r.a = ref->a;
    r.inv_a = 1.0 / ref->a;
    for (int a = 0; a < 3; ++a) r.n[a] = ref->n[a];
    const int m = 2 * ref->n[0] * ref->n[1] * ref->n[2];
    const int n = (int)s->n_atoms;
    // work: [0..2] collect counters, [3] bad position (then the propagation
    // flag), [4..5] vacancy cluster count / largest, [6..7] the same for
    // interstitials
    int32_t h[NEP_WS_WORK_INTS];
    k_ws_fill<<<(m + 255) / 256, 256, 0, st>>>(m, occ, 0);
    k_ws_fill<<<1, 64, 0, st>>>(NEP_WS_WORK_INTS, work, 0);
    k_ws_assign<<<(n + 255) / 256, 256, 0, st>>>(n, s->x, s->y, s->z, r, occ, site_of_atom, work + 3);
    k_ws_collect<<<(m + 255) / 256, 256, 0, st>>>(m, occ, cap, vac_label, int_label, work);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, work, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out->n_vacancies = h[0];
    out->n_interstitial_sites = h[1];
    out->n_interstitials = h[2];
    out->n_vacancy_clusters = out->largest_vacancy_cluster = 0;
    out->n_interstitial_clusters = out->largest_interstitial_cluster = 0;
    if (h[3]) return NEP_E_NONFINITE;
    if (h[0] > cap || h[1] > cap) return NEP_E_CAPACITY;
    const int nv = h[0], ni = h[1];
    // sorted lists (the label arrays held the unsorted ones)
    if (nv) k_ws_sort<<<(nv + 255) / 256, 256, 0, st>>>(nv, vac_label, vac_sites, occ, nullptr);
    if (ni) k_ws_sort<<<(ni + 255) / 256, 256, 0, st>>>(ni, int_label, int_sites, occ, int_mult);
    HIP_TRY(hipGetLastError());
    int32_t flag_h = 0;
    const double a2 = ref->a * ref->a * (1.0 + 1e-9);
    int rc = ws_cluster(nv, vac_sites, a2, r, vac_label, work + 3, &flag_h, st);
    if (rc == NEP_OK) rc = ws_cluster(ni, int_sites, 2.0 * a2, r, int_label, work + 3, &flag_h, st);
    if (rc != NEP_OK) return rc;
    if (nv) k_ws_cluster_sizes<<<(nv + 255) / 256, 256, 0, st>>>(nv, vac_label, nullptr, work + 4);
    if (ni) k_ws_cluster_sizes<<<(ni + 255) / 256, 256, 0, st>>>(ni, int_label, int_mult, work + 6);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, work, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out->n_vacancy_clusters = h[4];
    out->largest_vacancy_cluster = h[5];
    out->n_interstitial_clusters = h[6];
    out->largest_interstitial_cluster = h[7];
    return NEP_OK;
}


// ---------------------------------------------------------------- SNES population

static const int POP_FBLK = 256;    // blocks of the force-error reduction per member

int nep_population_reserve(nep_ctx *c, int32_t n_pop)
{
    if (!c || n_pop < 1 || n_pop > NEP_MAX_POPULATION) return NEP_E_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return NEP_E_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return NEP_E_HIP;
    free_population(c);
    const size_t P = (size_t)n_pop, N = (size_t)c->cfg.max_atoms, C = (size_t)c->cfg.max_cells;
    // chunks never span cells and hold at most 4096 atoms
    const int64_t chunks = (int64_t)C + (int64_t)(N / 4096) + 1;
    bool ok = true;
    auto A = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes > 0 ? bytes : 16) != hipSuccess) ok = false;
    };
    if (c->wide) {
        // members evaluated one after another through the staged phases:
        // parameter blocks and the per-member results only
        A((void **)&c->pop_P, P * W_SIZE * sizeof(float));
        A((void **)&c->pop_c64, P * W_C64 * sizeof(double));
        A((void **)&c->pop_F, P * N * 3 * sizeof(float));
        A((void **)&c->pop_E, P * C * sizeof(double));
        A((void **)&c->pop_W, P * C * 9 * sizeof(double));
        A((void **)&c->pop_fpart, P * POP_FBLK * sizeof(double));
        if (!ok) { free_population(c); return NEP_E_HIP; }
        c->pop_cap = n_pop;
        c->pop_chunk_cap = chunks;
        return NEP_OK;
    }
    A((void **)&c->pop_P, P * P_SIZE * sizeof(float));
    A((void **)&c->pop_c64, P * C64N * sizeof(double));
    A((void **)&c->pop_xp, P * N * sizeof(AtomRec));
    A((void **)&c->pop_pg, P * N * c->cfg.max_neigh_ang * sizeof(float4));
    A((void **)&c->pop_fown, P * N * sizeof(float4));
    A((void **)&c->pop_w, P * N * 9 * sizeof(float));
    A((void **)&c->pop_F, P * N * 3 * sizeof(float));
    A((void **)&c->pop_e, P * N * sizeof(double));
    A((void **)&c->pop_E, P * C * sizeof(double));
    A((void **)&c->pop_W, P * C * 9 * sizeof(double));
    A((void **)&c->pop_part, P * (size_t)chunks * 10 * sizeof(double));
    A((void **)&c->pop_fpart, P * POP_FBLK * sizeof(double));
    if (!ok) { free_population(c); return NEP_E_HIP; }
    c->pop_cap = n_pop;
    c->pop_chunk_cap = chunks;
    return NEP_OK;
}

int nep_population_efv(nep_ctx *c, const nep_system *s, int32_t n_pop, const float *theta, double *energy,
                       float *forces, double *virial, const nep_targets *tg, double *loss, void *stream)
{
    if (!c || !theta || n_pop < 1) return NEP_E_ARG;
    if (n_pop > c->pop_cap) return NEP_E_ARG;
    int rc = check_system(c, s, false);
    if (rc) return rc;
    if (!same_system(c, s)) return NEP_E_STATE;
    if (c->n_chunks > c->pop_chunk_cap) return NEP_E_INTERNAL;
    if (loss && (!tg || !tg->energy || !tg->fx || !tg->fy || !tg->fz)) return NEP_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)s->n_atoms;
    const int nc = c->built_cells;
    if (c->wide) {
        // the paper-size model: each member's evaluation in turn, with the
        // context's parameter block swapped for the member's (the launches
        // take the pointers by value); results into the member's rows
        k_w_pop_params<<<n_pop, 256, 0, st>>>(theta, c->params, c->pop_P, c->pop_c64);
        float *F = forces ? forces : c->pop_F;
        double *E = energy ? energy : c->pop_E;
        double *W = virial ? virial : c->pop_W;
        float *const params0 = c->params;
        double *const c640 = c->c64;
        for (int m = 0; m < n_pop && rc == NEP_OK; ++m) {
            c->params = c->pop_P + (size_t)m * W_SIZE;
            c->c64 = c->pop_c64 + (size_t)m * W_C64;
            float *fm = F + 3 * (size_t)m * n;
            nep_efv om = {E + (size_t)m * nc, fm, fm + n, fm + 2 * (size_t)n, W + (size_t)m * nc * 9, nullptr};
            rc = launch_efv(c, s, &om, st, m == 0);
        }
        c->params = params0;
        c->c64 = c640;
        if (rc) return rc;
        if (loss) {
            const int nblk = std::min(POP_FBLK, grid_for(n, 256));
            k_pop_force_err<<<dim3(nblk, n_pop), 256, 0, st>>>(n, F, tg->fx, tg->fy, tg->fz, c->pop_fpart);
            k_pop_loss<<<n_pop, 256, 0, st>>>(nc, n, W_NPARAM, nblk, c->cell_start_d, E, W, tg->energy, tg->virial,
                                              tg->has_virial, c->pop_fpart, theta, tg->lambda_e, tg->lambda_f,
                                              tg->lambda_v, tg->lambda_1, tg->lambda_2, loss);
        }
        HIP_TRY(hipGetLastError());
        return NEP_OK;
    }
    k_sort_positions<<<grid_for(n, 256), 256, 0, st>>>(n, c->perm, s->x, s->y, s->z, c->wrap, c->cell_of, c->cells,
                                                       c->xq, c->status, nullptr,
                                                       c->bin_sorted, c->pc.qsinv, wide_xf(c));
    k_pop_params<<<n_pop, 256, 0, st>>>(theta, c->params, c->pop_P, c->pop_c64);
    const int tiles_d = (n + POP_DESC_BS - 1) / POP_DESC_BS;
    const int grid_d = xcd_grid((int)((int64_t)tiles_d * n_pop));
    const int tiles = (n + 255) / 256;
    const int grid = xcd_grid((int)((int64_t)tiles * n_pop));
    float *F = forces ? forces : c->pop_F;
    double *E = energy ? energy : c->pop_E;
    double *W = virial ? virial : c->pop_W;
    k_pop_descriptor<<<grid_d, POP_DESC_BS, 0, st>>>(c->pc, c->xq, c->pop_xp, c->cell_of, c->cells, c->nl_ang,
                                                     c->nl_rad, c->ncnt, c->pop_P, c->pop_c64, c->pop_pg,
                                                     c->pop_fown, c->pop_w, c->pop_e, c->status, tiles_d, n_pop);
    k_pop_force<<<grid, 256, 0, st>>>(c->pc, c->pop_xp, c->cell_of, c->cells, c->nl_ang, c->nl_rad, c->ncnt, c->rev,
                                      c->pop_pg, c->pop_fown, c->perm, F, c->pop_w, c->status, tiles, n_pop);
    k_pop_reduce_chunks<<<dim3(c->n_chunks, n_pop), 256, 0, st>>>(n, c->n_chunks, c->chunk_begin, c->chunk_end,
                                                                   c->pop_e, c->pop_w, c->pop_part, c->status);
    k_pop_reduce_cells<<<dim3(nc, n_pop), 256, 0, st>>>(nc, c->n_chunks, c->cell_chunk, c->pop_part, E, W,
                                                        c->status);
    if (loss) {
        const int nblk = std::min(POP_FBLK, grid_for(n, 256));
        k_pop_force_err<<<dim3(nblk, n_pop), 256, 0, st>>>(n, F, tg->fx, tg->fy, tg->fz, c->pop_fpart);
        k_pop_loss<<<n_pop, 256, 0, st>>>(nc, n, N_PARAMS, nblk, c->cell_start_d, E, W, tg->energy, tg->virial,
                                          tg->has_virial, c->pop_fpart, theta, tg->lambda_e, tg->lambda_f,
                                          tg->lambda_v, tg->lambda_1, tg->lambda_2, loss);
    }
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

int nep_snes_sample(int32_t n_pop, int32_t n_params, const float *mu, const float *sigma, const float *draws,
                    float *theta, void *stream)
{
    if (n_pop < 1 || n_params < 1 || !mu || !sigma || !draws || !theta) return NEP_E_ARG;
    const int64_t total = (int64_t)n_pop * n_params;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    k_snes_sample<<<grid, 256, 0, (hipStream_t)stream>>>(n_pop, n_params, mu, sigma, draws, theta);
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

int nep_snes_update(int32_t n_pop, int32_t n_params, const double *loss, int32_t loss_stride, const float *draws,
                    float *mu, float *sigma, double eta_mu, double eta_sigma, void *stream)
{
    if (n_pop < 2 || n_pop > NEP_MAX_POPULATION || n_params < 1 || loss_stride < 1 || !loss || !draws || !mu ||
        !sigma)
        return NEP_E_ARG;
    if (!(eta_mu > 0)) eta_mu = 1.0;
    if (!(eta_sigma > 0)) eta_sigma = (3.0 + std::log((double)n_params)) / (5.0 * std::sqrt((double)n_params));
    k_snes_update<<<grid_for(n_params, 256), 256, 0, (hipStream_t)stream>>>(n_pop, n_params, loss, loss_stride,
                                                                             draws, mu, sigma, eta_mu, eta_sigma);
    HIP_TRY(hipGetLastError());
    return NEP_OK;
}

}  // extern "C"
