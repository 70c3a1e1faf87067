/*
 * nep.h - C ABI of the MI355X (gfx950) NEP-ZBL energy / force / virial library.
 *
 * The potential (arXiv 2305.08140, Sec. II.A):
 *   U_i = U_i^NEP({q_nu^i}) + 1/2 sum_{j != i} U_ZBL(r_ij)                 (Eq. 1)
 *   U_ZBL(r) = e^2/(4 pi eps0) Z^2/r phi(r/a) f_c(r)                        (Eq. 2)
 *   phi(x) = 0.32825 e^{-2.54931x} + 0.09219 e^{-0.29182x} + 0.58110 e^{-0.59231x}   (Eq. 3)
 *   a = 0.46848 / (Z_i^0.23 + Z_j^0.23)                                     (Eq. 4)
 *   f_c: Tersoff switch between 1.0 A and 2.0 A (Sec. II.A)
 * U^NEP is a one-hidden-layer tanh network of a descriptor made of Chebyshev
 * radial components (cutoff 6 A) and Legendre angular components l <= 4
 * (cutoff 4 A), as in the NEP framework the paper builds on (Sec. II.A,
 * hyperparameter names in Sec. III.A).  Forces are F = -grad E and the
 * virial is W_ab = -sum_i sum_j (dU_i/dr_ij)_a (r_ij)_b, r_ij = x_j - x_i.
 * Molecular dynamics uses velocity Verlet with the time step chosen so that
 * the fastest atom moves at most a given distance per step (Sec. II.B).
 *
 * Conventions
 *   Units: eV, A, fs, u.  Positions and velocities are FP64, forces FP32,
 *   energy and virial FP64.  All arrays are structure-of-arrays.
 *   Device pointers are HIP device memory owned by the caller; the library
 *   never frees caller memory.  `stream` is a hipStream_t (NULL = default).
 *   Calls are stream-ordered and asynchronous.  Argument errors are returned
 *   immediately.  Errors found on the device (neighbour overflow, overlapping
 *   atoms, non-finite positions, time-step underflow) are latched in the
 *   context; they are returned by nep_status() and by nep_step_verlet(), which
 *   synchronises at the end of its chunk.  Once an error is latched, the
 *   kernels of later calls return without work until nep_status() clears it.
 *   A context may be used from one host thread at a time; calls that overlap
 *   on different streams with the same context race.
 */
#ifndef NEP_H
#define NEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define NEP_OK                 0
#define NEP_E_ARG             -1  /* bad argument (NULL pointer, size out of range, ...) */
#define NEP_E_HIP             -2  /* a HIP runtime call failed */
#define NEP_E_NEIGH_OVERFLOW  -3  /* a neighbour list exceeded its capacity, see nep_required_neighbors */
#define NEP_E_OVERLAP         -4  /* two atoms closer than 1e-3 A */
#define NEP_E_NONFINITE       -5  /* a position or velocity is NaN or infinite */
#define NEP_E_DT_UNDERFLOW    -6  /* adaptive time step fell below nep_md.dt_min */
#define NEP_E_STATE           -7  /* call order: nep_compute_efv before nep_build_neighbors on this system */
#define NEP_E_UNSUPPORTED     -8  /* hyperparameters for which no kernel is compiled */
#define NEP_E_INTERNAL        -9  /* internal consistency check failed (neighbour lists not symmetric),
                                     or an atom far outside its bin of the last build (bin-offset mode) */
#define NEP_E_CAPACITY       -10  /* more defect sites than the caller's arrays hold */

typedef struct nep_ctx nep_ctx;

/* Model hyperparameters (names as in Sec. III.A).  Compiled kernels exist for
 *   the default model: n_rad = 9 (n_max^R = 8), n_ang = 5 (n_max^A = 4),
 *     k_rad = k_ang = 9 (Chebyshev k = 0..8), l_max = 4, n_hidden = 30;
 *   the paper's model size: n_rad = k_rad = 16 (n_max^R = 15), n_ang = k_ang
 *     = 11 (n_max^A = 10), l_max = 4, n_hidden = 100.  It supports every call.
 * Other values give NEP_E_UNSUPPORTED. */
typedef struct {
    int32_t n_rad;      /* radial descriptor components */
    int32_t n_ang;      /* radial functions of the angular components */
    int32_t k_rad;      /* Chebyshev basis size, radial */
    int32_t k_ang;      /* Chebyshev basis size, angular */
    int32_t l_max;      /* Legendre orders 1..l_max */
    int32_t n_hidden;   /* tanh neurons */
    int32_t Z;          /* nuclear charge of the (single) species */
    int32_t pad_;
    double rc_rad;      /* radial cutoff, A (6) */
    double rc_ang;      /* angular cutoff, A (4) */
    double zbl_r1;      /* ZBL Tersoff switch inner cutoff, A (1) */
    double zbl_r2;      /* ZBL Tersoff switch outer cutoff, A (2) */
} nep_hparams;

/* Model parameters, FP32, row-major.  D = n_rad + n_ang * l_max.
 * Descriptor order: nu = n for radial; nu = n_rad + n_ang*(l-1) + n for angular.
 * U^NEP = sum_mu w1[mu] tanh(sum_nu w0[mu][nu] q_scale[nu] q_nu - b0[mu]) - b1. */
typedef struct {
    const float *c_rad;    /* [n_rad][k_rad] radial expansion coefficients */
    const float *c_ang;    /* [n_ang][k_ang] angular radial-function coefficients */
    const float *q_scale;  /* [D] descriptor scale */
    const float *w0;       /* [n_hidden][D] */
    const float *b0;       /* [n_hidden] */
    const float *w1;       /* [n_hidden] */
    float b1;
    int32_t pad_;
} nep_weights;

/* Capacities, fixed at creation. */
typedef struct {
    int64_t max_atoms;      /* total atoms over all cells; at most 2^26 */
    int32_t max_cells;      /* cells per batch */
    int32_t max_neigh_ang;  /* per-atom capacity of the list r < rc_ang + skin (<= 255) */
    int32_t max_neigh_rad;  /* per-atom capacity of the list rc_ang + skin <= r < rc_rad + skin (<= 255) */
    int32_t pad_;
    double skin;            /* neighbour-list skin, A; lists are rebuilt when an atom moved > skin/2 */
} nep_config;

/* A batch of independent cells (one cell for a bulk MD system). */
typedef struct {
    int64_t n_atoms;
    int32_t n_cells;
    int32_t pbc[3];              /* periodic along lattice vector a (1) or open (0) */
    const int64_t *cell_start;   /* HOST [n_cells + 1]; NULL means one cell of n_atoms */
    const double *h;             /* HOST [n_cells][9]; rows are lattice vectors, x = s h */
    double *x, *y, *z;           /* DEVICE [n_atoms] positions, A */
    double *vx, *vy, *vz;        /* DEVICE [n_atoms] velocities, A/fs (nep_step_verlet only) */
    double mass;                 /* atomic mass, u */
} nep_system;

/* Outputs (DEVICE, caller-owned, written by nep_compute_efv / nep_step_verlet). */
typedef struct {
    double *energy;       /* [n_cells] total energy per cell, eV */
    float *fx, *fy, *fz;  /* [n_atoms] forces, eV/A, in the caller's atom order */
    double *virial;       /* [n_cells][9] W_ab row-major, eV; may be NULL */
    float *energy_atom;   /* [n_atoms] site energies U_i, eV; may be NULL */
} nep_efv;

/* Molecular-dynamics controls.
 *
 * Border thermostat (Sec. II.B: the cascade runs hold a layer of about 3 a0
 * at the periodic faces at the target temperature with a Nose-Hoover chain,
 * Martyna, Klein and Tuckerman 1992).  With thermo_chain = M > 0, the atoms
 * whose wrapped coordinate along an axis selected by thermo_axes lies within
 * thermo_border of a face of the (orthorhombic, single) cell are coupled to a
 * chain of M thermostats at thermo_T with masses Q_1 = N_f k T tau^2,
 * Q_j = k T tau^2 (N_f = 3 x border atoms).  Each step is: half a chain step
 * (the border velocities are scaled), the velocity-Verlet step, half a chain
 * step.  The border set and the chain state persist between calls on the same
 * system; they are (re)initialised (chain at rest) on the first thermostatted
 * call for a system, when thermo_reset is nonzero, or when thermo_chain,
 * thermo_axes or thermo_border change.  thermo_T and thermo_tau may change
 * between calls. */
typedef struct {
    double dt_max;        /* fs, upper limit of the step (Sec. II.B: 1 fs) */
    double max_disp;      /* A, the fastest atom moves at most this far per step; 0 = fixed dt_max */
    double dt_min;        /* fs, a step below this latches NEP_E_DT_UNDERFLOW */
    int32_t forces_valid; /* nonzero: out->f* already hold the forces of the current positions */
    int32_t thermo_chain; /* chain length M of the border thermostat, 0 = none, at most 8 */
    double thermo_T;      /* K, target temperature (> 0 when thermo_chain > 0) */
    double thermo_tau;    /* fs, chain time constant (> 0) */
    double thermo_border; /* A, layer thickness at each selected face (>= 0; 0 selects no atom) */
    int32_t thermo_axes;  /* bit a (0..2) set: the two faces normal to lattice vector a; 1..7 */
    int32_t thermo_reset; /* nonzero: rebuild the border set and put the chain at rest first */
    int32_t time_kernels; /* nonzero: HIP events on `stream` around the descriptor and force
                             kernels of each step (the first 4096 steps of the call); the mean
                             durations are returned in nep_md_stats */
    int32_t pad_;
} nep_md;

typedef struct {
    int64_t n_rebuilds;   /* neighbour rebuilds during the chunk */
    double dt_last;       /* fs, the step length for a following step */
    double time;          /* fs, simulated time of the chunk */
    int64_t n_border;     /* atoms in the thermostatted layer (0 without thermostat) */
    double thermo_energy; /* eV, chain energy sum_j Q_j v_j^2 / 2 + N_f kT xi_1 + kT sum_{j>1} xi_j;
                             total energy + kinetic energy + this is conserved */
    double border_temperature; /* K, 2 K_border / (N_f k_B) of the final velocities */
    double ms_descriptor;  /* with md->time_kernels: mean ms per step of the descriptor kernel(s) */
    double ms_force;       /* ... and of the force kernel */
    int64_t n_timed_steps; /* steps those means cover (0 without time_kernels) */
} nep_md_stats;

/* Create a context for the given hyperparameters and capacities; weights are
 * set with nep_set_weights.  Allocates device memory on the current device.
 * Returns NEP_OK, NEP_E_ARG, NEP_E_UNSUPPORTED or NEP_E_HIP; *out is NULL on error. */
int nep_create(const nep_hparams *hp, const nep_config *cfg, nep_ctx **out);

/* Free the context and its device memory (synchronises the device). NULL is allowed. */
void nep_destroy(nep_ctx *ctx);

/* Copy the model parameters into the context.  weights_on_device = 0: the
 * pointers are host memory (copied synchronously); 1: device memory (copied
 * asynchronously on `stream`).  Returns NEP_OK, NEP_E_ARG or NEP_E_HIP. */
int nep_set_weights(nep_ctx *ctx, const nep_weights *w, int32_t weights_on_device, void *stream);

/* Build the cell list and the neighbour lists of `sys`: the pair sets that
 * the sums of Eq. 1 run over, every periodic image of every atom j != i (and
 * the atom's own images) within the radial cutoff rc_rad (6 A) for the radial
 * descriptor and within rc_ang (4 A) for the angular one (Sec. III.A, the
 * cutoffs of the model), widened by the skin so the lists stay valid until an
 * atom has moved skin/2.  Positions (DEVICE, caller order) may lie anywhere;
 * they are wrapped into the cell internally, and open axes (pbc = 0) take no
 * images.  The lists, the cell list and the sorted atom order are stored in
 * the context (memory allocated by nep_create; nothing is allocated here).
 * Overflow of a list capacity latches NEP_E_NEIGH_OVERFLOW (the lengths needed
 * are returned by nep_required_neighbors) and non-finite positions latch
 * NEP_E_NONFINITE; after such a build the lists stay unusable, and evaluations
 * on them latch NEP_E_STATE until a build succeeds.
 * Bin-offset mode: a system of one cell, periodic along all three axes, at
 * least three bins of rc_rad + skin wide along each, and at most 2^23 atoms,
 * stores in each list entry the offset of the neighbour's bin from the
 * atom's own instead of the periodic image, and the force evaluation (and
 * every walk of the paper-size model) reads positions as fixed-point offsets
 * (units 2^-k A, k as large as the bin size allows) from the corner of the
 * atom's bin at this list build.  The results are those of the general
 * layout up to that rounding (~4e-9 A).  The range of
 * the offsets covers the bin plus at least skin + 1 A on every side; an atom
 * beyond it (possible only on lists used long after they went stale)
 * latches NEP_E_INTERNAL at the next evaluation.
 * Returns NEP_OK, NEP_E_ARG or NEP_E_HIP. */
int nep_build_neighbors(nep_ctx *ctx, const nep_system *sys, void *stream);

/* The lists of nep_build_neighbors kept while they are valid: for the system
 * the lists were built for (same atom count, cells and cell sizes), the
 * device compares the positions with those of the last build and rebuilds
 * only if an atom has moved more than skin/2 (the skin criterion of the
 * paper's MD, Sec. II.B) or the lists are unusable; any other system is
 * built in full.  The decision stays on the device (no synchronisation), so
 * repeated evaluations of slowly changing configurations (a differentiable
 * training loop, a relaxation) pay for a build only when one is due.  Same
 * arguments, errors and allocation behaviour as nep_build_neighbors. */
int nep_update_neighbors(nep_ctx *ctx, const nep_system *sys, void *stream);

/* Energy, forces and virial of `sys` at its current positions (Eq. 1: the
 * network site energies of the radial and angular descriptors plus half of
 * the ZBL pair energy of Eqs. 2-4 for every pair closer than the outer
 * switch radius; forces F_i = -dE/dx_i; virial W_ab = -sum_i sum_j
 * (dU_i/dr_ij)_a (r_ij)_b), using the neighbour lists of the last
 * nep_build_neighbors on the same system (atoms may have moved by less than
 * skin/2 since).  Inputs: the DEVICE positions of `sys`; outputs: the DEVICE
 * arrays of `out` (caller-owned; energy and virial per cell, forces and site
 * energies in the caller's atom order).  Work buffers are the context's.
 * Asynchronous on `stream`; device errors (overlapping atoms, unusable
 * lists) are latched as described above.  Returns NEP_OK, NEP_E_ARG,
 * NEP_E_STATE (no lists built for this system) or NEP_E_HIP. */
int nep_compute_efv(nep_ctx *ctx, const nep_system *sys, nep_efv *out, void *stream);

/* Advance `sys` by n_steps velocity-Verlet steps (x, v updated in place), with
 * the adaptive step of `md` (Sec. II.B), rebuilding the neighbour lists on the
 * device when an atom has moved more than skin/2 since the last build, and
 * with the border thermostat when md->thermo_chain > 0 (one cell only, and
 * its h must be diagonal, else NEP_E_UNSUPPORTED).  On return `out` holds
 * energy, forces and virial of the final positions.  Synchronises `stream` at
 * the end; returns NEP_OK or the first latched device error, or NEP_E_ARG /
 * NEP_E_UNSUPPORTED / NEP_E_HIP.  `stats` may be NULL. */
int nep_step_verlet(nep_ctx *ctx, nep_system *sys, const nep_md *md, int32_t n_steps,
                    nep_efv *out, nep_md_stats *stats, void *stream);

/* Synchronise `stream`, return the latched device error (NEP_OK if none) and clear it. */
int nep_status(nep_ctx *ctx, void *stream);

/* After NEP_E_NEIGH_OVERFLOW: the per-atom list lengths the last build needed. */
int nep_required_neighbors(nep_ctx *ctx, int32_t *ang, int32_t *rad);

/* Mean neighbour counts inside the cutoffs at the last nep_compute_efv
 * (synchronises `stream`); used for algorithmic-flop accounting. */
int nep_mean_neighbors(nep_ctx *ctx, void *stream, double *mean_rad, double *mean_ang);

/* Same evaluation as nep_compute_efv, replayed from a HIP graph: the first
 * call (and any call whose system size, position or output pointers differ
 * from the captured ones) captures the launch sequence on `stream` into a
 * graph; later calls launch the graph.  `stream` must not be the NULL stream
 * (capture is not allowed there).  Positions may change between calls by less
 * than skin/2 as for nep_compute_efv.  Returns NEP_OK, NEP_E_ARG,
 * NEP_E_STATE or NEP_E_HIP. */
int nep_compute_efv_graph(nep_ctx *ctx, const nep_system *sys, nep_efv *out, void *stream);

/* Autotune the launch shapes (threads per block 64/128/256, one block per
 * atom tile or a persistent grid striding over tiles) of the descriptor and
 * force kernels for `sys`: each candidate is timed `reps` times with HIP
 * events on `stream`; the fastest pair is kept for this system size bucket
 * (floor(log2 n_atoms)) and used by later evaluations in that bucket.
 * shape_out (host int32[2], may be NULL) receives the chosen shape indices
 * (0..2: 64/128/256 threads, one block per tile; 3..5: the same, persistent;
 * the paper-size model's phase kernels come in shapes 0..2 only, and its
 * matrix-core hidden layer keeps its own persistent grid).  Synchronises
 * `stream`.  Same preconditions as nep_compute_efv. */
int nep_autotune(nep_ctx *ctx, const nep_system *sys, nep_efv *out, int32_t reps, int32_t *shape_out,
                 void *stream);

/* Precision and unit of the network's hidden layer in later evaluations:
 *   0 (default) FP32 on the vector ALUs;
 *   1 BF16 inputs on the matrix cores (v_mfma_f32_32x32x16_bf16) with FP32
 *     accumulation, for the forward z = w0 s q and the backward dU/dq;
 *   2 FP32 inputs on the matrix cores (v_mfma_f32_32x32x2_f32), FP32
 *     accumulation: the precision of mode 0 in another summation order.
 * Descriptors, forces and reductions are unaffected; both model sizes take
 * every mode.  Returns NEP_OK or NEP_E_ARG. */
int nep_set_precision(nep_ctx *ctx, int32_t mode);

/* Number of trainable model parameters, theta = (c_rad, c_ang, w0, b0, w1, b1)
 * flattened row-major in that order (1057 for the compiled model). */
int nep_num_params(const nep_ctx *ctx);

/* Backward pass of L = sum_c gE[c] E_c at the positions of the last
 * nep_compute_efv on `sys`, whose outputs `out` must still hold that call's
 * forces and virial (same stream).  All pointers are DEVICE FP64 arrays:
 *   gE          [n_cells]        upstream gradient (input)
 *   grad_params [nep_num_params] dL/dtheta, by the chain rule through the
 *               network and the descriptor coefficients
 *   grad_x/y/z  [n_atoms]        dL/dx_i = -gE[c(i)] F_i (caller order); may be NULL
 *   grad_h      [n_cells][9]     dL/dh at fixed Cartesian positions,
 *               gE[c] h^-T (sum_i x_i (x) F_i - W^T); may be NULL
 * The forces and virial follow from Eq. 1; the parameter gradient is what a
 * gradient-based fit of the model would use (the paper trains by a
 * gradient-free evolution strategy, Sec. III.A).  grad_params is
 * deterministic: FP32 sums over 64-atom tiles, FP64 partials per block (at
 * most 1024 blocks), the partials summed in a fixed tree.  The first call,
 * or a call on more atoms than any before, allocates those partials in the
 * context (min(ceil(n_atoms / 64), 1024) x nep_num_params doubles, at most
 * 8.7 MB for the default model, 53.9 MB for the paper-size one); they are
 * freed by nep_destroy.  For the paper-size model the call first recomputes
 * the staged descriptor sums of the current positions (as nep_compute_efv
 * does before its force kernel).  Returns NEP_OK, NEP_E_ARG, NEP_E_STATE or
 * NEP_E_HIP; device errors are latched as for nep_compute_efv. */
int nep_backward(nep_ctx *ctx, const nep_system *sys, const nep_efv *out, const double *gE,
                 double *grad_params, double *grad_x, double *grad_y, double *grad_z, double *grad_h,
                 void *stream);

/* nep_backward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, preconditions, results (bit for bit) and errors as
 * nep_backward, and it calls no allocating routine.  The block partials live
 * in one file-scope device array per GPU instead of the context: 1024 rows of
 * 6,578 doubles (53.9 MB; the paper-size model's parameter count, the larger
 * one), the most any launch uses, so every system a context of either model
 * accepts fits (NEP_E_CAPACITY would report a launch wider than the array).  The array's address on a GPU is resolved by nep_create with
 * that GPU current and held until the process ends.  All calls on one GPU
 * share the array, which keeps the last call's partials (each call zeroes
 * the rows it uses before adding to them): two calls that overlap in time on
 * the same GPU, on different streams or from different threads, race and
 * give wrong gradients; serialise them. */
int nep_backward_noalloc(nep_ctx *ctx, const nep_system *sys, const nep_efv *out, const double *gE,
                         double *grad_params, double *grad_x, double *grad_y, double *grad_z,
                         double *grad_h, void *stream);

/* Measurement support: run the evaluation path of nep_compute_efv `reps`
 * times, each kernel bracketed by HIP events recorded on `stream`, and return
 * the mean duration per launch in milliseconds:
 *   ms[0] position refresh, ms[1] descriptor + network kernel,
 *   ms[2] force + virial kernel, ms[3] energy / virial reductions.
 * Synchronises `stream`.  Same preconditions as nep_compute_efv. */
int nep_time_efv(nep_ctx *ctx, const nep_system *sys, nep_efv *out, int32_t reps, double *ms, void *stream);

/* ---- defect analysis -------------------------------------------------- */

/* Reference lattice of the Wigner-Seitz analysis: perfect bcc, lattice
 * constant a, n[0] x n[1] x n[2] conventional cells filling the periodic box
 * diag(n[0] a, n[1] a, n[2] a).  Site ids: 2 ((k n1 + j) n0 + i) + b with
 * b = 0 for the corner (i, j, k) a and b = 1 for the body centre
 * (i + 1/2, j + 1/2, k + 1/2) a. */
typedef struct {
    double a;
    int32_t n[3];
    int32_t pad_;
} nep_bcc_ref;

typedef struct {
    int64_t n_vacancies;             /* sites holding no atom */
    int64_t n_interstitial_sites;    /* sites holding more than one atom */
    int64_t n_interstitials;         /* atoms beyond one per site */
    int32_t n_vacancy_clusters, largest_vacancy_cluster;           /* sizes in vacancies */
    int32_t n_interstitial_clusters, largest_interstitial_cluster; /* sizes in interstitial atoms */
} nep_defects;

#define NEP_WS_WORK_INTS 8

/* Wigner-Seitz defect analysis (the paper's identification of vacancies and
 * interstitials and their clustering, Methods): every atom is assigned to
 * the nearest reference site; a site with no atom is a vacancy, a site with
 * k > 1 atoms holds k - 1 interstitials.  Vacancy sites within the
 * second-neighbour distance a of each other, and interstitial sites within
 * the third-neighbour distance a sqrt(2), form clusters (connected
 * components, minimum-image distances).
 *   sys           one periodic cell (cell_start NULL or one cell) whose h is
 *                 diag(n a) to 1e-9 relative; positions DEVICE, any image
 *   occupancy     DEVICE int32[2 n0 n1 n2], written (atoms per site)
 *   site_of_atom  DEVICE int32[n_atoms] or NULL, written (site of every atom)
 *   capacity      length of each of the five arrays below
 *   vacancy_sites, interstitial_sites   DEVICE int32[capacity], written,
 *                 ascending site ids; interstitial_mult: atoms beyond one
 *   vacancy_cluster, interstitial_cluster  DEVICE int32[capacity], written:
 *                 cluster label of each listed site (index of the first
 *                 site of its cluster in the list)
 *   work          DEVICE int32[NEP_WS_WORK_INTS], scratch
 *   out           HOST, written
 * Exact ties between two sites go to the corner site.  Synchronises
 * `stream`.  Returns NEP_OK, NEP_E_ARG, NEP_E_NONFINITE (a position is not
 * finite or is beyond 1e8 a), NEP_E_CAPACITY (more vacancy or interstitial
 * sites than capacity; out holds the counts) or NEP_E_HIP. */
int nep_wigner_seitz(const nep_system *sys, const nep_bcc_ref *ref, int32_t *occupancy, int32_t *site_of_atom,
                     int32_t capacity, int32_t *vacancy_sites, int32_t *vacancy_cluster,
                     int32_t *interstitial_sites, int32_t *interstitial_mult, int32_t *interstitial_cluster,
                     int32_t *work, nep_defects *out, void *stream);

/* Static description of an error code. */
const char *nep_strerror(int code);

/* ---- SNES population evaluation --------------------------------------- */

/* The paper trains its model with the separable natural evolution strategy
 * (SNES, Schaul et al. 2011) with a population of 50, on a loss with weights
 * lambda_e = lambda_f = 1, lambda_v = 0.1, lambda_1 = lambda_2 = 0.05
 * (Sec. III.A; the loss itself is the NEP one the paper cites):
 *   L = le RMSE(E/N) + lf RMSE(F components) + lv RMSE(W/N, six components,
 *       cells with a virial target) + l1 mean|theta| + l2 sqrt(mean theta^2).
 * Parameter vectors theta use the layout of nep_backward's grad_params:
 * (c_rad [n_rad][k_rad], c_ang [n_ang][k_ang], w0 [n_hidden][D], b0, w1, b1),
 * nep_num_params() floats; the descriptor scale q_scale is not trained and is
 * taken from the weights last set with nep_set_weights. */

#define NEP_MAX_POPULATION 1024
#define NEP_LOSS_TERMS 6   /* total, rmse_e, rmse_f, rmse_v, mean|theta|, rms theta */

typedef struct {
    const double *energy;        /* DEVICE [n_cells] target energies, eV */
    const float *fx, *fy, *fz;   /* DEVICE [n_atoms] target forces, eV/A, caller order */
    const double *virial;        /* DEVICE [n_cells][9] target virials, eV; NULL: no virial term */
    const uint8_t *has_virial;   /* DEVICE [n_cells], nonzero where the cell has a virial target;
                                    NULL: every cell (when virial is given) */
    double lambda_e, lambda_f, lambda_v, lambda_1, lambda_2;
} nep_targets;

/* Allocate the per-member evaluation buffers of up to n_pop (1..1024)
 * members at the context's capacity (about 0.9 KB per atom and member with
 * max_neigh_ang = 48; for the paper-size model, whose members are evaluated
 * one after another, the parameter blocks and 12 bytes per atom and member),
 * replacing earlier ones.  Synchronises the device.  Returns NEP_OK,
 * NEP_E_ARG or NEP_E_HIP. */
int nep_population_reserve(nep_ctx *ctx, int32_t n_pop);

/* Energies, forces and virials of the batch `sys` for n_pop parameter
 * vectors at once (one launch over members x atom tiles; the paper-size
 * model runs its staged evaluation once per member, with the same results
 * as nep_compute_efv under that member's parameters), and, with targets,
 * each member's loss terms.  Same preconditions as nep_compute_efv (lists
 * built for `sys`); n_pop <= the reserved population.
 *   theta   DEVICE float [n_pop][nep_num_params()]
 *   energy  DEVICE double [n_pop][n_cells] or NULL
 *   forces  DEVICE float [n_pop][3][n_atoms] (fx, fy, fz rows, caller order) or NULL
 *   virial  DEVICE double [n_pop][n_cells][9] or NULL
 *   tg      targets (required with loss), read on the device
 *   loss    DEVICE double [n_pop][NEP_LOSS_TERMS] or NULL
 * Asynchronous on `stream`.  Returns NEP_OK, NEP_E_ARG, NEP_E_STATE,
 * NEP_E_UNSUPPORTED or NEP_E_HIP; device errors latch as for nep_compute_efv. */
int nep_population_efv(nep_ctx *ctx, const nep_system *sys, int32_t n_pop, const float *theta, double *energy,
                       float *forces, double *virial, const nep_targets *tg, double *loss, void *stream);

/* SNES sampling: theta[k][p] = mu[p] + sigma[p] draws[k][p] (all DEVICE float;
 * draws are the caller's standard-normal numbers).  Asynchronous. */
int nep_snes_sample(int32_t n_pop, int32_t n_params, const float *mu, const float *sigma, const float *draws,
                    float *theta, void *stream);

/* SNES update from the members' losses (DEVICE double, member k's loss at
 * loss[k loss_stride]; lower is better, NaN is worst, ties keep the member
 * order): rank-based utilities u (best first, summing to zero),
 * mu += eta_mu sigma sum_k u_k s_k, sigma *= exp(eta_sigma / 2 sum_k u_k (s_k^2 - 1)),
 * in place on DEVICE float mu, sigma [n_params].  eta_mu <= 0 selects 1,
 * eta_sigma <= 0 selects (3 + ln n_params) / (5 sqrt n_params).
 * 2 <= n_pop <= 1024.  Asynchronous. */
int nep_snes_update(int32_t n_pop, int32_t n_params, const double *loss, int32_t loss_stride, const float *draws,
                    float *mu, float *sigma, double eta_mu, double eta_sigma, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NEP_H */
