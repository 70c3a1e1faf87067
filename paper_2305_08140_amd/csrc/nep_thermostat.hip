// Nose-Hoover chain on the atoms near the box faces (Sec. II.B: the cascade
// runs keep a layer of about 3 a0 at every periodic face at the target
// temperature).  The chain follows Martyna, Klein and Tuckerman (1992) in the
// usual Trotter factorisation: half a step of the chain, the velocity-Verlet
// step, half a step of the chain.  Masses Q_1 = N_f kT tau^2 and
// Q_j = kT tau^2 (j > 1), N_f = 3 x (border atoms).
//
// Device side: the border set is one byte per atom in caller order; the kick
// kernels reduce the border |v|^2 per block (k_kick / k_vmax write block
// partials); k_nhc sums them in a fixed order and advances the chain, and the
// scaling of the border velocities is folded into the next k_kick_drift
// (md[MD_SCALE]), or applied by k_scale_border at the end of a call.
#include <hip/hip_runtime.h>

#include "nep_device.h"

namespace nep {

// Wrapped coordinate within `t` of a face of [0, L): the wrap is fmod (exact)
// plus L for negative remainders.
__device__ inline bool near_face(double x, double L, double t)
{
    double s = fmod(x, L);
    if (s < 0.0) s += L;
    return s < t || s >= L - t;
}

// Border set of an orthorhombic cell with edges L (axes: bit a selects the
// two faces normal to axis a); counts the set into *count.
__global__ __launch_bounds__(256) void k_border_mask(int n, const double *__restrict__ x,
                                                     const double *__restrict__ y, const double *__restrict__ z,
                                                     double Lx, double Ly, double Lz, int axes, double thick,
                                                     uint8_t *__restrict__ border, int32_t *__restrict__ count)
{
    int local = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bool b = false;
        if (axes & 1) b = b || near_face(x[i], Lx, thick);
        if (axes & 2) b = b || near_face(y[i], Ly, thick);
        if (axes & 4) b = b || near_face(z[i], Lz, thick);
        border[i] = (uint8_t)b;
        local += (int)b;
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count, local);
}

// v *= md[MD_SCALE] for the border atoms.
__global__ __launch_bounds__(256) void k_scale_border(int n, double *__restrict__ vx, double *__restrict__ vy,
                                                      double *__restrict__ vz, const uint8_t *__restrict__ border,
                                                      const double *__restrict__ md)
{
    const double s = md[MD_SCALE];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (border[i]) { vx[i] *= s; vy[i] *= s; vz[i] *= s; }
}

struct Chain {
    double *xi, *v;
    int M;
    double nf_kT, kT, Q1, Qj;

    __device__ double G(int j, double twoK) const
    {
        if (j == 0) return (twoK - nf_kT) / Q1;
        return ((j == 1 ? Q1 : Qj) * (v[j - 1] * v[j - 1]) - kT) / Qj;
    }

    // Advance the chain by dt/2 driven by the border kinetic energy twoK/2;
    // returns the factor for the border velocities (and scales twoK by its square).
    __device__ double half_step(double &twoK, double dt)
    {
        const double d4 = dt / 4.0, d8 = dt / 8.0;
        v[M - 1] += G(M - 1, twoK) * d4;
        for (int j = M - 2; j >= 0; --j) {
            v[j] *= exp(-v[j + 1] * d8);
            v[j] += G(j, twoK) * d4;
            v[j] *= exp(-v[j + 1] * d8);
        }
        const double s = exp(-v[0] * dt / 2.0);
        twoK *= s * s;
        for (int j = 0; j < M; ++j) xi[j] += v[j] * dt / 2.0;
        for (int j = 0; j < M - 1; ++j) {
            v[j] *= exp(-v[j + 1] * d8);
            v[j] += G(j, twoK) * d4;
            v[j] *= exp(-v[j + 1] * d8);
        }
        v[M - 1] += G(M - 1, twoK) * d4;
        return s;
    }

    __device__ double energy() const
    {
        double e = 0.0;
        for (int j = 0; j < M; ++j) e += 0.5 * (j == 0 ? Q1 : Qj) * v[j] * v[j];
        e += nf_kT * xi[0];
        for (int j = 1; j < M; ++j) e += kT * xi[j];
        return e;
    }
};

__device__ inline double next_dt(double vmax2, double dt_max, double max_disp, double dt_min, int32_t *status)
{
    const double vmax = sqrt(vmax2);
    double dt = dt_max;
    if (max_disp > 0.0 && vmax > 0.0) dt = fmin(dt_max, max_disp / vmax);
    if (!(dt >= dt_min)) latch_error(status, -6);
    return dt;
}

// One block of 256 threads.  Sums the nparts border partials of |v|^2 in a
// fixed order, then (thread 0):
//   phase 0 (start of a call): step length from the current velocities,
//     first chain half step of the first step;
//   phase 1 (end of a step with another to follow): second chain half step
//     of this step, the next step length from the velocities after it, the
//     first chain half step of the next step;
//   phase 2 (end of the last step of a call): second chain half step only
//     (the step length for a next step is still recorded).
// md[MD_SCALE] receives the product of the factors not yet applied to the
// border velocities.  A chain with no border atoms leaves velocities alone.
__global__ __launch_bounds__(256) void k_nhc(const double *__restrict__ ke_part, int nparts, double mass_conv,
                                             int M, double kT, double tau, double dt_max, double max_disp,
                                             double dt_min, const int32_t *__restrict__ count,
                                             double *__restrict__ md, int32_t *__restrict__ status, int phase)
{
    __shared__ double sh[256];
    double t = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) t += ke_part[k];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double twoK = sh[0] * mass_conv;
    const double nf = 3.0 * (double)(*count);
    Chain ch{md + MD_XI, md + MD_VXI, M, nf * kT, kT, nf * kT * tau * tau, kT * tau * tau};
    const bool on = nf > 0.0 && status[ST_ERR] == 0;
    const double vmax2 = md[MD_VMAX2], vmax2_b = md[MD_VMAX2B];
    double scale = 1.0;
    if (phase == 0) {
        const double dt = next_dt(fmax(vmax2, vmax2_b), dt_max, max_disp, dt_min, status);
        if (on) scale = ch.half_step(twoK, dt);
        md[MD_DT] = dt;
    } else {
        const double dt = md[MD_DT];
        md[MD_TIME] += dt;
        double s2 = 1.0;
        if (on) s2 = ch.half_step(twoK, dt);
        const double dt_next = next_dt(fmax(vmax2, s2 * s2 * vmax2_b), dt_max, max_disp, dt_min, status);
        scale = s2;
        if (phase == 1 && on) scale *= ch.half_step(twoK, dt_next);
        md[MD_DT] = dt_next;
    }
    md[MD_SCALE] = scale;
    md[MD_TWOK] = twoK;
    md[MD_ENHC] = nf > 0.0 ? ch.energy() : 0.0;
    md[MD_NBORDER] = (double)(*count);
    md[MD_VMAX2] = 0.0;
    md[MD_VMAX2B] = 0.0;
}

}  // namespace nep
