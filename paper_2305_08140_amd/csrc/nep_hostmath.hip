// Host-compiled copies of the kernels' scalar building blocks, exported for
// the CPU unit tests (the same source as the device code, compiled for x86).
// Not part of the library ABI; built into libnep_hostmath.so.
#include "nep_device.h"

using namespace nep;

extern "C" {

void nep_test_sincos(float y, float *s, float *c) { sincos_halfpi(y, *s, *c); }

void nep_test_cutoff(float r, float rc, float *fc, float *dfc)
{
    const float inv = (float)(1.0 / rc);
    const float lo = (float)(1.0 / rc - (double)inv);
    cutoff(scaled_minus_one(r, inv, lo), inv, *fc, *dfc);
}

void nep_test_cheb(float x, float *T, float *dT) { cheb_d(x, T, dT); }

void nep_test_basis_d(double r, double rc, double *fc, double *T) { basis_d(r, 1.0 / rc, *fc, T); }

void nep_test_sph(float x, float y, float z, float *Y) { sph(x, y, z, Y); }

void nep_test_sph_d(double x, double y, double z, double *Y)
{
    sph_degree_d<1>(x, y, z, Y);
    sph_degree_d<2>(x, y, z, Y + 3);
    sph_degree_d<3>(x, y, z, Y + 8);
    sph_degree_d<4>(x, y, z, Y + 15);
}

void nep_test_sph_grad(float x, float y, float z, const float *Dc, float *v)
{
    sph_grad_contract(x, y, z, Dc, v[0], v[1], v[2]);
}

void nep_test_sph_unnorm(float x, float y, float z, float *Y) { sph_unnorm(SphMono(x, y, z), Y); }

void nep_test_sph_norm(float *K)
{
    for (int lm = 0; lm < NLM; ++lm) K[lm] = sph_norm(lm);
}

void nep_test_sph_unnorm_grad(float x, float y, float z, const float *Dc, float *v)
{
    sph_unnorm_grad_contract(SphMono(x, y, z), Dc, v[0], v[1], v[2]);
}

void nep_test_zbl(double r, double Z, double r1, double r2, double *U, double *dU) { zbl_pair(r, Z, r1, r2, *U, *dU); }

void nep_test_decode(int32_t e, int jbits, int ibits, int ioff, int *out)
{
    decode_entry(e, jbits, ibits, ioff, out[0], out[1], out[2], out[3]);
}

void nep_test_sort32(uint32_t *a) { sort32(a); }

uint32_t nep_test_delta_code(int q, int m0, int m1, int m2)
{
    const int m[3] = {m0, m1, m2};
    return delta_code(q, m);
}

}  // extern "C"
