"""The kernels' scalar building blocks, compiled for the host from the same
source, against numpy / scipy and finite differences (CPU only)."""
import ctypes as C
import math
import os

import numpy as np
import pytest
import scipy.special as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2305_08140_amd", "libnep_hostmath.so")

F = C.c_float
FP = C.POINTER(C.c_float)
DP = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("libnep_hostmath.so not built")
    lib = C.CDLL(LIB)
    lib.nep_test_sincos.argtypes = [F, FP, FP]
    lib.nep_test_cutoff.argtypes = [F, F, FP, FP]
    lib.nep_test_cheb.argtypes = [F, FP, FP]
    lib.nep_test_basis_d.argtypes = [C.c_double, C.c_double, DP, DP]
    lib.nep_test_sph.argtypes = [F, F, F, FP]
    lib.nep_test_sph_d.argtypes = [C.c_double, C.c_double, C.c_double, DP]
    lib.nep_test_sph_grad.argtypes = [F, F, F, FP, FP]
    lib.nep_test_sph_unnorm.argtypes = [F, F, F, FP]
    lib.nep_test_sph_norm.argtypes = [FP]
    lib.nep_test_sph_unnorm_grad.argtypes = [F, F, F, FP, FP]
    lib.nep_test_zbl.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, DP, DP]
    lib.nep_test_decode.argtypes = [C.c_int32, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
    lib.nep_test_sort32.argtypes = [C.POINTER(C.c_uint32)]
    lib.nep_test_delta_code.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    lib.nep_test_delta_code.restype = C.c_uint32
    return lib


def _f32(n):
    return np.zeros(n, dtype=np.float32)


def _fp(a):
    return a.ctypes.data_as(FP)


def test_sincos_series(L):
    s, c = F(), F()
    for y in np.linspace(-math.pi / 2, math.pi / 2, 201):
        L.nep_test_sincos(y, C.byref(s), C.byref(c))
        assert abs(s.value - math.sin(y)) < 1.5e-7
        assert abs(c.value - math.cos(y)) < 1.5e-7


def test_cutoff_and_derivative(L):
    fc, dfc = F(), F()
    for rc in (4.0, 6.0):
        for r in np.linspace(0.05, rc - 1e-4, 300):
            L.nep_test_cutoff(r, rc, C.byref(fc), C.byref(dfc))
            assert abs(fc.value - 0.5 * (1 + math.cos(math.pi * r / rc))) < 1.5e-7
            assert abs(dfc.value + 0.5 * math.pi / rc * math.sin(math.pi * r / rc)) < 3e-7
        L.nep_test_cutoff(rc * (1 - 1e-6), rc, C.byref(fc), C.byref(dfc))
        assert abs(fc.value) < 1e-7


def test_double_precision_basis(L):
    fc = C.c_double()
    T = np.zeros(9)
    for rc in (4.0, 6.0):
        for r in np.linspace(0.05, rc - 1e-9, 300):
            L.nep_test_basis_d(r, rc, C.byref(fc), T.ctypes.data_as(DP))
            assert abs(fc.value - 0.5 * (1 + math.cos(math.pi * r / rc))) < 1e-13
            x = 2 * (r / rc - 1) ** 2 - 1
            assert np.allclose(T, np.cos(np.arange(9) * math.acos(max(-1.0, min(1.0, x)))), atol=1e-12)


def test_chebyshev_values_and_derivatives(L):
    T, dT = _f32(9), _f32(9)
    for x in np.linspace(-1, 1, 41):
        L.nep_test_cheb(x, _fp(T), _fp(dT))
        for k in range(9):
            e = np.eye(9)[k]
            assert abs(T[k] - np.polynomial.chebyshev.chebval(x, e)) < 2e-6
            assert abs(dT[k] - np.polynomial.chebyshev.chebval(x, np.polynomial.chebyshev.chebder(e))) < 2e-5


def _real_sh_scaled(l, u):
    """sqrt(4 pi/(2l+1)) times scipy's real spherical harmonics, up to an
    orthogonal change of basis within l: compared through P_l(u.v)."""
    theta = math.acos(max(-1.0, min(1.0, u[2])))
    phi = math.atan2(u[1], u[0])
    return np.array([sp.sph_harm_y(l, m, theta, phi) for m in range(-l, l + 1)])


def test_harmonics_addition_theorem(L):
    rng = np.random.default_rng(0)
    Ya, Yb = _f32(24), _f32(24)
    lo = [0, 3, 8, 15, 24]
    for _ in range(50):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        L.nep_test_sph(*u.astype(np.float32), _fp(Ya))
        L.nep_test_sph(*v.astype(np.float32), _fp(Yb))
        for l in range(1, 5):
            got = float(np.dot(Ya[lo[l - 1]:lo[l]], Yb[lo[l - 1]:lo[l]]))
            assert abs(got - sp.eval_legendre(l, float(u @ v))) < 2e-6
            # same span as scipy's complex harmonics: sum_m |Y_lm|^2 agree
            ca = _real_sh_scaled(l, u)
            assert abs(np.sum(Ya[lo[l - 1]:lo[l]] ** 2) - 4 * math.pi / (2 * l + 1) * np.sum(np.abs(ca) ** 2)) < 2e-6


def test_double_harmonics_addition_theorem_and_single_agreement(L):
    # the FP64 degree-by-degree harmonics used for the descriptor sums: the
    # addition theorem to FP64 accuracy, and the same functions as sph
    rng = np.random.default_rng(4)
    Ya, Yb = np.zeros(24), np.zeros(24)
    Yf = _f32(24)
    lo = [0, 3, 8, 15, 24]
    for _ in range(50):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        L.nep_test_sph_d(*u, Ya.ctypes.data_as(DP))
        L.nep_test_sph_d(*v, Yb.ctypes.data_as(DP))
        for l in range(1, 5):
            got = float(np.dot(Ya[lo[l - 1]:lo[l]], Yb[lo[l - 1]:lo[l]]))
            assert abs(got - sp.eval_legendre(l, float(u @ v))) < 1e-13
        uf = u.astype(np.float32)
        L.nep_test_sph(*uf, _fp(Yf))
        L.nep_test_sph_d(*uf.astype(np.float64), Ya.ctypes.data_as(DP))
        assert np.allclose(Yf, Ya, atol=3e-6)


def test_harmonics_parity(L):
    rng = np.random.default_rng(1)
    Ya, Yb = _f32(24), _f32(24)
    sign = np.array([-1] * 3 + [1] * 5 + [-1] * 7 + [1] * 9, dtype=np.float32)
    for _ in range(10):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        L.nep_test_sph(*u.astype(np.float32), _fp(Ya))
        L.nep_test_sph(*(-u).astype(np.float32), _fp(Yb))
        assert np.allclose(Yb, sign * Ya, atol=1e-7)


def test_harmonic_gradient_contraction_fd(L):
    rng = np.random.default_rng(2)
    Y = _f32(24)
    v = _f32(3)
    for _ in range(20):
        D = rng.normal(size=24).astype(np.float32)
        u = rng.normal(size=3) * 0.6
        L.nep_test_sph_grad(*u.astype(np.float32), _fp(D), _fp(v))
        h = 1e-3
        fd = np.zeros(3)
        for a in range(3):
            e = np.zeros(3); e[a] = h
            L.nep_test_sph(*(u + e).astype(np.float32), _fp(Y)); yp = float(D.astype(np.float64) @ Y)
            L.nep_test_sph(*(u - e).astype(np.float32), _fp(Y)); ym = float(D.astype(np.float64) @ Y)
            fd[a] = (yp - ym) / (2 * h)
        assert np.allclose(v, fd, rtol=2e-3, atol=2e-3)


def test_unnormalised_harmonics(L):
    # y_lm times its constant is the normalised harmonic (on and off the unit
    # sphere: both are the same polynomials); the contraction of the
    # unnormalised gradients matches finite differences
    rng = np.random.default_rng(3)
    K = _f32(24)
    L.nep_test_sph_norm(_fp(K))
    Y, y, v = _f32(24), _f32(24), _f32(3)
    for _ in range(50):
        u = rng.normal(size=3)
        u = (u / np.linalg.norm(u)).astype(np.float32)
        L.nep_test_sph(*u, _fp(Y))
        L.nep_test_sph_unnorm(*u, _fp(y))
        assert np.allclose(K.astype(np.float64) * y, Y, rtol=0, atol=5e-6)
    for _ in range(20):
        D = rng.normal(size=24).astype(np.float32)
        u = rng.normal(size=3) * 0.6
        L.nep_test_sph_unnorm_grad(*u.astype(np.float32), _fp(D), _fp(v))
        h = 1e-3
        fd = np.zeros(3)
        for a in range(3):
            e = np.zeros(3); e[a] = h
            L.nep_test_sph_unnorm(*(u + e).astype(np.float32), _fp(y)); yp = float(D.astype(np.float64) @ y)
            L.nep_test_sph_unnorm(*(u - e).astype(np.float32), _fp(y)); ym = float(D.astype(np.float64) @ y)
            fd[a] = (yp - ym) / (2 * h)
        assert np.allclose(v, fd, rtol=2e-3, atol=5e-3)


def test_zbl_pair_matches_oracle(L):
    import oracle
    U, dU = C.c_double(), C.c_double()
    for r in [0.2, 0.5, 0.8, 1.0, 1.3, 1.7, 1.99]:
        L.nep_test_zbl(r, 74.0, 1.0, 2.0, C.byref(U), C.byref(dU))
        Uo, dUo = oracle.zbl(r)
        assert abs(U.value - Uo) <= 1e-12 * max(1.0, Uo)
        assert abs(dU.value - dUo) <= 1e-12 * max(1.0, abs(dUo))


def test_neighbour_entry_decoding(L):
    out = (C.c_int * 4)()
    for jbits, ibits, ioff in ((26, 2, 1), (20, 4, 8)):
        for j, n in [(0, (0, 0, 0)), (12345, (-1, 1, 0)), ((1 << jbits) - 1, (1, -1, 1))]:
            code = (n[0] + ioff) | ((n[1] + ioff) << ibits) | ((n[2] + ioff) << (2 * ibits))
            e = np.int32(np.uint32(j | (code << jbits)))
            L.nep_test_decode(int(e), jbits, ibits, ioff, out)
            assert tuple(out) == (j,) + n


def test_bin_offset_entry_code(L):
    # bin-offset lists: an entry's code is q | (crossed faces << 5) with
    # q = (o0+1) + 3 (o1+1) + 9 (o2+1) the neighbour bin's offset; the image
    # on a crossed axis is the offset itself (a face is crossed only by a
    # nonzero offset), zero elsewhere.  The entry of the same pair seen from
    # the neighbour has offset -o, image -m: code (26 - q) with the same
    # crossed faces, which is what the reverse-index search looks for.
    import itertools
    seen = set()
    for o in itertools.product((-1, 0, 1), repeat=3):
        q = (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)
        for cross in itertools.product((0, 1), repeat=3):
            if any(c and oa == 0 for c, oa in zip(cross, o)):
                continue
            m = [oa if c else 0 for oa, c in zip(o, cross)]
            code = L.nep_test_delta_code(q, *m)
            assert code & 31 == q and code >> 5 == cross[0] | (cross[1] << 1) | (cross[2] << 2)
            cr = code >> 5
            n = [(q % 3 - 1) if cr & 1 else 0, ((q // 3) % 3 - 1) if cr & 2 else 0, (q // 9 - 1) if cr & 4 else 0]
            assert n == m
            rcode = L.nep_test_delta_code(26 - q, *[-x for x in m])
            assert rcode == ((26 - (code & 31)) | (code & ~31))
            assert code < (1 << 8) and code not in seen   # 8 bits beside 23 index bits, one code per case
            seen.add(code)
    assert len(seen) == 125


def test_sort32_network(L):
    # the list build's bin order: 27 keys (bin << 5 | offset) padded with
    # 0xffffffff to 32, sorted ascending by the odd-even merge network; also
    # duplicates, reversed and all-equal inputs
    rng = np.random.default_rng(11)
    cases = [rng.integers(0, 2**32 - 1, 32, dtype=np.uint64).astype(np.uint32) for _ in range(300)]
    cases += [rng.integers(0, 4, 32).astype(np.uint32) for _ in range(100)]
    for _ in range(200):
        k = np.full(32, 0xFFFFFFFF, dtype=np.uint32)
        n = int(rng.integers(0, 28))
        k[:n] = (rng.integers(0, 2**27, n).astype(np.uint32) << 5) | rng.permutation(27)[:n].astype(np.uint32)
        cases.append(rng.permutation(k))
    cases += [np.arange(32, dtype=np.uint32)[::-1].copy(), np.full(32, 7, dtype=np.uint32)]
    for a in cases:
        a = np.ascontiguousarray(a, dtype=np.uint32)
        ref = np.sort(a)
        L.nep_test_sort32(a.ctypes.data_as(C.POINTER(C.c_uint32)))
        assert np.array_equal(a, ref)
