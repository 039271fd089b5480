"""The allocation-free Pauli-sum expectation value
(qs_calc_expec_pauli_sum_noalloc) against qs_calc_expec_pauli_sum on the
same device amplitudes: two calls in a row per case, the second on a
smaller state, so the second call runs on scratch the first one left
behind.  Both compute the same FP64 sums in the same order."""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2311_01512_amd as pkg
    return pkg


def noalloc(q, codes, coeffs):
    from paper_2311_01512_amd import native as N
    lib = N.lib
    f = lib.qs_calc_expec_pauli_sum_noalloc
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    f.restype = C.c_int
    p = np.ascontiguousarray(np.asarray(codes, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    re, im = C.c_double(), C.c_double()
    rc = f(q.tensor.data_ptr(), q.num_qubits, int(q.density), N.QS_C64 if q.precision == "c64" else N.QS_C128,
           q.stream.cuda_stream, p.ctypes.data, c.ctypes.data, c.size, C.byref(re), C.byref(im))
    assert rc == 0, lib.qs_last_error()
    return complex(re.value, im.value)


def close(a, b, prec, scale):
    tol = (1e-12 if prec == "c128" else 1e-5) * max(1.0, scale)
    return abs(a - b) <= tol


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("density,sizes", [(False, (22, 9)), (False, (12, 5)), (True, (9, 4))])
def test_noalloc_matches_expec_pauli_sum(qs, prec, density, sizes):
    rng = np.random.default_rng(77 + sizes[0])
    for n in sizes:
        banner(f"noalloc expec {prec} density={density} n={n}")
        q = qs.Qureg(n, density=density, precision=prec).init_hashed(1000 + n)
        codes = rng.integers(0, 4, size=(20, n)).astype(np.int32)
        coeffs = rng.standard_normal(20)
        want = q.expec_pauli_sum(codes, coeffs)
        got = noalloc(q, codes, coeffs)
        scale = float(np.abs(coeffs).sum())
        assert close(got.real, want.real, prec, scale), (n, got, want)
        assert close(got.imag, want.imag, prec, scale), (n, got, want)
        del q


def test_noalloc_rejects_bad_arguments(qs):
    from paper_2311_01512_amd import native as N
    f = N.lib.qs_calc_expec_pauli_sum_noalloc
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    re, im = C.c_double(), C.c_double()
    assert f(None, 4, 0, 1, None, None, None, 0, C.byref(re), C.byref(im)) == -1
    host = np.zeros(32, np.complex128)      # host memory is refused
    assert f(host.ctypes.data, 4, 0, 1, None, None, None, 0, C.byref(re), C.byref(im)) == -1
