"""Pins of the oracle's 1D tables (Section 5.1 bases; Section 5.2 time and curl
factors) against closed forms of textbook Legendre identities and against
scipy's Legendre routine."""
import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import basis


@pytest.mark.parametrize("j", range(9))
def test_legendre_matches_library(j):
    xi = np.linspace(0, 1, 17)
    ref = np.sqrt(2 * j + 1) * eval_legendre(j, 2 * xi - 1)
    assert np.allclose(basis.L(j, xi), ref, atol=1e-13, rtol=0)


def test_orthonormal_on_unit_interval():
    x, w = basis.gauss01(12)
    V = basis.legendre_matrix(9, x)
    G = (V * w[:, None]).T @ V
    assert np.abs(G - np.eye(9)).max() < 1e-13


def test_integrated_legendre_definition():
    # l_0 = 1 - xi, l_1 = xi, l_m(0) = 0, l_m' = L_{m-1}, and l_m(1) = 0 for m >= 2
    xi = np.linspace(0, 1, 11)
    assert np.allclose(basis.ltrial(0, xi), 1 - xi)
    assert np.allclose(basis.ltrial(1, xi), xi)
    h = 1e-6
    for m in range(2, 8):
        assert abs(basis.ltrial(m, np.array([0.0]))[0]) < 1e-14
        assert abs(basis.ltrial(m, np.array([1.0]))[0]) < 1e-14
        fd = (basis.ltrial(m, xi[1:-1] + h) - basis.ltrial(m, xi[1:-1] - h)) / (2 * h)
        assert np.allclose(fd, basis.L(m - 1, xi[1:-1]), atol=1e-7)


@pytest.mark.parametrize("q", range(1, 7))
def test_time_derivative_table_is_shift(q):
    # int L_i l_m' = delta_{m, i+1} - delta_{i0} delta_{m0}
    D, _ = basis.time_tables(q)
    ref = np.zeros((q, q + 1))
    for i in range(q):
        ref[i, i + 1] = 1.0
    ref[0, 0] = -1.0
    assert np.abs(D - ref).max() < 1e-14


@pytest.mark.parametrize("q", range(1, 7))
def test_time_curl_table_closed_form(q):
    # l_m = (L_m/sqrt(2m+1) - L_{m-2}/sqrt(2m-3)) / (2 sqrt(2m-1)), m >= 2;
    # l_0 = (L_0 - L_1/sqrt3)/2, l_1 = (L_0 + L_1/sqrt3)/2
    _, N = basis.time_tables(q)
    ref = np.zeros((q, q + 1))
    ref[0, 0] = ref[0, 1] = 0.5
    if q > 1:
        ref[1, 0] = -0.5 / np.sqrt(3)
        ref[1, 1] = 0.5 / np.sqrt(3)
    for m in range(2, q + 1):
        if m < q:
            ref[m, m] = 1.0 / (2 * np.sqrt((2 * m - 1) * (2 * m + 1)))
        if m - 2 < q:
            ref[m - 2, m] = -1.0 / (2 * np.sqrt((2 * m - 1) * (2 * m - 3)))
    assert np.abs(N - ref).max() < 1e-14


@pytest.mark.parametrize("a", range(2, 10))
def test_derivative_table_closed_form(a):
    # int L_n L_j' = 2 sqrt((2n+1)(2j+1)) for n < j, j - n odd; else 0
    Dh = basis.derivative_table(a)
    ref = np.zeros((a, a))
    for n in range(a):
        for j in range(a):
            if n < j and (j - n) % 2 == 1:
                ref[n, j] = 2 * np.sqrt((2 * n + 1) * (2 * j + 1))
    assert np.abs(Dh - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("a", range(1, 10))
def test_trace_values(a):
    t0, t1 = basis.trace_values(a)
    j = np.arange(a)
    assert np.allclose(t0, (-1.0) ** j * np.sqrt(2 * j + 1), atol=1e-13)
    assert np.allclose(t1, np.sqrt(2 * j + 1), atol=1e-13)
