"""1D functions of the tensor-product bases and their tables (oracle step O1).

Section 5.1: spatial basis L_j(x-hat) L_k(y-hat) L_l(z-hat) e_c with L_j the
orthonormal Legendre polynomials on [0, 1]; trial basis in time the integrated
Legendre polynomials l_0 = 1 - xi, l_1 = xi, l_m = int_0^xi L_{m-1} (eq.
def:ilegendre); test basis in time L_i, i = 0..q-1.

Reading of the interval: the implementation section works on [0, 1] (the proofs
of Section 3 use [-1, 1]); the oracle uses [0, 1] throughout.  Every table is
computed by Gauss quadrature, never typed in; the tests pin them to the closed
forms of the Legendre identities.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gauss01(n):
    """n-point Gauss-Legendre rule mapped to [0, 1]."""
    x, w = npleg.leggauss(int(n))
    return 0.5 * (x + 1.0), 0.5 * w


def _unit(j):
    c = np.zeros(j + 1)
    c[j] = 1.0
    return c


def L(j, xi):
    """Orthonormal Legendre polynomial of degree j on [0, 1]: sqrt(2j+1) P_j(2 xi - 1)."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.sqrt(2 * j + 1) * npleg.legval(2.0 * xi - 1.0, _unit(j))


def dL(j, xi):
    """d/dxi of L(j, xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    if j == 0:
        return np.zeros_like(xi)
    return 2.0 * np.sqrt(2 * j + 1) * npleg.legval(2.0 * xi - 1.0, npleg.legder(_unit(j)))


def ltrial(m, xi):
    """Integrated Legendre trial function l_m of eq. def:ilegendre."""
    xi = np.asarray(xi, dtype=np.float64)
    if m == 0:
        return 1.0 - xi
    if m == 1:
        return xi.copy()
    # int_0^xi L_{m-1}(s) ds with u = 2s - 1, ds = du / 2
    ci = npleg.legint(_unit(m - 1), lbnd=-1.0)
    return np.sqrt(2 * m - 1) * 0.5 * npleg.legval(2.0 * xi - 1.0, ci)


def dltrial(m, xi):
    """d/dxi of ltrial(m, xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    if m == 0:
        return -np.ones_like(xi)
    if m == 1:
        return np.ones_like(xi)
    return L(m - 1, xi)


def legendre_matrix(a, xi):
    """V[g, j] = L_j(xi_g), j = 0..a-1."""
    return np.stack([L(j, xi) for j in range(a)], axis=-1)


def dlegendre_matrix(a, xi):
    return np.stack([dL(j, xi) for j in range(a)], axis=-1)


def time_tables(q_test, q_trial=None):
    """D[i, m] = int_0^1 L_i l_m' and N[i, m] = int_0^1 L_i l_m for test levels
    i = 0..q_test-1 and trial levels m = 0..q_trial (Section 5.2, mass and curl
    residuals).  q_trial defaults to q_test."""
    if q_trial is None:
        q_trial = q_test
    xg, wg = gauss01(max(q_test, q_trial) + 2)
    D = np.zeros((q_test, q_trial + 1))
    N = np.zeros((q_test, q_trial + 1))
    for i in range(q_test):
        Li = L(i, xg)
        for m in range(q_trial + 1):
            D[i, m] = np.sum(wg * Li * dltrial(m, xg))
            N[i, m] = np.sum(wg * Li * ltrial(m, xg))
    return D, N


def derivative_table(a):
    """Dhat[n, j] = int_0^1 L_n L_j' (the 1D factor of the reference curl)."""
    xg, wg = gauss01(a + 1)
    V = legendre_matrix(a, xg)
    dV = dlegendre_matrix(a, xg)
    return (V * wg[:, None]).T @ dV


def trace_values(a):
    """(L_j(0), L_j(1)) for j = 0..a-1: the face evaluations of the spatial basis."""
    return legendre_matrix(a, np.array([0.0]))[0], legendre_matrix(a, np.array([1.0]))[0]
