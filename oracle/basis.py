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


# ----------------------------------------------------------------------------
# local time steps: a macro-element's interval bisected into n equal
# sub-intervals (Section 2.2), trial space continuous piecewise P_q and test
# space piecewise P_{q-1} (eq. spaces:local:patch)
# ----------------------------------------------------------------------------

def trial_level(q, n, j, m):
    """Level of the local trial function l_m of sub-interval j (of n) in the
    flattened trial block of 1 + n q levels.  Level 0 is the value at the slab
    start, level 1 the value at the slab end (as for n = 1); sub-interval j
    then owns the q levels 2 + j q .. 1 + (j + 1) q: its interior functions
    l_2..l_q, then (j < n - 1) the value at its right end, which is also l_0
    of sub-interval j + 1 (continuity in time inside the slab).  For n = 1
    this is the identity m -> m."""
    if m == 0:
        return 0 if j == 0 else 1 + j * q
    if m == 1:
        return 1 if j == n - 1 else 1 + (j + 1) * q
    return 2 + j * q + (m - 2)


def subinterval_trial_values(q, n, s):
    """Values and d/ds of the 1 + n q flattened trial functions at slab
    coordinates s in (0, 1) that are not sub-interval ends: [..., level]."""
    s = np.asarray(s, dtype=np.float64)
    j = np.minimum((s * n).astype(np.int64), n - 1)
    xi = n * s - j
    V = np.zeros(s.shape + (1 + n * q,))
    dV = np.zeros_like(V)
    for m in range(q + 1):
        lev = np.array([trial_level(q, n, int(jj), m) for jj in np.ravel(j)]).reshape(s.shape)
        np.add.at(V, (np.arange(s.size), lev.ravel()), ltrial(m, xi).ravel())
        np.add.at(dV, (np.arange(s.size), lev.ravel()), n * dltrial(m, xi).ravel())
    return V, dV


def subinterval_test_values(q, n, s):
    """Test functions L_i^(j)(s) = L_i(n s - j) on sub-interval j, zero
    elsewhere; column j q + i."""
    s = np.asarray(s, dtype=np.float64)
    j = np.minimum((s * n).astype(np.int64), n - 1)
    xi = n * s - j
    V = np.zeros(s.shape + (n * q,))
    for jj in range(n):
        on = j == jj
        for i in range(q):
            V[on, jj * q + i] = L(i, xi[on])
    return V


def subinterval_time_table(qr, nr, qc, nc, deriv=False, proj=None):
    """T[(j, i), M] = int_0^1 (pi L_i^(j))(s) phi_M(s) ds over the slab in
    its unit coordinate s = (t - t_{n-1}) / dt: test function i of sub-interval
    j of the row element (degree qr, nr sub-intervals) against flattened trial
    level M of the column element (qc, nc), or against d phi_M / ds with
    ``deriv``.  ``proj = (r, n_p)`` applies pi, the L2 projection onto
    piecewise polynomials of degree < r on n_p equal sub-intervals, to the
    test function (the common temporal test space of S_h, Section 4.1 eq.
    bilinearform:S); without it pi is the identity.  All n are powers of two,
    so the partitions nest and a composite Gauss rule on the finest one
    integrates every product exactly."""
    nf = max(nr, nc, proj[1] if proj is not None else 1)
    xg, wg = gauss01(qr + qc + 2)
    s = ((np.arange(nf)[:, None] + xg[None, :]) / nf).ravel()
    w = np.tile(wg, nf) / nf
    test = subinterval_test_values(qr, nr, s)
    if proj is not None:
        r, npj = proj
        c = np.minimum((s * npj).astype(np.int64), npj - 1)
        xi = npj * s - c
        out = np.zeros_like(test)
        for cc in range(npj):
            on = c == cc
            for rho in range(r):
                Lr = L(rho, xi[on])
                # coefficient of L_rho(n_p s - cc), whose square integrates to 1 / n_p
                beta = npj * np.sum((w[on] * Lr)[:, None] * test[on], axis=0)
                out[on] += Lr[:, None] * beta[None, :]
        test = out
    V, dV = subinterval_trial_values(qc, nc, s)
    return (test * w[:, None]).T @ (dV if deriv else V)
