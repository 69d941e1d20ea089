"""Analytic fields and their projections onto the discrete space.

* TE101 cube-cavity mode (eps = mu = 1): E = e_y sin(pi x) sin(pi z) cos(w t),
  H = (pi / w) sin(w t) (sin(pi x) cos(pi z), 0, -cos(pi x) sin(pi z)),
  w = pi sqrt(2).  (The paper names cavity modes in Section 5.4 and 6.1 without
  writing this one out; it solves eq. maxwell with n x E = 0 on the unit cube.)
* Manufactured solution of Section 6.1.2: E = e^t x(x-1) z(1-z) e_y with its
  H and J; the generalisation E = a(t) x(1-x) z(1-z) e_y (MS-1) and the static
  H = (y^2, z^2, x^2), E = 0, J = -curl H (MS-2).
* Cavity-mode superpositions and the Gaussian-pulse current.

Projections: the L2 projection onto the covariant discrete space (solve with
the element mass matrix), and, for fields whose covariant pull-back is a
polynomial inside Q_p, the exact reference coefficients int E-hat_c phi_s.
"""
import numpy as np

from . import basis
from .dg import tensor_points, basis_at, mass_matrix
from .geometry import jacobian, map_point

W101 = np.pi * np.sqrt(2.0)


def te101(x, t):
    s = np.sin
    c = np.cos
    pi = np.pi
    E = np.zeros_like(x)
    H = np.zeros_like(x)
    E[:, 1] = s(pi * x[:, 0]) * s(pi * x[:, 2]) * c(W101 * t)
    H[:, 0] = (pi / W101) * s(W101 * t) * s(pi * x[:, 0]) * c(pi * x[:, 2])
    H[:, 2] = -(pi / W101) * s(W101 * t) * c(pi * x[:, 0]) * s(pi * x[:, 2])
    return E, H


def ms1(acoef, eps=1.0, mu=1.0):
    """MS-1 with a(t) = sum_k acoef[k] t^k: returns (E, H, J) callables of (x, t).
    A(t) = int_0^t a, so H(0) = 0."""
    acoef = np.asarray(acoef, dtype=np.float64)

    def a(t):
        return sum(c * t ** k for k, c in enumerate(acoef))

    def da(t):
        return sum(k * c * t ** (k - 1) for k, c in enumerate(acoef) if k > 0)

    def A(t):
        return sum(c * t ** (k + 1) / (k + 1) for k, c in enumerate(acoef))

    def fields(x, t):
        X, Z = x[:, 0], x[:, 2]
        E = np.zeros_like(x)
        H = np.zeros_like(x)
        E[:, 1] = a(t) * X * (1 - X) * Z * (1 - Z)
        H[:, 0] = (A(t) / mu) * X * (1 - X) * (1 - 2 * Z)
        H[:, 2] = -(A(t) / mu) * (1 - 2 * X) * Z * (1 - Z)
        return E, H

    def J(x, t):
        X, Z = x[:, 0], x[:, 2]
        out = np.zeros_like(x)
        out[:, 1] = eps * da(t) * X * (1 - X) * Z * (1 - Z) + (2 * A(t) / mu) * (X * (1 - X) + Z * (1 - Z))
        return out

    return fields, J


def exp_solution():
    """Section 6.1.2: E = e^t x(x-1) z(1-z) e_y,
    H = e^t (x(x-1)(1-2z), 0, -(2x-1) z(1-z)), eps = mu = 1."""
    def fields(x, t):
        X, Z = x[:, 0], x[:, 2]
        E = np.zeros_like(x)
        H = np.zeros_like(x)
        E[:, 1] = np.exp(t) * X * (X - 1) * Z * (1 - Z)
        H[:, 0] = np.exp(t) * X * (X - 1) * (1 - 2 * Z)
        H[:, 2] = -np.exp(t) * (2 * X - 1) * Z * (1 - Z)
        return E, H

    def J(x, t):
        # eps E_t - curl H
        X, Z = x[:, 0], x[:, 2]
        out = np.zeros_like(x)
        out[:, 1] = np.exp(t) * (X * (X - 1) * Z * (1 - Z) + 2 * X * (X - 1) - 2 * Z * (1 - Z))
        return out

    return fields, J


def ms2():
    """MS-2: E = 0, H = (y^2, z^2, x^2) (static), J = -curl H = (2z, 2x, 2y)."""
    def fields(x, t):
        E = np.zeros_like(x)
        H = np.stack([x[:, 1] ** 2, x[:, 2] ** 2, x[:, 0] ** 2], axis=1)
        return E, H

    def J(x, t):
        return np.stack([2 * x[:, 2], 2 * x[:, 0], 2 * x[:, 1]], axis=1)

    return fields, J


def mode_superposition(mnl, abc):
    """E = sum_r (A cos(m pi x) sin(n pi y) sin(l pi z), B sin cos sin, C sin sin cos), H = 0."""
    mnl = np.asarray(mnl, dtype=np.float64)
    abc = np.asarray(abc, dtype=np.float64)

    def fields(x, t):
        E = np.zeros_like(x)
        for (m, n, l), (A, B, C) in zip(mnl, abc):
            kx, ky, kz = np.pi * m * x[:, 0], np.pi * n * x[:, 1], np.pi * l * x[:, 2]
            E[:, 0] += A * np.cos(kx) * np.sin(ky) * np.sin(kz)
            E[:, 1] += B * np.sin(kx) * np.cos(ky) * np.sin(kz)
            E[:, 2] += C * np.sin(kx) * np.sin(ky) * np.cos(kz)
        return E, np.zeros_like(x)

    return fields


def gaussian_pulse(amp, center, sigma_x, f0, t0, sigma_t, direction):
    center = np.asarray(center, dtype=np.float64)
    direction = np.asarray(direction, dtype=np.float64)

    def J(x, t):
        r2 = ((x - center[None, :]) ** 2).sum(axis=1)
        g = amp * np.exp(-r2 / (2 * sigma_x ** 2)) * np.sin(2 * np.pi * f0 * (t - t0)) \
            * np.exp(-(t - t0) ** 2 / (2 * sigma_t ** 2))
        return g[:, None] * direction[None, :]

    return J


def project(disc, fields, t, nq=None):
    """L2 projection of (E, H)(., t) onto the discrete space: per element, solve
    M c = int F . DF^{-T} e_c phi_s |J| with the unit-coefficient mass matrix,
    both by an nq^3 Gauss rule (default p + 4).  Returns a state vector."""
    S = np.zeros(disc.state_off[-1])
    for e in range(disc.ne):
        a = int(disc.a[e])
        n = a + 3 if nq is None else nq
        X = disc.X(e)
        pts, w = tensor_points(n)
        x = map_point(X, pts)
        DF = jacobian(X, pts)
        det = np.linalg.det(DF)
        Dinv = np.linalg.inv(DF)
        Phi, _ = basis_at(a, pts)
        M = mass_matrix(X, a, 1.0, n)
        E, H = fields(x, t)
        out = []
        for F in (E, H):
            Fr = np.einsum("pcm,pm->pc", Dinv, F) * (det * w)[:, None]
            rhs = (Fr.T @ Phi).ravel()
            out.append(np.linalg.solve(M, rhs))
        S[disc.state_off[e]:disc.state_off[e + 1]] = np.concatenate(out)
    return S


def reference_coefficients(disc, fields, t, nq=None):
    """Coefficients of the covariant pull-back E-hat = DF^T (E o F): for each
    component, int_Khat E-hat_c phi_s (exact when E-hat_c lies in Q_p and the
    rule is exact for the product)."""
    S = np.zeros(disc.state_off[-1])
    for e in range(disc.ne):
        a = int(disc.a[e])
        n = 2 * a + 2 if nq is None else nq
        X = disc.X(e)
        pts, w = tensor_points(n)
        x = map_point(X, pts)
        DF = jacobian(X, pts)
        Phi, _ = basis_at(a, pts)
        E, H = fields(x, t)
        out = []
        for F in (E, H):
            Fh = np.einsum("pmc,pm->pc", DF, F)          # (DF^T F)_c
            out.append(((Fh * w[:, None]).T @ Phi).ravel())
        S[disc.state_off[e]:disc.state_off[e + 1]] = np.concatenate(out)
    return S


def l2_error(disc, state, fields, t, nq=None):
    """|| (E_h, H_h) - (E, H)(t) ||_{L2(Omega)} for a discrete state."""
    tot = 0.0
    for e in range(disc.ne):
        a = int(disc.a[e])
        n = a + 4 if nq is None else nq
        X = disc.X(e)
        pts, w = tensor_points(n)
        x = map_point(X, pts)
        DF = jacobian(X, pts)
        det = np.linalg.det(DF)
        Dinv = np.linalg.inv(DF)
        Phi, _ = basis_at(a, pts)
        E, H = fields(x, t)
        blk = state[disc.state_off[e]:disc.state_off[e + 1]].reshape(2, 3, a ** 3)
        for fld, F in enumerate((E, H)):
            hat = Phi @ blk[fld].T                         # [P, 3] reference components
            Fh = np.einsum("pmc,pm->pc", Dinv, hat)        # DF^{-T} hat: (DF^{-T})_{cm} hat_m
            tot += np.sum(w * det * ((Fh - F) ** 2).sum(axis=1))
    return np.sqrt(tot)
