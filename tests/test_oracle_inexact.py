"""Pins of the inexact-solve pieces of the oracle (Section 5.3): the dual norm
of a residual in W_h' and the guaranteed iteration-error bound eta_it.

* the dual norm is the supremum of R(V) / ||V||_{L2(I; L2)} over the test
  space: attained by the Riesz representor, never exceeded by random V;
* eta_it bounds the actual iteration error of inexact slab solutions (any
  trial function with the right l_0 block) at the end of the slabs, over
  one and several slabs, on affine meshes with uneven materials."""
import numpy as np
import pytest

import synth
from oracle import basis
from oracle.dg import Discretisation, mass_matrix


def _mesh(seed, shape=(2, 2, 1), p=2, q=2):
    v, h = synth.box_mesh(shape, hi=(0.6, 0.5, 0.3))
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    return Discretisation(v, h, np.full(ne, p), np.full(ne, q), rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


def _test_l2_norm2(d, V, dt):
    """||V||^2 in L2(I_n; L2(Omega)) of a residual-layout test function by
    quadrature in time (Legendre values at Gauss points) and the mass in space."""
    tx, tw = basis.gauss01(int(d.q.max()) + 2)
    tot = 0.0
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        M = mass_matrix(d.X(e), int(d.a[e]), 1.0, d.nq(e))
        blk = V[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)
        for f in range(2):
            for tau, w in zip(tx, tw):
                vt = sum(basis.L(i, tau) * blk[f][:, i, :] for i in range(qe)).reshape(-1)
                tot += dt * w * vt @ M @ vt
    return tot


def test_dual_norm_is_the_supremum():
    d = _mesh(1)
    dt = 0.07
    rng = np.random.default_rng(2)
    R = rng.standard_normal(d.unk_off[-1])
    rE, rH = d.dual_norms(R, dt)
    full = rE + rH
    # the functional V -> R . V (coefficients) attains sqrt(full) at the representor
    z = np.zeros_like(R)
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        M = mass_matrix(d.X(e), int(d.a[e]), 1.0, d.nq(e))
        blk = R[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)
        zb = np.zeros_like(blk)
        for f in range(2):
            rhs = blk[f].transpose(0, 2, 1).reshape(3 * a3, qe)
            zb[f] = (np.linalg.solve(M, rhs) / dt).reshape(3, a3, qe).transpose(0, 2, 1)
        z[d.unk_off[e]:d.unk_off[e + 1]] = zb.ravel()
    val = R @ z / np.sqrt(_test_l2_norm2(d, z, dt))
    assert abs(val - np.sqrt(full)) < 1e-10 * np.sqrt(full)
    for _ in range(20):
        V = rng.standard_normal(d.unk_off[-1])
        assert R @ V / np.sqrt(_test_l2_norm2(d, V, dt)) <= np.sqrt(full) * (1 + 1e-12)


@pytest.mark.parametrize("n_slabs", [1, 3])
def test_eta_it_bounds_the_iteration_error(n_slabs):
    d = _mesh(3)
    dt = 0.05
    rng = np.random.default_rng(4)
    s_exact = rng.standard_normal(d.state_off[-1])
    s_inexact = s_exact.copy()
    eta2 = 0.0
    t_final = n_slabs * dt
    for n in range(n_slabs):
        U_ex = d.solve_direct(s_exact, dt)
        # an inexact slab solution: start from the inexact state, perturb the unknowns
        U_in = d.solve_direct(s_inexact, dt)
        x = d.unknowns_of(U_in) + 1e-3 * rng.standard_normal(d.unk_off[-1])
        U_in = d.embed_unknowns(x, s_inexact)
        R = d.residual(U_in, dt) - d.residual(d.solve_direct(s_inexact, dt), dt)  # B(U^m - U_h(s), V)
        eta2 += d.eta_it_term(R, dt, t_final)
        s_exact = d.level_state(U_ex, 1)
        s_inexact = d.level_state(U_in, 1)
    err = s_inexact - s_exact
    err2 = 2.0 * d.energy(err)          # ||eps^1/2 e||^2 + ||mu^1/2 h||^2
    print("efficiency index", np.sqrt(eta2 / err2))
    assert err2 <= eta2, (err2, eta2)
    assert err2 > 1e-4 * eta2           # and not vacuous
