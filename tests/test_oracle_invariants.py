"""Pins of the oracle's residual, load, solve and energy against what the paper
and the mathematics fix:

* skew-symmetry of the curl + centred-flux operator (the cancellation in the
  proof of Thm 3.1, Section 3.1);
* exact energy conservation for PEC cavities without sources, uniform q
  (Thm 3.1) and mixed q with the stabilisation S_h (Thm 4.1), and the energy
  identity E(t_n) - E(t_{n-1}) = (J, pi_W E_h) with a source;
* the time discretisation: with uniform q and no source the end-of-slab map
  equals the (q, q) Pade approximant of exp(-dt M^{-1} K) (continuous
  Petrov-Galerkin in time with test degree q-1 = q-stage Gauss collocation);
  q = 1 is Crank-Nicolson;
* exact reproduction of manufactured solutions inside the discrete space
  (Section 6.1.2 family), on affine and trilinear meshes, uniform and mixed q;
* the temporal convergence orders of Section 6.1.2 (nodal order 2q);
* the TE101 cavity mode: projected energy and one-slab error.
"""
from math import factorial

import numpy as np
import pytest

import synth
from oracle import fields
from oracle.dg import Discretisation


def _disc(shape, p, q, eps=None, mu=None, vertices=None, hi=(1.0, 1.0, 1.0)):
    v, h = synth.box_mesh(shape, hi=hi)
    if vertices is not None:
        v = vertices
    ne = h.shape[0]
    p = np.broadcast_to(np.asarray(p), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q), (ne,)).copy()
    eps = np.ones(ne) if eps is None else np.asarray(eps, dtype=float)
    mu = np.ones(ne) if mu is None else np.asarray(mu, dtype=float)
    return Discretisation(v, h, p, q, eps, mu)


def test_spatial_operator_is_skew():
    rng = np.random.default_rng(0)
    d = _disc((2, 2, 1), [1, 2, 2, 1], 1, rng.uniform(1, 4, 4), rng.uniform(1, 2, 4))
    M, K = d.spatial_operators()
    assert np.abs(K + K.T).max() < 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(M).min() > 0


def test_skew_through_residual_apply():
    # x only in level m = 1: <y_0 - M x_1, x_1> = 0 since N_{0,1} = 1/2 and the
    # spatial operator is skew.
    rng = np.random.default_rng(1)
    d = _disc((2, 2, 2), 2, 2, rng.uniform(1, 4, 8), np.ones(8))
    x = np.zeros(d.unk_off[-1])
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        blk = x[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, 2, a3)
        blk[:, :, 0, :] = rng.standard_normal((2, 3, a3))
    y = d.operator(x, 0.1)
    tot = 0.0
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        xb = x[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, 2, a3)[:, :, 0, :].reshape(2, 3 * a3)
        yb = y[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, 2, a3)[:, :, 0, :].reshape(2, 3 * a3)
        tot += (yb[0] - d.mass(e, "eps") @ xb[0]) @ xb[0] + (yb[1] - d.mass(e, "mu") @ xb[1]) @ xb[1]
    assert abs(tot) < 1e-12 * np.abs(y).sum()


@pytest.mark.parametrize("qs", [(1, 1), (2, 2), (3, 3), (1, 3), (2, 1)])
def test_energy_conserved_without_source(qs):
    # Thm 3.1 (uniform q) and Thm 4.1 (mixed q, with S_h): PEC, J = 0
    rng = np.random.default_rng(2)
    q = np.array([qs[0], qs[1]] * 4)
    d = _disc((2, 2, 2), [2, 1, 1, 2, 2, 1, 1, 2], q, rng.uniform(1, 4, 8), rng.uniform(1, 2, 8))
    s0 = rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.15)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) < 1e-12 * e0


def test_energy_conserved_on_trilinear_mesh():
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=4)
    rng = np.random.default_rng(5)
    d = Discretisation(v, h, np.full(8, 2), np.array([1, 2] * 4), rng.uniform(1, 3, 8), np.ones(8))
    s0 = rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.1)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) < 1e-12 * e0


def test_energy_identity_with_source():
    # E(t_n) - E(t_{n-1}) = (J, pi_W E_h) = sum L_E[i] . (N e)_i  (Thm 3.1)
    rng = np.random.default_rng(6)
    d = _disc((2, 2, 2), 2, 2, rng.uniform(1, 4, 8), np.ones(8))
    J = fields.gaussian_pulse(3.0, (0.4, 0.5, 0.6), 0.3, 1.5, -0.1, 0.2, (0.3, -0.5, 1.0))
    dt = 0.1
    L = d.load(J, 0.0, dt)
    s0 = 1e-3 * rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, dt, L)
    work = 0.0
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        _, N = d.tables(qe, qe)
        Ut = d.split_trial(U, e)[0]                       # E part [(c,s), m]
        piE = Ut @ N.T                                    # [(c,s), i]
        Lb = L[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)[0].transpose(0, 2, 1).reshape(3 * a3, qe)
        work += np.sum(Lb * piE)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs((e1 - e0) - work) < 1e-11 * max(abs(work), e0)
    assert abs(work) > 1e-2 * e0


def _pade(q, A):
    def P(z):
        out = np.zeros_like(z)
        zk = np.eye(z.shape[0])
        for j in range(q + 1):
            out = out + factorial(2 * q - j) * factorial(q) / (factorial(2 * q) * factorial(j) * factorial(q - j)) * zk
            zk = zk @ z
        return out
    return np.linalg.solve(P(-A), P(A))


@pytest.mark.parametrize("q", [1, 2, 3])
def test_end_of_slab_map_is_pade(q):
    rng = np.random.default_rng(10 + q)
    d = _disc((2, 1, 2), [2, 1, 1, 2], q, rng.uniform(1, 3, 4), rng.uniform(1, 2, 4))
    dt = 0.3
    M, K = d.spatial_operators()
    A = -dt * np.linalg.solve(M, K)
    s0 = rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, dt)
    ref = _pade(q, A) @ s0
    got = d.level_state(U, 1)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_q1_is_crank_nicolson():
    rng = np.random.default_rng(20)
    d = _disc((1, 2, 2), 2, 1, rng.uniform(1, 3, 4))
    dt = 0.2
    M, K = d.spatial_operators()
    s0 = rng.standard_normal(d.state_off[-1])
    ref = np.linalg.solve(M + 0.5 * dt * K, (M - 0.5 * dt * K) @ s0)
    got = d.level_state(d.solve_direct(s0, dt), 1)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("q,acoef", [(1, [0.7]), (2, [0.3, -1.2]), (3, [0.5, 0.2, 2.0])])
def test_manufactured_solution_reproduced_affine(q, acoef):
    # MS-1 on axis-aligned boxes, p = 2 (E, H in Q_2), deg a <= q - 1
    eps, mu = 2.0, 0.5
    d = _disc((2, 1, 2), 2, q, np.full(4, eps), np.full(4, mu))
    F, J = fields.ms1(acoef, eps, mu)
    t0, dt = 0.2, 0.3
    s0 = fields.reference_coefficients(d, F, t0)
    L = d.load(J, t0, dt)
    U = d.solve_direct(s0, dt, L)
    for tau in (1.0, 0.37):
        ref = fields.reference_coefficients(d, F, t0 + tau * dt)
        got = _state_at(d, U, tau)
        assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_manufactured_static_solution_trilinear_mixed_q():
    # MS-2: E = 0, H = (y^2, z^2, x^2); covariant pull-back in Q_3 on trilinear
    # elements; static in time, so it lies in every common test space (S_h active)
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.2, seed=8)
    q = np.array([1, 2, 3, 1, 2, 1, 3, 2])
    d = Discretisation(v, h, np.full(8, 3), q, np.full(8, 1.5), np.full(8, 0.7))
    F, J = fields.ms2()
    s0 = fields.reference_coefficients(d, F, 0.0)
    L = d.load(J, 0.0, 0.25)
    U = d.solve_direct(s0, 0.25, L)
    got = d.level_state(U, 1)
    assert np.abs(got - s0).max() < 1e-11 * np.abs(s0).max()


def _state_at(d, U, tau):
    from oracle import basis
    S = np.zeros(d.state_off[-1])
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        blk = U[d.trial_off[e]:d.trial_off[e + 1]].reshape(2, 3, qe + 1, a3)
        lt = np.array([basis.ltrial(m, np.array([tau]))[0] for m in range(qe + 1)])
        S[d.state_off[e]:d.state_off[e + 1]] = np.einsum("fcma,m->fca", blk, lt).ravel()
    return S


@pytest.mark.parametrize("q", [1, 2])
def test_temporal_order_exp_solution(q):
    # Section 6.1.2: spatial part exact for p >= 2, so the nodal error is the
    # time error of order 2q
    F, J = fields.exp_solution()
    d = _disc((1, 1, 1), 2, q)
    T = 0.4
    errs = []
    for nsteps in (2, 4):
        dt = T / nsteps
        s = fields.reference_coefficients(d, F, 0.0)
        for n in range(nsteps):
            L = d.load(J, n * dt, dt, nt=q + 8)
            U = d.solve_direct(s, dt, L)
            s = d.level_state(U, 1)
        errs.append(np.abs(s - fields.reference_coefficients(d, F, T)).max())
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - 2 * q) < 0.3, (errs, rate)


def test_te101_energy_and_one_slab_error():
    # TE101 on the 4^3 cavity, p = 2, q = 1, dt = 0.05: projected energy ~ 1/8
    # and the one-slab error stays at the size of the projection error.
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    s0 = fields.project(d, fields.te101, 0.0)
    assert abs(d.energy(s0) - 0.125) < 2e-3
    U = d.solve_direct(s0, cfg["dt"])
    err = fields.l2_error(d, d.level_state(U, 1), fields.te101, cfg["dt"])
    err0 = fields.l2_error(d, s0, fields.te101, 0.0)
    assert err < 1.5 * err0 and err < 5e-3
