"""Pins of the oracle with local time steps: each element's slab interval
bisected into n = 1, 2, 4 equal sub-intervals (Section 2.2), trial space
continuous piecewise P_q in time and test space piecewise P_{q-1} (eq.
spaces:local:patch), and S_h (Section 4.1, eq. bilinearform:S) coupling
neighbours through the projection onto their common temporal test space.

* with one sub-interval on both sides the sub-interval tables are the plain
  tables, and the projection keeps the test levels i < min(q, q');
* the flattened trial basis is continuous, reproduces constants and puts
  the slab start and end values at levels 0 and 1;
* the oracle's slab matrix (S_h reduced to a projected neighbour coupling)
  equals the physical-space brute-force assembler (S_h written out for both
  sides, the projection by its Gram matrix), for mixed n, q and p, on
  reoriented and on 2:1 hanging meshes;
* Thm 4.1: the energy is conserved without sources for mixed n and q, and
  without the projection it is not (planted mistake); with a source the
  energy changes by (J, pi_W E_h);
* n = 2 everywhere is two successive slabs of half the length;
* a manufactured solution of time degree < min q is reproduced exactly
  with mixed n (S_h vanishes on it);
* the preconditioner inverts the time-derivative part of B_h (the operator
  at dt = 0), and the dual norm matches the Gram matrix of the piecewise
  test functions computed by quadrature."""
import numpy as np
import pytest

import synth
from oracle import basis, brute, fields
from oracle.dg import Discretisation, mass_matrix


def _box(shape, p, q, nk, seed, reorient=False):
    v, h = synth.box_mesh(shape)
    if reorient:
        h = synth.reorient(h, seed=seed)
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    b = lambda x: np.broadcast_to(np.asarray(x), (ne,)).copy()
    return v, h, b(p), b(q), rng.uniform(1, 3, ne), rng.uniform(1, 2, ne), b(nk)


def test_tables_reduce_with_one_subinterval():
    for q in (1, 2, 3):
        D, N = basis.time_tables(q, q)
        assert np.abs(basis.subinterval_time_table(q, 1, q, 1, deriv=True) - D).max() < 1e-14
        assert np.abs(basis.subinterval_time_table(q, 1, q, 1) - N).max() < 1e-14
        for qk in (1, 2, 3):
            _, Nc = basis.time_tables(q, qk)
            Nc = Nc.copy()
            Nc[min(q, qk):, :] = 0.0
            T = basis.subinterval_time_table(q, 1, qk, 1, proj=(min(q, qk), 1))
            assert np.abs(T - Nc).max() < 1e-14


@pytest.mark.parametrize("q,n", [(1, 2), (2, 4), (3, 2)])
def test_flattened_trial_basis(q, n):
    # every level is used once; node values at 0 and 1 sit at levels 0 and 1
    levels = sorted({basis.trial_level(q, n, j, m) for j in range(n) for m in range(q + 1)})
    assert levels == list(range(1 + n * q))
    eps = 1e-9
    V0, _ = basis.subinterval_trial_values(q, n, np.array([eps]))
    V1, _ = basis.subinterval_trial_values(q, n, np.array([1 - eps]))
    assert abs(V0[0, 0] - 1) < 1e-8 and abs(V1[0, 1] - 1) < 1e-8
    # continuity at the interior nodes, and the node functions sum to one
    for j in range(1, n):
        Vl, _ = basis.subinterval_trial_values(q, n, np.array([j / n - eps]))
        Vr, _ = basis.subinterval_trial_values(q, n, np.array([j / n + eps]))
        assert np.abs(Vl - Vr).max() < 1e-7
    s = np.linspace(0.013, 0.987, 29)
    V, dV = basis.subinterval_trial_values(q, n, s)
    nodes = [0, 1] + [1 + j * q for j in range(1, n)]
    assert np.abs(V[:, nodes].sum(axis=1) - 1).max() < 1e-13
    assert np.abs(dV[:, nodes].sum(axis=1)).max() < 1e-12


@pytest.mark.parametrize("p,q,nk", [((1, 1), (1, 1), (1, 2)), ((1, 2), (2, 1), (2, 1)),
                                    ((2, 1), (2, 2), (4, 2)), ((1, 1), (1, 2), (1, 4))])
def test_slab_matrix_matches_brute(p, q, nk):
    v, h, p, q, eps, mu, nk = _box((2, 1, 1), p, q, nk, seed=sum(nk))
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    Bo = d.slab_matrix(0.1).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, 0.1, nk=nk)
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() < 1e-12


def test_slab_matrix_matches_brute_reoriented_mixed():
    v, h, p, q, eps, mu, nk = _box((2, 2, 1), 1, 1, 1, seed=7, reorient=True)
    rng = np.random.default_rng(7)
    p = rng.integers(1, 3, 4)
    q = rng.integers(1, 3, 4)
    nk = np.array([1, 2, 4, 2])
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    Bo = d.slab_matrix(0.07).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, 0.07, nk=nk)
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() < 1e-12


def test_slab_matrix_matches_brute_hanging():
    v, h = synth.hanging_mesh(2, 1)
    ne = h.shape[0]
    rng = np.random.default_rng(1)
    nk = np.where(rng.random(ne) < 0.5, 1, 2)
    p, q = np.ones(ne, np.int64), rng.integers(1, 3, ne)
    eps, mu = rng.uniform(1, 3, ne), rng.uniform(1, 2, ne)
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    Bo = d.slab_matrix(0.1).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, 0.1, nk=nk)
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() < 1e-12


@pytest.mark.parametrize("q,nk", [((1, 1, 1, 1), (1, 2, 4, 1)), ((2, 1, 3, 2), (2, 1, 1, 4)),
                                  ((3, 2, 1, 2), (4, 4, 2, 1))])
def test_energy_conserved(q, nk):
    # Thm 4.1, PEC cavity, J = 0
    v, h, p, q, eps, mu, nk = _box((2, 2, 1), 1, q, nk, seed=3)
    p = np.array([1, 2, 2, 1])
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    s0 = np.random.default_rng(3).standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.2)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) < 1e-12 * e0


def test_planted_unprojected_coupling_breaks_energy(monkeypatch):
    v, h, p, q, eps, mu, nk = _box((2, 2, 1), 1, (2, 1, 3, 2), (2, 1, 1, 4), seed=3)
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)

    def unprojected(e, k, trial=None):
        t = k if trial is None else trial
        return basis.subinterval_time_table(int(d.q[e]), int(d.nk[e]), int(d.q[t]), int(d.nk[t]))

    monkeypatch.setattr(d, "coupling_table", unprojected)
    s0 = np.random.default_rng(3).standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.2)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) > 1e-5 * e0


def test_energy_identity_with_source():
    # E(t_n) - E(t_{n-1}) = (J, pi_W E_h): test function I of an element with n
    # sub-intervals has squared norm dt / n in time, so pi_W E has the
    # coefficients n (N_own e)_I with N_own[I, M] = int_0^1 L_I phi_M ds
    v, h, p, q, eps, mu, nk = _box((2, 2, 2), 2, 2, 1, seed=6)
    nk = np.array([1, 2, 4, 1, 2, 1, 1, 2])
    q = np.array([2, 1, 2, 3, 2, 2, 1, 2])
    d = Discretisation(v, h, p, q, eps, np.ones(8), nk=nk)
    F, J = fields.exp_solution()
    s0 = fields.reference_coefficients(d, F, 0.0)
    dt = 0.15
    L = d.load(J, 0.0, dt)
    U = d.solve_direct(s0, dt, L)
    work = 0.0
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        te = int(d.nt[e])
        _, N = d.own_tables(e)
        Ut = d.split_trial(U, e)[0]
        piE = int(d.nk[e]) * (Ut @ N.T)
        Lb = L[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, te, a3)[0].transpose(0, 2, 1).reshape(3 * a3, te)
        work += np.sum(Lb * piE)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs((e1 - e0) - work) < 1e-11 * max(abs(work), e0)
    assert abs(work) > 1e-2 * e0


def test_uniform_split_is_two_half_slabs():
    v, h, p, q, eps, mu, _ = _box((2, 1, 2), (2, 1, 1, 2), (2, 1, 3, 2), 1, seed=11)
    rng = np.random.default_rng(11)
    d2 = Discretisation(v, h, p, q, eps, mu, nk=np.full(4, 2))
    d1 = Discretisation(v, h, p, q, eps, mu)
    s0 = rng.standard_normal(d1.state_off[-1])
    dt = 0.3
    got = d2.level_state(d2.solve_direct(s0, dt), 1)
    s = d1.level_state(d1.solve_direct(s0, dt / 2), 1)
    ref = d1.level_state(d1.solve_direct(s, dt / 2), 1)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def _state_at(d, U, tau):
    S = np.zeros(d.state_off[-1])
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        te = int(d.nt[e])
        blk = U[d.trial_off[e]:d.trial_off[e + 1]].reshape(2, 3, te + 1, a3)
        V, _ = basis.subinterval_trial_values(int(d.q[e]), int(d.nk[e]), np.array([tau]))
        S[d.state_off[e]:d.state_off[e + 1]] = np.einsum("fcma,m->fca", blk, V[0]).ravel()
    return S


def test_manufactured_solution_reproduced():
    # MS-1, time degree 1 < min q = 2: lies in every common test space
    eps, mu = 2.0, 0.5
    v, h = synth.box_mesh((2, 1, 2))
    d = Discretisation(v, h, np.full(4, 2), np.array([2, 3, 2, 2]), np.full(4, eps), np.full(4, mu),
                       nk=np.array([1, 2, 4, 2]))
    F, J = fields.ms1([0.3, -1.2], eps, mu)
    t0, dt = 0.2, 0.3
    s0 = fields.reference_coefficients(d, F, t0)
    L = d.load(J, t0, dt)
    U = d.solve_direct(s0, dt, L)
    for tau in (1.0 - 1e-12, 0.37, 0.61):
        ref = fields.reference_coefficients(d, F, t0 + tau * dt)
        got = _state_at(d, U, tau)
        assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_preconditioner_inverts_time_derivative_part():
    # at dt = 0 the operator is the time-derivative part P (D kron mass)
    v, h, p, q, eps, mu, nk = _box((2, 1, 1), (1, 2), (2, 3), (4, 2), seed=12)
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    y = np.random.default_rng(12).standard_normal(d.unk_off[-1])
    got = d.operator(d.precond_solve(y), 0.0)
    assert np.abs(got - y).max() < 1e-12 * np.abs(y).max()
    # the centre-metric variant is the same on these affine elements
    assert np.abs(d.precond_centre_solve(y) - d.precond_solve(y)).max() < 1e-12 * np.abs(d.precond_solve(y)).max()


def test_dual_norm_against_quadrature_gram():
    v, h, p, q, eps, mu, nk = _box((2, 1, 1), (1, 2), (2, 1), (2, 4), seed=13)
    d = Discretisation(v, h, p, q, eps, mu, nk=nk)
    R = np.random.default_rng(13).standard_normal(d.unk_off[-1])
    dt = 0.25
    ref = np.zeros(2)
    for e in range(d.ne):
        a = int(d.a[e])
        a3 = a ** 3
        te = int(d.nt[e])
        # Gram matrix of the element's test functions in L2(I_n) by quadrature
        n = int(d.nk[e])
        s = ((np.arange(n)[:, None] + basis.gauss01(8)[0][None, :]) / n).ravel()
        w = np.tile(basis.gauss01(8)[1], n) / n
        Tv = basis.subinterval_test_values(int(d.q[e]), n, s)
        Gt = dt * (Tv * w[:, None]).T @ Tv
        G = np.kron(Gt, mass_matrix(d.X(e), a, 1.0, a + 1))      # rows (I, (c, s)) per field
        blk = R[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, te, a3)
        for f in range(2):
            r = blk[f].transpose(1, 0, 2).reshape(te * 3 * a3)
            ref[f] += r @ np.linalg.solve(G, r)
    got = d.dual_norms(R, dt)
    assert np.abs(got - ref).max() < 1e-12 * ref.max()


@pytest.mark.parametrize("n_slabs", [1, 3])
def test_eta_it_bounds_the_iteration_error(n_slabs):
    # Section 5.3 with the dual norm of the piecewise test space (dt / n per
    # test level): eta_it still bounds the iteration error of inexact slab
    # solutions with mixed sub-intervals (the stability behind it is Thm 4.1)
    v, h = synth.box_mesh((2, 2, 1), hi=(0.6, 0.5, 0.3))
    rng = np.random.default_rng(30 + n_slabs)
    d = Discretisation(v, h, np.full(4, 2), rng.integers(1, 4, 4), rng.uniform(1, 4, 4), rng.uniform(1, 2, 4),
                       nk=np.array([4, 2, 1, 2]))
    dt = 0.05
    s_exact = rng.standard_normal(d.state_off[-1])
    s_inexact = s_exact.copy()
    eta2 = 0.0
    for n in range(n_slabs):
        U_ex = d.solve_direct(s_exact, dt)
        U_in = d.solve_direct(s_inexact, dt)
        x = d.unknowns_of(U_in) + 1e-3 * rng.standard_normal(d.unk_off[-1])
        U_in = d.embed_unknowns(x, s_inexact)
        R = d.residual(U_in, dt) - d.residual(d.solve_direct(s_inexact, dt), dt)
        eta2 += d.eta_it_term(R, dt, n_slabs * dt)
        s_exact = d.level_state(U_ex, 1)
        s_inexact = d.level_state(U_in, 1)
    err2 = 2.0 * d.energy(s_inexact - s_exact)
    assert err2 <= eta2, (err2, eta2)
    assert err2 > 1e-4 * eta2


@pytest.mark.parametrize("q,nk", [(1, (1, 2)), (2, (1, 2)), (2, (2, 4))])
def test_temporal_order_with_local_time_steps(q, nk):
    # Section 6.1.2 (local refinement in time): the manufactured exp solution
    # (spatial part exact for p = 2) keeps the nodal order 2 q when elements
    # take different numbers of sub-intervals
    F, J = fields.exp_solution()
    v, h = synth.box_mesh((2, 1, 1))
    d = Discretisation(v, h, np.full(2, 2), np.full(2, q), np.ones(2), np.ones(2), nk=np.array(nk))
    T = 0.4
    errs = []
    for nsteps in (2, 4):
        dt = T / nsteps
        s = fields.reference_coefficients(d, F, 0.0)
        for n in range(nsteps):
            s = d.level_state(d.solve_direct(s, dt, d.load(J, n * dt, dt, nt=q + 8)), 1)
        errs.append(np.abs(s - fields.reference_coefficients(d, F, T)).max())
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - 2 * q) < 0.3, (errs, rate)


@pytest.mark.parametrize("nk", [(1, 2, 4, 1), (2, 1, 2, 4)])
def test_dissipation_with_local_time_steps(nk):
    # D_h (remark closing Section 4) with the test function projected onto the
    # common temporal test space of each face's pair: the slab matrix against
    # the brute-force assembler on a sheared mesh, and the energy decreases
    v, h = synth.box_mesh((2, 2, 1))
    v = synth.affine_transform(v, np.array([[1.0, 0.2, -0.1], [0.1, 0.9, 0.15], [-0.05, 0.1, 1.1]]))
    rng = np.random.default_rng(sum(nk))
    p, q = rng.integers(1, 3, 4), rng.integers(1, 3, 4)
    eps, mu = rng.uniform(1, 3, 4), rng.uniform(1, 2, 4)
    d = Discretisation(v, h, p, q, eps, mu, c_diss=0.7, nk=np.array(nk))
    Bo = d.slab_matrix(0.1).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, 0.1, c_diss=0.7, nk=np.array(nk))
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() < 1e-12
    s0 = rng.standard_normal(d.state_off[-1])
    e1 = d.energy(d.level_state(d.solve_direct(s0, 0.1), 1))
    assert e1 < d.energy(s0)
