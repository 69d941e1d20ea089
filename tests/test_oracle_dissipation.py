"""Pins of the oracle's dissipative stabilisation D_h (the remark at the end of
Section 4: upwind-type face terms alpha_E [E]_T . [pi v]_T on interior faces,
alpha_E [E]_T . [v]_T on PEC faces, alpha_H [H]_T . [pi w]_T on interior faces,
alpha_E = c / {sqrt(mu/eps)}, alpha_H = c / {sqrt(eps/mu)}):

* its slab blocks against the physical-space brute-force assembler, which
  integrates the face terms with the physical normal and the time projection
  by quadrature (affine, sheared, trilinear, mixed p and q, jumps in eps, mu);
* the energy balance stated with it: without sources the energy drops by
  exactly D_h(U, pi_W U) = int alpha_E |[pi E]_T|^2 + ..., which is > 0;
* consistency: solutions inside the discrete space with continuous tangential
  traces and PEC walls are still reproduced exactly (the jumps vanish);
* c = 0 gives the non-dissipative operator unchanged.
"""
import numpy as np
import pytest

import synth
from oracle import brute, fields
from oracle.dg import Discretisation


def _compare(v, h, p, q, eps, mu, dt, c, tol, mass_nq=None, **kw):
    d0 = Discretisation(v, h, p, q, eps, mu, mass_nq=mass_nq)
    dc = Discretisation(v, h, p, q, eps, mu, mass_nq=mass_nq, c_diss=c)
    Bo = dc.slab_matrix(dt).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, dt, c_diss=c, **kw)
    scale = np.abs(Bb).max()
    assert np.abs(Bo - Bb).max() / scale < tol
    # the dissipative part itself is a sizeable change
    D = Bo - d0.slab_matrix(dt).toarray()
    Db = Bb - brute.assemble(v, h, p, q, eps, mu, dt, **kw)
    assert np.abs(D).max() > 1e-2 * scale
    assert np.abs(D - Db).max() / np.abs(Db).max() < tol


def test_single_element_boundary_terms():
    v, h = synth.box_mesh((1, 1, 1), hi=(0.7, 0.4, 1.3))
    _compare(v, h, [2], [2], [2.0], [3.0], 0.1, 0.8, 1e-12)


def test_two_elements_mixed_p_q_and_materials():
    v, h = synth.box_mesh((2, 1, 1), hi=(1.0, 0.5, 0.5))
    _compare(v, h, [1, 2], [1, 3], [1.0, 4.0], [1.0, 2.0], 0.05, 1.3, 1e-12)


def test_two_elements_each_axis():
    for shape in ((1, 2, 1), (1, 1, 2)):
        v, h = synth.box_mesh(shape)
        _compare(v, h, [2, 1], [2, 1], [1.0, 2.0], [2.0, 1.0], 0.2, 0.5, 1e-12)


def test_sheared_affine_cube():
    v, h = synth.box_mesh((2, 2, 2))
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    v = synth.affine_transform(v, A)
    rng = np.random.default_rng(11)
    _compare(v, h, [2, 1, 2, 1, 1, 2, 1, 2], [1, 2, 2, 1, 1, 2, 2, 1],
             rng.uniform(1, 3, 8), rng.uniform(1, 3, 8), 0.07, 0.9, 1e-12)


def test_trilinear_perturbed():
    v, h = synth.box_mesh((2, 1, 1), hi=(1.0, 0.5, 0.5))
    rng = np.random.default_rng(12)
    v = v + rng.uniform(-0.04, 0.04, v.shape)
    _compare(v, h, [2, 1], [2, 1], [1.5, 1.0], [1.0, 2.5], 0.05, 1.1, 1e-9,
             mass_nq=14, nvol_extra=12, nface_extra=10)


def _pi_w(d, U):
    """pi_W U in the residual layout: the trial field projected in time onto
    the element's test space (coefficients N U against the orthonormal L_i)."""
    out = np.zeros(d.unk_off[-1])
    for e in range(d.ne):
        qe, a3 = int(d.q[e]), int(d.a[e]) ** 3
        _, N = d.tables(qe, qe)
        blk = U[d.trial_off[e]:d.trial_off[e + 1]].reshape(2, 3, qe + 1, a3)
        out[d.unk_off[e]:d.unk_off[e + 1]] = np.einsum("im,fcma->fcia", N, blk).ravel()
    return out


@pytest.mark.parametrize("qs", [(2, 2), (1, 3)])
def test_energy_drops_by_the_dissipation(qs):
    rng = np.random.default_rng(13)
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.1, seed=14) if qs == (1, 3) else v
    p = np.array([2, 1, 1, 2, 2, 1, 1, 2])
    q = np.array([qs[0], qs[1]] * 4)
    eps, mu = rng.uniform(1, 4, 8), rng.uniform(1, 2, 8)
    dc = Discretisation(v, h, p, q, eps, mu, c_diss=0.7)
    d0 = Discretisation(v, h, p, q, eps, mu)
    s0 = rng.standard_normal(dc.state_off[-1])
    dt = 0.15
    U = dc.solve_direct(s0, dt)
    # D_h(U, .) rows: the dissipative operator's residual minus the plain one
    Drows = dc.residual(U, dt) - d0.residual(U, dt)
    diss = Drows @ _pi_w(dc, U)
    e0, e1 = dc.energy(dc.level_state(U, 0)), dc.energy(dc.level_state(U, 1))
    assert diss > 1e-3 * e0
    assert abs((e1 - e0) + diss) < 1e-11 * e0


def test_manufactured_solutions_still_reproduced():
    # MS-1 on axis-aligned boxes (tangential traces continuous, n x E = 0 on the walls)
    eps, mu = 2.0, 0.5
    v, h = synth.box_mesh((2, 1, 2))
    d = Discretisation(v, h, np.full(4, 2), np.full(4, 2), np.full(4, eps), np.full(4, mu), c_diss=1.5)
    F, J = fields.ms1([0.3, -1.2], eps, mu)
    t0, dt = 0.2, 0.3
    s0 = fields.reference_coefficients(d, F, t0)
    U = d.solve_direct(s0, dt, d.load(J, t0, dt))
    ref = fields.reference_coefficients(d, F, t0 + dt)
    assert np.abs(d.level_state(U, 1) - ref).max() < 1e-11 * np.abs(ref).max()
    # MS-2: static H on a trilinear mesh with mixed q (E = 0 on the walls)
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.2, seed=8)
    q = np.array([1, 2, 3, 1, 2, 1, 3, 2])
    d = Discretisation(v, h, np.full(8, 3), q, np.full(8, 1.5), np.full(8, 0.7), c_diss=2.0)
    F, J = fields.ms2()
    s0 = fields.reference_coefficients(d, F, 0.0)
    U = d.solve_direct(s0, 0.25, d.load(J, 0.0, 0.25))
    assert np.abs(d.level_state(U, 1) - s0).max() < 1e-11 * np.abs(s0).max()


def test_c_zero_is_the_plain_operator():
    v, h = synth.box_mesh((2, 1, 1))
    args = (v, h, [2, 1], [2, 1], [1.0, 2.0], [1.0, 1.0])
    a = Discretisation(*args).slab_matrix(0.1)
    b = Discretisation(*args, c_diss=0.0).slab_matrix(0.1)
    assert (a != b).nnz == 0
