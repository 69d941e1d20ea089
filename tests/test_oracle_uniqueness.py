"""Uniqueness of the mixed-q slab problems the tests solve.

With a uniform temporal degree the slab system is nonsingular (Lemma 3.3 with
zero data gives U = 0).  With mixed q the paper proves only the energy
identity (Thm 4.1), which does not exclude a null space, so every mixed-q slab
matrix that a test solves (built here by the same recipe and seed) is checked
directly: its smallest singular value on the unknown columns is bounded away
from zero.  Small systems use a dense SVD (backward stable: the computed
sigma_min is within ~1e-16 sigma_max of the true one); larger ones use
shift-invert Lanczos on B^T B through a sparse LU, which agrees with the
dense SVD on a mixed 8-element mesh to 1e-10."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle.dg import Discretisation

DENSE_MAX = 3000  # unknowns up to which sigma_min comes from a dense SVD


def _square(d, dt):
    B = d.slab_matrix(dt)
    return B[:, d.unknown_columns()].tocsc()


def _sigma_dense(Bu):
    s = sla.svdvals(Bu.toarray())
    return s.min(), s.max()


def _sigma_min_sparse(Bu):
    lu = spla.splu(Bu)
    n = Bu.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(lu.solve(v, trans="T")), dtype=float)
    w, _ = spla.eigsh(op, k=1, which="LA", tol=1e-12)
    return 1.0 / np.sqrt(w[0])


def _mixed_box_321(seed, perturb=None):
    v, h = synth.box_mesh((3, 2, 2))
    if perturb is not None:
        v = synth.perturb_interior(v, (3, 2, 2), perturb[0], perturb[1])
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    return Discretisation(v, h, rng.integers(1, 4, ne), rng.integers(1, 4, ne),
                          rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


def _cases():
    out = []
    # GPU slab solve with mixed degrees and a source (affine 3x2x2, seed 21, dt 0.04)
    out.append(("affine 3x2x2 mixed p,q", lambda: _mixed_box_321(21), 0.04))
    # the same on a trilinear mesh (perturbed 0.2, seed 14; degrees seed 15)
    out.append(("trilinear 3x2x2 mixed p,q", lambda: _mixed_box_321(15, (0.2, 14)), 0.04))

    def energy_case(qs):
        rng = np.random.default_rng(2)
        v, h = synth.box_mesh((2, 2, 2))
        return Discretisation(v, h, np.array([2, 1, 1, 2, 2, 1, 1, 2]), np.array([qs[0], qs[1]] * 4),
                              rng.uniform(1, 4, 8), rng.uniform(1, 2, 8))
    for qs in ((1, 3), (2, 1)):
        out.append(("energy 2x2x2 q=%s" % (qs,), lambda qs=qs: energy_case(qs), 0.15))

    def trilinear_energy():
        v, h = synth.box_mesh((2, 2, 2))
        v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=4)
        rng = np.random.default_rng(5)
        return Discretisation(v, h, np.full(8, 2), np.array([1, 2] * 4), rng.uniform(1, 3, 8), np.ones(8))
    out.append(("trilinear energy 2x2x2", trilinear_energy, 0.1))

    def ms2():
        v, h = synth.box_mesh((2, 2, 2))
        v = synth.perturb_interior(v, (2, 2, 2), 0.2, seed=8)
        return Discretisation(v, h, np.full(8, 3), np.array([1, 2, 3, 1, 2, 1, 3, 2]), np.full(8, 1.5),
                              np.full(8, 0.7))
    out.append(("MS-2 trilinear q=1..3", ms2, 0.25))

    def dissipative():
        v, h = synth.box_mesh((2, 2, 2))
        rng = np.random.default_rng(34)
        return Discretisation(v, h, np.full(8, 2), np.array([1, 2] * 4), rng.uniform(1, 3, 8),
                              rng.uniform(1, 2, 8), c_diss=0.7)
    out.append(("dissipative 2x2x2 c=0.7", dissipative, 0.15))
    return out


@pytest.mark.parametrize("name,make,dt", _cases(), ids=[c[0] for c in _cases()])
def test_mixed_q_slab_matrix_is_nonsingular(name, make, dt):
    d = make()
    assert len(set(int(v) for v in d.q)) > 1
    Bu = _square(d, dt)
    if Bu.shape[0] <= DENSE_MAX:
        smin, smax = _sigma_dense(Bu)
    else:
        smin = _sigma_min_sparse(Bu)
        smax = spla.svds(Bu, k=1, which="LM", return_singular_vectors=False)[0]
    assert smin > 1e-6 * smax, (name, smin, smax)


def test_serving_trilinear_mixed_q_is_nonsingular():
    # the 27-element trilinear serving request (perturbed 0.1, seed 21), dt 0.02
    v, h = synth.box_mesh((3, 3, 3))
    v = synth.perturb_interior(v, (3, 3, 3), 0.1, seed=21)
    rng = np.random.default_rng(21)
    p = rng.integers(1, 4, 27)
    q = rng.integers(1, 3, 27)
    d = Discretisation(v, h, p, q, rng.uniform(1, 3, 27), np.ones(27))
    assert len(set(int(v) for v in q)) > 1
    Bu = _square(d, 0.02)
    smin = _sigma_min_sparse(Bu)
    smax = spla.svds(Bu, k=1, which="LM", return_singular_vectors=False)[0]
    assert smin > 1e-6 * smax, (smin, smax)


def test_sparse_estimate_matches_dense_svd():
    v, h = synth.box_mesh((2, 2, 2))
    rng = np.random.default_rng(9)
    d = Discretisation(v, h, rng.integers(1, 3, 8), rng.integers(1, 4, 8), rng.uniform(1, 4, 8),
                       rng.uniform(1, 2, 8))
    Bu = _square(d, 0.1)
    assert 500 < Bu.shape[0] <= DENSE_MAX
    smin, _ = _sigma_dense(Bu)
    assert abs(_sigma_min_sparse(Bu) - smin) < 1e-10 * smin
