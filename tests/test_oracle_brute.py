"""Pin of the oracle's slab matrix (reference-space local matrices, derived face
weights and S_h truncation) against the separately written physical-space
brute-force assembler of C_h + S_h (Section 2.5 eq. bilinearform:C, Section
4.1 eq. bilinearform:S)."""
import numpy as np
import pytest

import synth
from oracle import brute
from oracle.dg import Discretisation


def _compare(v, h, p, q, eps, mu, dt, tol, mass_nq=None, **kw):
    disc = Discretisation(v, h, p, q, eps, mu, mass_nq=mass_nq)
    Bo = disc.slab_matrix(dt).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, dt, **kw)
    scale = np.abs(Bb).max()
    err = np.abs(Bo - Bb).max() / scale
    assert err < tol, err
    return Bo


def test_single_box_element():
    v, h = synth.box_mesh((1, 1, 1), hi=(0.7, 0.4, 1.3))
    _compare(v, h, [2], [2], [2.0], [3.0], 0.1, 1e-12)


def test_two_elements_mixed_p_and_q():
    # p differs (face truncation) and q differs (S_h) across the shared face
    v, h = synth.box_mesh((2, 1, 1), hi=(1.0, 0.5, 0.5))
    _compare(v, h, [1, 2], [1, 3], [1.0, 4.0], [1.0, 2.0], 0.05, 1e-12)


def test_two_elements_mixed_q_each_axis():
    for shape in ((1, 2, 1), (1, 1, 2)):
        v, h = synth.box_mesh(shape)
        _compare(v, h, [2, 1], [2, 1], [1.0, 2.0], [2.0, 1.0], 0.2, 1e-12)


def test_sheared_affine_cube():
    v, h = synth.box_mesh((2, 2, 2))
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    v = synth.affine_transform(v, A)
    p = [2, 1, 2, 1, 1, 2, 1, 2]
    q = [1, 2, 2, 1, 1, 2, 2, 1]
    rng = np.random.default_rng(3)
    _compare(v, h, p, q, rng.uniform(1, 3, 8), rng.uniform(1, 3, 8), 0.07, 1e-12)


def test_trilinear_perturbed():
    # non-affine: physical integrands are rational, so agreement is limited by
    # the quadrature of both sides; both use high-order rules here.
    v, h = synth.box_mesh((2, 1, 1), hi=(1.0, 0.5, 0.5))
    rng = np.random.default_rng(7)
    v = v + rng.uniform(-0.04, 0.04, v.shape)
    _compare(v, h, [2, 1], [2, 1], [1.5, 1.0], [1.0, 2.5], 0.05, 1e-9,
             mass_nq=14, nvol_extra=12, nface_extra=10)


def test_boundary_only_terms_sign():
    # a single element: every face is a PEC boundary face with weight 1
    v, h = synth.box_mesh((1, 1, 1))
    _compare(v, h, [1], [1], [1.0], [1.0], 0.3, 1e-12)
