"""Pins of the oracle on conforming meshes whose neighbours meet in any
orientation (element vertex numbers relabelled by random cube rotations:
face axes swapped and reversed between neighbours; the face coupling of
Section 5.2 with the permutations of the face parametrisation):

* the slab matrix against the physical-space brute-force assembler, which
  finds neighbour points by inverting the neighbour's map and so needs no
  orientation logic (affine, sheared, trilinear; mixed p, q; with D_h);
* the same physical problem numbered two ways gives the same discrete
  solution: energies and L2 errors against the exact field agree after a
  slab (TE101, mixed degrees, a two-material sheared mesh);
* energy conservation (Thm 3.1, 4.1) on a reoriented trilinear mesh.
"""
import numpy as np
import pytest

import synth
from oracle import brute, fields
from oracle.dg import Discretisation
from oracle.geometry import face_topology


def _compare(v, h, p, q, eps, mu, dt, tol, c=0.0, mass_nq=None, **kw):
    d = Discretisation(v, h, p, q, eps, mu, mass_nq=mass_nq, c_diss=c)
    assert len(d.fmap) > 0                      # some faces really are permuted
    Bo = d.slab_matrix(dt).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, dt, c_diss=c, **kw)
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() < tol


def test_rotations_cover_every_face_map():
    # every symmetry of the square (8) appears between neighbours of a
    # reoriented 3x3x3 lattice
    v, h = synth.box_mesh((3, 3, 3))
    h = synth.reorient(h, seed=0)
    d = Discretisation(v, h, np.full(27, 1), np.full(27, 1), np.ones(27), np.ones(27))
    maps = {(tuple(A.ravel()), tuple(b)) for A, b in d.fmap.values()}
    assert len(maps) == 8                       # the identity too, on faces of other axes
    nb, nbf, canon = face_topology(h)
    assert (~canon[nb >= 0]).sum() > 0 and (nbf[nb >= 0] // 2 != np.nonzero(nb >= 0)[1] // 2).any()


def test_box_mixed_degrees():
    v, h = synth.box_mesh((2, 2, 1), hi=(1.0, 0.8, 0.5))
    h = synth.reorient(h, seed=1)
    _compare(v, h, [1, 2, 2, 1], [1, 2, 3, 2], [1.0, 2.0, 3.0, 1.5], [1.0, 1.5, 1.0, 2.0], 0.07, 1e-12)


def test_sheared_affine():
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.affine_transform(v, np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]]))
    h = synth.reorient(h, seed=2)
    rng = np.random.default_rng(2)
    _compare(v, h, [2, 1, 2, 1, 1, 2, 1, 2], [1, 2, 2, 1, 1, 2, 2, 1], rng.uniform(1, 3, 8), rng.uniform(1, 3, 8),
             0.07, 1e-12)


def test_with_dissipation():
    v, h = synth.box_mesh((2, 2, 1), hi=(0.6, 1.0, 0.7))
    h = synth.reorient(h, seed=3)
    _compare(v, h, [2, 1, 2, 2], [2, 1, 2, 3], [1.0, 4.0, 2.0, 1.0], [2.0, 1.0, 1.0, 1.5], 0.05, 1e-12, c=0.9)


def test_trilinear():
    v, h = synth.box_mesh((2, 1, 1), hi=(1.0, 0.5, 0.5))
    rng = np.random.default_rng(4)
    v = v + rng.uniform(-0.04, 0.04, v.shape)
    h = synth.reorient(h, seed=5)
    _compare(v, h, [2, 1], [2, 1], [1.5, 1.0], [1.0, 2.5], 0.05, 1e-9, mass_nq=14, nvol_extra=12, nface_extra=10)


@pytest.mark.parametrize("case", ["te101", "mixed", "sheared"])
def test_numbering_does_not_change_the_solution(case):
    rng = np.random.default_rng(6)
    if case == "sheared":
        v, h = synth.box_mesh((2, 2, 2))
        v = synth.affine_transform(v, np.array([[1.0, 0.2, 0.0], [0.0, 1.0, 0.1], [0.1, 0.0, 1.0]]))
        p, q = np.full(8, 2), np.array([1, 2] * 4)
        eps, mu = rng.uniform(1, 3, 8), rng.uniform(1, 2, 8)
        F = fields.mode_superposition(np.array([[1, 0, 1], [1, 1, 1]]), np.array([[0.0, 1.0, 0.0], [1.0, -1.0, 0.5]]))
    else:
        v, h = synth.box_mesh((2, 2, 2))
        ne = 8
        p = np.full(ne, 2) if case == "te101" else rng.integers(1, 4, ne)
        q = np.full(ne, 1) if case == "te101" else rng.integers(1, 4, ne)
        eps = np.ones(ne) if case == "te101" else rng.uniform(1, 3, ne)
        mu = np.ones(ne)
        F = fields.te101
    h2 = synth.reorient(h, seed=7)
    out = []
    for hh in (h, h2):
        d = Discretisation(v, hh, p, q, eps, mu)
        s = fields.project(d, F, 0.0)
        s1 = d.level_state(d.solve_direct(s, 0.1), 1)
        out.append((d.energy(s), d.energy(s1), fields.l2_error(d, s1, F, 0.1)))
    (e0a, e1a, la), (e0b, e1b, lb) = out
    assert abs(e0a - e0b) < 1e-13 * e0a and abs(e1a - e1b) < 1e-12 * e0a
    assert abs(la - lb) < 1e-10 * max(la, 1e-300) and la > 0


def test_energy_conserved_reoriented_trilinear():
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=8)
    h = synth.reorient(h, seed=9)
    rng = np.random.default_rng(10)
    d = Discretisation(v, h, np.full(8, 2), np.array([1, 2] * 4), rng.uniform(1, 3, 8), np.ones(8))
    s0 = rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.1)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) < 1e-12 * e0


def test_relabelling_keeps_the_physical_mesh():
    # every rotated element has the same vertex set and volume, and a face
    # that does not match as a quadrilateral is refused
    from oracle.geometry import face_map, face_vertices, jacobian
    v, h = synth.box_mesh((2, 2, 2))
    h2 = synth.reorient(h, seed=11)
    for e in range(h.shape[0]):
        assert sorted(h[e]) == sorted(h2[e])
        det = np.linalg.det(jacobian(v[h2[e]], np.array([0.5, 0.5, 0.5])))
        assert abs(det - np.linalg.det(jacobian(v[h[e]], np.array([0.5, 0.5, 0.5])))) < 1e-14
    # element 1 meets element 0 across its face 0 (reference x = 0, corners
    # 0, 2, 4, 6); two adjacent corners exchanged make the shared quadrilateral
    # a bow-tie in element 1's numbering
    assert sorted(face_vertices(h[0], 1)) == sorted(face_vertices(h[1], 0))
    twisted = h[1].copy()
    twisted[[0, 2]] = twisted[[2, 0]]
    with pytest.raises(ValueError):
        face_map(h[0], 1, twisted, 0)
