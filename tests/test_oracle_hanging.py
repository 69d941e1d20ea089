"""Pins of the oracle on 2:1 nonconforming meshes (hanging faces; Section 5.2
sums the flux terms of a face over the neighbours that share parts of it).

* detection: every coarse face against four fine faces, the face maps halve
  or double the face coordinates and send the quarter's corners to the fine
  face's corners;
* the oracle's slab matrix (reference-space face matrices restricted to the
  quarters, covariant components scaled by the face map) equals the
  separately written physical-space brute-force assembler, including mixed
  p and q across the hanging faces and reoriented fine elements;
* energy conservation without sources (Thm 3.1, 4.1: the centred fluxes of
  the two sides of every face piece cancel in B_h(U, pi U));
* a planted mistake (the quarters of one coarse face swapped) breaks the
  brute comparison."""
import numpy as np
import pytest

import synth
from oracle import brute
from oracle.dg import Discretisation
from oracle.geometry import face_topology, face_vertices, hanging_faces


def _mesh(n=2, split=1, p=2, q=1, seed=0, reorient=False):
    v, h = synth.hanging_mesh(n, split)
    if reorient:
        h = synth.reorient(h, seed=seed)
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    p = np.broadcast_to(np.asarray(p), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q), (ne,)).copy()
    return v, h, p, q, rng.uniform(1, 4, ne), rng.uniform(1, 2, ne)


def test_detection_and_face_maps():
    v, h = synth.hanging_mesh(2, 1)
    nb, nbf, _ = face_topology(h)
    hang = hanging_faces(v, h, nb)
    coarse = {k: e for k, e in hang.items() if e[0][4] is not None}
    fine = {k: e for k, e in hang.items() if e[0][4] is None}
    assert len(coarse) == 4 and len(fine) == 16
    for (e, f), entries in coarse.items():
        assert len(entries) == 4
        assert sorted(x[4] for x in entries) == [(0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]
        for k, fk, A, b, sub in entries:
            assert sorted(np.abs(A).ravel().tolist()) == [0.0, 0.0, 2.0, 2.0]
            # the quarter's corners, in the coarse face's coordinates, land on the
            # fine face's corners (0/1 coordinates) and match its vertices
            own = face_vertices(h[e], f)
            fverts = face_vertices(h[k], fk)
            P = v[own]
            for iv in range(2):
                for iu in range(2):
                    uv = np.array([sub[0] + 0.5 * iu, sub[1] + 0.5 * iv])
                    uvp = A @ uv + b
                    assert np.allclose(uvp, np.round(uvp)) and np.all((uvp > -1e-12) & (uvp < 1 + 1e-12))
                    s, t = uv
                    x = (1 - s) * (1 - t) * P[0] + s * (1 - t) * P[1] + (1 - s) * t * P[2] + s * t * P[3]
                    j = int(round(uvp[0])) + 2 * int(round(uvp[1]))
                    assert np.allclose(v[fverts[j]], x)
            back = hang[(k, fk)]
            assert len(back) == 1 and back[0][0] == e and back[0][1] == f
            assert np.allclose(back[0][2] @ A, np.eye(2))


def _compare(v, h, p, q, eps, mu, dt, tol=1e-12):
    d = Discretisation(v, h, p, q, eps, mu)
    Bo = d.slab_matrix(dt).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, dt)
    err = np.abs(Bo - Bb).max() / np.abs(Bb).max()
    assert err < tol, err
    return d, Bo, Bb


def test_slab_matrix_matches_brute_uniform():
    _compare(*_mesh(2, 1, p=2, q=1, seed=1), 0.1)


def test_slab_matrix_matches_brute_mixed_degrees_and_orientations():
    v, h, p, q, eps, mu = _mesh(2, 1, seed=2, reorient=True)
    rng = np.random.default_rng(2)
    p = rng.integers(1, 4, h.shape[0])
    q = rng.integers(1, 3, h.shape[0])
    _compare(v, h, p, q, eps, mu, 0.07)


@pytest.mark.parametrize("qs", [(1, 1), (2, 2), (1, 2)])
def test_energy_conserved(qs):
    v, h, p, q, eps, mu = _mesh(2, 1, p=2, seed=3)
    rng = np.random.default_rng(3)
    q = np.where(rng.random(h.shape[0]) < 0.5, qs[0], qs[1])
    p = rng.integers(1, 3, h.shape[0])
    d = Discretisation(v, h, p, q, eps, mu)
    s0 = rng.standard_normal(d.state_off[-1])
    U = d.solve_direct(s0, 0.1)
    e0, e1 = d.energy(d.level_state(U, 0)), d.energy(d.level_state(U, 1))
    assert abs(e1 - e0) < 1e-12 * e0


def test_planted_quarter_swap_is_caught():
    v, h, p, q, eps, mu = _mesh(2, 1, p=1, q=1, seed=4)
    d = Discretisation(v, h, p, q, eps, mu)
    (e, f), entries = next((k, x) for k, x in d.hang.items() if x[0][4] is not None)
    # swap which fine element covers the first two quarters
    a0, a1 = entries[0], entries[1]
    entries[0] = (a1[0], a1[1], a0[2], a0[3], a0[4])
    entries[1] = (a0[0], a0[1], a1[2], a1[3], a1[4])
    Bo = d.slab_matrix(0.1).toarray()
    Bb = brute.assemble(v, h, p, q, eps, mu, 0.1)
    assert np.abs(Bo - Bb).max() / np.abs(Bb).max() > 1e-3
