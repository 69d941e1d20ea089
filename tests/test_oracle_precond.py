"""Pins of the oracle's block preconditioners (Section 5.4, eq. preconditioner).

P is the time-derivative part of the slab operator restricted to the unknowns:
the identity in time kron the element mass.  precond_solve inverts the
quadrature mass exactly; precond_centre_solve uses the metric at the element
centre.  With an orthonormal basis and a constant metric (affine elements) the
mass is G (x) I exactly, so both must agree there; on trilinear elements the
centre metric is only an approximation and they must differ."""
import numpy as np

import synth
from oracle.dg import Discretisation


def _disc(v, h, seed):
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    return Discretisation(v, h, rng.integers(1, 4, ne), rng.integers(1, 3, ne),
                          rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


def test_centre_metric_is_exact_on_sheared_affine_elements():
    v, h = synth.box_mesh((2, 2, 1))
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    d = _disc(synth.affine_transform(v, A), h, 3)
    y = np.random.default_rng(4).standard_normal(d.unk_off[-1])
    exact = d.precond_solve(y)
    centre = d.precond_centre_solve(y)
    assert np.linalg.norm(centre - exact) < 1e-12 * np.linalg.norm(exact)
    # and P itself: the mass applied to the centre solve gives back y
    e = 2
    a3 = int(d.a[e]) ** 3
    qe = int(d.q[e])
    blk = centre[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)
    M = d.mass(e, "eps")
    back = (M @ blk[0].transpose(0, 2, 1).reshape(3 * a3, qe)).reshape(3, a3, qe).transpose(0, 2, 1)
    ye = y[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)[0]
    assert np.allclose(back, ye, rtol=0, atol=1e-12 * np.abs(ye).max())


def test_centre_metric_differs_on_trilinear_elements():
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.25, 1)
    d = _disc(v, h, 5)
    y = np.random.default_rng(6).standard_normal(d.unk_off[-1])
    exact = d.precond_solve(y)
    centre = d.precond_centre_solve(y)
    rel = np.linalg.norm(centre - exact) / np.linalg.norm(exact)
    assert 1e-4 < rel < 0.5
