"""Pins of the oracle's block preconditioners (Section 5.4, eq. preconditioner).

P is the time-derivative part of the slab operator restricted to the unknowns:
the identity in time kron the element mass.  precond_solve inverts the
quadrature mass exactly; precond_centre_solve uses the metric at the element
centre.  With an orthonormal basis and a constant metric (affine elements) the
mass is G (x) I exactly, so both must agree there; on trilinear elements the
centre metric is only an approximation and they must differ."""
import numpy as np
import pytest

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


# ---------------------------------------------------------------------------
# The centre metric itself on trilinear elements, pinned by an independent
# construction: at the centre of the reference cube the derivative of the
# trilinear map along axis m is the mean of the element's four edges parallel
# to that axis (every shape-function derivative there is +-1/4), so
# DF(1/2, 1/2, 1/2) follows from the vertices by differences alone.  It is
# cross-checked with the physical-space assembler's own geometry routine.
# ---------------------------------------------------------------------------

def _centre_jacobian_from_edges(X):
    DF = np.zeros((3, 3))
    for m in range(3):
        edges = [X[v | (1 << m)] - X[v] for v in range(8) if not (v >> m) & 1]
        DF[:, m] = np.mean(edges, axis=0)
    return DF


def _centre_pin_residual(d, y):
    """max over elements and fields of |kappa G_c z - y| / |y| for
    z = precond_centre_solve(y), G_c from the edge construction."""
    z = d.precond_centre_solve(y)
    worst = 0.0
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        DF = _centre_jacobian_from_edges(d.X(e))
        Di = np.linalg.inv(DF)
        G = np.linalg.det(DF) * Di @ Di.T
        zb = z[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe * a3)
        yb = y[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe * a3)
        for f, kap in ((0, d.eps[e]), (1, d.mu[e])):
            back = kap * G @ zb[f]
            worst = max(worst, np.abs(back - yb[f]).max() / np.abs(yb[f]).max())
    return worst


def _trilinear_disc():
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.25, 1)
    return _disc(v, h, 5)


def test_centre_metric_on_trilinear_elements_pinned_by_edge_means():
    d = _trilinear_disc()
    y = np.random.default_rng(6).standard_normal(d.unk_off[-1])
    assert _centre_pin_residual(d, y) < 1e-13
    # the edge construction agrees with the brute-force assembler's geometry
    from oracle.brute import _Element
    for e in range(d.ne):
        _, DF, _ = _Element(d.X(e), 2).geometry(np.array([[0.5, 0.5, 0.5]]))
        assert np.abs(DF[0] - _centre_jacobian_from_edges(d.X(e))).max() < 1e-15


@pytest.mark.parametrize("mistake", ["corner", "transposed"])
def test_centre_metric_pin_catches_planted_mistakes(monkeypatch, mistake):
    # a metric taken at a corner, or DF transposed, must fail the pin
    import oracle.dg as dg
    true_jac = dg.jacobian

    def planted(X, pts):
        if mistake == "corner":
            return true_jac(X, np.zeros_like(np.asarray(pts, dtype=np.float64)))
        return np.swapaxes(true_jac(X, pts), -1, -2)
    monkeypatch.setattr(dg, "jacobian", planted)
    d = _trilinear_disc()
    y = np.random.default_rng(6).standard_normal(d.unk_off[-1])
    assert _centre_pin_residual(d, y) > 1e-3
