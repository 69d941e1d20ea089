"""Pin of the oracle's iterative slab solve: right-preconditioned restarted
GMRES (Section 5.4, eq. preconditioner) on the oracle's own block apply must
reach the sparse direct solution of the same slab problem (Section 3
eq. weakform, Section 4 eq. weakform_stabilized), on meshes where every part
of the operator is active: mixed p and q (S_h, p-truncated faces), a sheared
affine mesh (non-diagonal metric), a trilinear one (quadrature mass), and a
source."""
import numpy as np
import pytest

import synth
from oracle import fields
from oracle.dg import Discretisation


def _mesh(kind, seed):
    v, h = synth.box_mesh((2, 2, 2))
    if kind == "sheared":
        v = synth.affine_transform(v, np.array([[1.0, 0.25, -0.1], [0.05, 0.95, 0.2], [0.15, -0.1, 1.05]]))
    elif kind == "trilinear":
        v = synth.perturb_interior(v, (2, 2, 2), 0.2, seed)
    rng = np.random.default_rng(seed)
    return Discretisation(v, h, rng.integers(1, 4, 8), rng.integers(1, 4, 8), rng.uniform(1, 4, 8),
                          rng.uniform(1, 2, 8))


@pytest.mark.parametrize("kind", ["sheared", "trilinear"])
def test_gmres_matches_direct_solve(kind):
    d = _mesh(kind, 11)
    assert len(set(int(v) for v in d.q)) > 1 and len(set(int(v) for v in d.a)) > 1
    rng = np.random.default_rng(12)
    s0 = rng.standard_normal(d.state_off[-1])
    J = fields.gaussian_pulse(2.0, (0.4, 0.6, 0.5), 0.3, 2.0, 0.05, 0.1, (0.2, 1.0, -0.4))
    dt = 0.06
    L = d.load(J, 0.02, dt)
    U_dir = d.solve_direct(s0, dt, L)
    U_it = d.solve_gmres(s0, dt, L, rtol=1e-14)
    assert np.linalg.norm(U_it - U_dir) < 1e-12 * np.linalg.norm(U_dir)
    # and the iterate is a solution: the residual vanishes
    r = d.residual(U_it, dt, L)
    r0 = d.residual(d.embed_unknowns(np.zeros(d.unk_off[-1]), s0), dt, L)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(r0)
