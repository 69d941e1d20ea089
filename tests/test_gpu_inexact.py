"""GPU parity of the inexact-solve pieces (Section 5.3): the dual norm of the
residual in W_h' and slab solves stopped by the iteration-error bound eta_it
(eq. a_posteriori:iteration), against the FP64 oracle.

Bars: dual norms <= 1e-12 relative; the actual iteration error of a marched
inexact solution stays below the accumulated eta_it (the guarantee), with
fewer GMRES iterations than the solve to rtol."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note, oracle_disc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return Lib()


def test_dual_norm_matches_oracle(lib):
    v, h = synth.box_mesh((3, 2, 2))
    A = np.array([[1.0, 0.2, 0.0], [0.1, 0.9, 0.15], [0.0, 0.1, 1.1]])
    v = synth.affine_transform(v, A)
    ne = h.shape[0]
    rng = np.random.default_rng(31)
    m = synth.Mesh(v, h, rng.integers(1, 5, ne).astype(np.int32), rng.integers(1, 4, ne).astype(np.int32),
                   rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    d = oracle_disc(m)
    mh = lib.upload(m)
    R = rng.standard_normal(d.unk_off[-1])
    for dt in (0.03, 0.2):
        got = lib.stdg.stdg_residual_dual_norm(mh, dt, lib.dev(R, lib.torch.float64))
        ref = d.dual_norms(R, dt)
        assert abs(got[0] - ref[0]) < 1e-12 * ref[0] and abs(got[1] - ref[1]) < 1e-12 * ref[1], (got, ref)
    lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_inexact_march_respects_eta_it(lib, inner, krylov):
    cfg = synth.cavity_two_material(n=2, p=3, q=2)
    m = cfg["mesh"]
    d = oracle_disc(m)
    from oracle import fields
    dt, n_slabs = 0.05, 3
    s = fields.project(d, fields.mode_superposition(cfg["init"].mnl, cfg["init"].abc), 0.0)
    e0 = d.energy(s)
    eta_tol = 1e-4 * np.sqrt(2 * e0)
    mh = lib.upload(m)
    st = lib.dev(s, lib.torch.float64)
    s_ex = s.copy()
    eta2 = 0.0
    iters_in = iters_ex = 0
    for n in range(n_slabs):
        r = lib.stdg.stdg_slab_solve(mh, n * dt, dt, None, st, inner_prec=inner, krylov_prec=krylov, rtol=1e-12,
                                     max_iters=2000, max_refine=200, eta_tol=eta_tol, eta_t_final=n_slabs * dt)
        assert r["status"] == 0, r
        assert r["eta2"] <= eta_tol ** 2
        eta2 += r["eta2"]
        iters_in += r["iters"]
        st_ex = lib.dev(s_ex, lib.torch.float64)
        rx = lib.stdg.stdg_slab_solve(mh, n * dt, dt, None, st_ex, inner_prec=inner, krylov_prec=krylov,
                                      rtol=1e-12, max_iters=2000, max_refine=200)
        iters_ex += rx["iters"]
        note("slab %d: oracle direct solve" % n)
        s_ex = d.level_state(d.solve_direct(s_ex, dt), 1)
    err = st.cpu().numpy() - s_ex
    err2 = 2.0 * d.energy(err)
    note("inexact: iters %d vs %d, error %.3e <= eta_it %.3e" % (iters_in, iters_ex, np.sqrt(err2), np.sqrt(eta2)))
    assert err2 <= eta2
    assert iters_in < iters_ex
    lib.stdg.stdg_mesh_free(mh)


def _trilinear_mesh(seed):
    shape = (3, 2, 2)
    v, h = synth.box_mesh(shape)
    v = synth.perturb_interior(v, shape, 0.25, seed)
    ne = h.shape[0]
    rng = np.random.default_rng(seed + 1)
    return synth.Mesh(v, h, rng.integers(1, 4, ne).astype(np.int32), rng.integers(1, 4, ne).astype(np.int32),
                      rng.uniform(1, 4, ne), rng.uniform(1, 2, ne), shape=shape)


def test_dual_norm_trilinear_matches_oracle(lib):
    """On trilinear elements the W_h' norm needs the element's own quadrature
    mass (not its centre metric): the library solves with it by conjugate
    gradients; against the oracle's dense solves with the same mass, 1e-12,
    and visibly different from the centre-metric value."""
    m = _trilinear_mesh(51)
    d = oracle_disc(m)
    mh = lib.upload(m)
    try:
        assert lib.stdg.stdg_mesh_info(mh)["n_nonaffine"] > 0
        R = np.random.default_rng(52).standard_normal(d.unk_off[-1])
        for dt in (0.03, 0.2):
            got = lib.stdg.stdg_residual_dual_norm(mh, dt, lib.dev(R, lib.torch.float64))
            ref = d.dual_norms(R, dt)
            assert abs(got[0] - ref[0]) < 1e-12 * ref[0] and abs(got[1] - ref[1]) < 1e-12 * ref[1], (got, ref)
        # the centre-metric value (what an affine formula would give) differs
        Rc = d.precond_centre_solve(R)
        cen = 0.0
        for e in range(d.ne):
            blk = R[d.unk_off[e]:d.unk_off[e + 1]]
            z = Rc[d.unk_off[e]:d.unk_off[e + 1]]
            cen += float(blk[:blk.size // 2] @ z[:z.size // 2]) * d.eps[e]
        cen /= 0.2
        assert abs(cen - ref[0]) > 1e-4 * ref[0]
    finally:
        lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_inexact_march_trilinear_respects_eta_it(lib, inner, krylov):
    """The inexact solve on a trilinear mesh with mixed degrees: the true
    iteration error of the march (against the oracle's direct solves) stays
    below the accumulated eta_it, now computed with the exact element masses."""
    m = _trilinear_mesh(61)
    d = oracle_disc(m)
    dt, n_slabs = 0.04, 3
    s = np.random.default_rng(62).standard_normal(d.state_off[-1])
    e0 = d.energy(s)
    eta_tol = 1e-4 * np.sqrt(2 * e0)
    mh = lib.upload(m)
    try:
        st = lib.dev(s, lib.torch.float64)
        s_ex = s.copy()
        eta2 = 0.0
        for n in range(n_slabs):
            r = lib.stdg.stdg_slab_solve(mh, n * dt, dt, None, st, inner_prec=inner, krylov_prec=krylov,
                                         rtol=1e-12, max_iters=2000, max_refine=200, eta_tol=eta_tol,
                                         eta_t_final=n_slabs * dt)
            assert r["status"] == 0, r
            assert r["eta2"] <= eta_tol ** 2
            eta2 += r["eta2"]
            note("trilinear slab %d: oracle direct solve" % n)
            s_ex = d.level_state(d.solve_direct(s_ex, dt), 1)
        err2 = 2.0 * d.energy(st.cpu().numpy() - s_ex)
        note("trilinear inexact: error %.3e <= eta_it %.3e" % (np.sqrt(err2), np.sqrt(eta2)))
        assert 0.0 < err2 <= eta2
    finally:
        lib.stdg.stdg_mesh_free(mh)
