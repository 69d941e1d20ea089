"""GPU parity of the dissipative stabilisation D_h (the remark closing Section 4)
through the C ABI (stdg_mesh_set_dissipation, then stdg_residual_apply and
stdg_slab_solve) against the oracle's B_h + D_h on the same seeded inputs.

Bars as for the plain apply: FP64 <= 1e-12, raw FP32 <= 1e-5; the slab solve
<= 1e-10 against the oracle's direct solve, with the energy dropping by the
oracle's amount.  The three neighbour paths of the kernel are covered (FP32
staged faces, gathered faces, mixed degrees), as are the PEC faces, jumps in
eps and mu, sheared affine elements (full face metric) and switching back
to c = 0."""
import numpy as np
import pytest

import synth
from oracle.dg import Discretisation
from tests.gpu_util import Lib, note, random_mixed_mesh, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _disc(mesh, c):
    return Discretisation(mesh.vertices, mesh.hexes, mesh.p, mesh.q, mesh.eps, mesh.mu, c_diss=c)


def _check(lib, mesh, dt, c, seed, name, precs=(0, 1)):
    stdg = lib.stdg
    d = _disc(mesh, c)
    mh = lib.upload(mesh)
    stdg.stdg_mesh_set_dissipation(mh, c)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(d.unk_off[-1])
    U = rng.standard_normal(d.trial_off[-1])
    L = rng.standard_normal(d.unk_off[-1])
    try:
        for prec in precs:
            cast = (lambda v: v) if prec == 0 else (lambda v: v.astype(np.float32).astype(np.float64))
            xs, Us, Ls = cast(x), cast(U), cast(L)
            note("%s prec=%d operator" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xs)
            assert rel_err(got, d.operator(xs, dt)) < TOL[prec], (name, prec, "operator")
            note("%s prec=%d residual" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls)
            assert rel_err(got, d.residual(Us, dt, Ls)) < TOL[prec], (name, prec, "residual")
            note("%s prec=%d precond" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs)
            assert rel_err(got, d.operator(d.precond_solve(xs), dt)) < TOL[prec], (name, prec, "precond")
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("p,q", [(1, 1), (3, 2), (4, 3), (6, 4)])
def test_uniform_degrees(lib, p, q):
    # 12 elements, box cells of unequal sides; FP32 a <= 5 stages neighbour
    # faces through LDS, a = 7 gathers them
    v, h = synth.box_mesh((3, 2, 2), hi=(0.9, 0.5, 0.7))
    ne = h.shape[0]
    rng = np.random.default_rng(100 + 10 * p + q)
    mesh = synth.Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                      rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    _check(lib, mesh, 0.07, 0.8, p, "diss uniform p%d q%d" % (p, q))


def test_p8_four_elements(lib):
    # a = 9: the largest kernels (the FP32 dissipative one keeps a few values in scratch)
    v, h = synth.box_mesh((2, 2, 1), hi=(0.6, 0.8, 0.5))
    rng = np.random.default_rng(108)
    mesh = synth.Mesh(v, h, np.full(4, 8, np.int32), np.full(4, 2, np.int32), rng.uniform(1, 4, 4), rng.uniform(1, 2, 4))
    _check(lib, mesh, 0.05, 1.1, 108, "diss uniform p8 q2")


def test_mixed_degrees_and_materials(lib):
    mesh = random_mixed_mesh((3, 2, 2), 4, 3, seed=31)
    _check(lib, mesh, 0.05, 1.3, 31, "diss mixed")


def test_sheared_affine_mixed(lib):
    v, h = synth.box_mesh((2, 2, 2))
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    v = synth.affine_transform(v, A)
    rng = np.random.default_rng(32)
    mesh = synth.Mesh(v, h, np.array([2, 1, 2, 3, 1, 2, 3, 2], np.int32), np.array([1, 2, 2, 1, 3, 2, 2, 1], np.int32),
                      rng.uniform(1, 3, 8), rng.uniform(1, 3, 8))
    _check(lib, mesh, 0.07, 0.6, 32, "diss sheared")


def test_off_again_and_errors(lib):
    stdg = lib.stdg
    mesh = random_mixed_mesh((2, 2, 1), 3, 2, seed=33)
    mh = lib.upload(mesh)
    x = np.random.default_rng(33).standard_normal(stdg.stdg_mesh_info(mh)["unknown_size"])
    try:
        plain = lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x)
        stdg.stdg_mesh_set_dissipation(mh, 2.0)
        diss = lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x)
        assert rel_err(diss, plain) > 1e-3
        stdg.stdg_mesh_set_dissipation(mh, 0.0)
        assert np.array_equal(lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x), plain)
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(stdg.StdgError) as ei:
                stdg.stdg_mesh_set_dissipation(mh, bad)
            assert ei.value.status == -1
    finally:
        stdg.stdg_mesh_free(mh)
    # trilinear elements: the face metric is not constant
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=4)
    mesh = synth.Mesh(v, h, np.full(8, 2, np.int32), np.full(8, 1, np.int32), np.ones(8), np.ones(8))
    mh = lib.upload(mesh)
    try:
        with pytest.raises(stdg.StdgError) as ei:
            stdg.stdg_mesh_set_dissipation(mh, 1.0)
        assert ei.value.status == -2
        stdg.stdg_mesh_set_dissipation(mh, 0.0)
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_slab_solve_energy_drops(lib, inner, krylov):
    # two-material box with mixed q: the solve matches the oracle's direct solve
    # and the energy drops by the oracle's dissipation
    v, h = synth.box_mesh((2, 2, 2))
    rng = np.random.default_rng(34)
    mesh = synth.Mesh(v, h, np.full(8, 2, np.int32), np.array([1, 2] * 4, np.int32),
                      rng.uniform(1, 3, 8), rng.uniform(1, 2, 8))
    c, dt = 0.7, 0.15
    d = _disc(mesh, c)
    s0 = rng.standard_normal(d.state_off[-1])
    note("diss solve: oracle")
    U = d.solve_direct(s0, dt)
    ref = d.level_state(U, 1)
    mh = lib.upload(mesh)
    try:
        lib.stdg.stdg_mesh_set_dissipation(mh, c)
        st = lib.dev(s0, lib.torch.float64)
        note("diss solve inner=%d krylov=%d" % (inner, krylov))
        info = lib.stdg.stdg_slab_solve(mh, 0.0, dt, None, st, inner_prec=inner, rtol=1e-13, max_iters=600,
                                        max_refine=60, krylov_prec=krylov)
        got = st.cpu().numpy()
    finally:
        lib.stdg.stdg_mesh_free(mh)
    assert info["status"] == 0, info
    assert rel_err(got, ref) < 1e-10
    e0, e1 = d.energy(s0), d.energy(ref)
    assert e1 < (1 - 1e-3) * e0
    assert abs(info["energy_end"] - e1) < 1e-10 * e0
