"""GPU parity of the dissipative stabilisation D_h (the remark closing Section 4)
through the C ABI (stdg_mesh_set_dissipation, then stdg_residual_apply and
stdg_slab_solve) against the oracle's B_h + D_h on the same seeded inputs.

Bars as for the plain apply: FP64 <= 1e-12, raw FP32 <= 1e-5; the slab solve
<= 1e-10 against the oracle's direct solve, with the energy dropping by the
oracle's amount.  The three neighbour paths of the kernel are covered (FP32
staged faces, gathered faces, mixed degrees), as are the PEC faces, jumps in
eps and mu, sheared affine elements (full face metric) and switching back
to c = 0; on trilinear elements (face metric at the points of the face rule),
next to affine ones, with mixed degrees, and in the slab solve."""
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


def _check(lib, mesh, dt, c, seed, name, precs=(0, 1), centre=False):
    """centre: P^{-1} with the element-centre metric (trilinear elements;
    exact on affine ones)"""
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
            pre = d.precond_centre_solve(xs) if centre else d.precond_solve(xs)
            assert rel_err(got, d.operator(pre, dt)) < TOL[prec], (name, prec, "precond")
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
    # trilinear elements (D_h by its own kernel): on, then off again bitwise
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=4)
    mesh = synth.Mesh(v, h, np.full(8, 2, np.int32), np.full(8, 1, np.int32), np.ones(8), np.ones(8))
    mh = lib.upload(mesh)
    x = np.random.default_rng(4).standard_normal(stdg.stdg_mesh_info(mh)["unknown_size"])
    try:
        plain = lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x)
        stdg.stdg_mesh_set_dissipation(mh, 1.0)
        assert rel_err(lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x), plain) > 1e-3
        stdg.stdg_mesh_set_dissipation(mh, 0.0)
        assert np.array_equal(lib.apply(mh, 0.1, 0, stdg.STDG_OPERATOR, x), plain)
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


# ---- trilinear elements: the face metric varies over each face -------------

def _trilinear(shape, p, q, seed, perturb=0.15):
    v, h = synth.box_mesh(shape, hi=(0.9, 0.6, 0.7))
    v = synth.perturb_interior(v, shape, perturb, seed=seed, hi=(0.9, 0.6, 0.7))
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    p = np.broadcast_to(np.asarray(p, np.int32), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q, np.int32), (ne,)).copy()
    return synth.Mesh(v, h, p, q, rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


@pytest.mark.parametrize("p,q", [(1, 1), (2, 2), (3, 2), (6, 4)])
def test_trilinear_uniform_degrees(lib, p, q):
    mesh = _trilinear((3, 2, 2), p, q, 200 + p)
    _check(lib, mesh, 0.06, 0.9, 200 + p, "diss trilinear p%d q%d" % (p, q), centre=True)


def test_trilinear_mixed_degrees(lib):
    # face rules of max(a, a') + 2 points between different degrees, the
    # neighbour's time levels truncated at min(q, q')
    rng = np.random.default_rng(210)
    mesh = _trilinear((3, 2, 2), 1, 1, 210)
    mesh.p[:] = rng.integers(1, 5, mesh.n_elements)
    mesh.q[:] = rng.integers(1, 4, mesh.n_elements)
    _check(lib, mesh, 0.05, 1.2, 210, "diss trilinear mixed", centre=True)


def test_trilinear_next_to_affine(lib):
    # one interior vertex moved: the eight elements around it are trilinear,
    # the other four stay boxes (the affine D_h kernels meet trilinear neighbours)
    v, h = synth.box_mesh((3, 2, 2))
    idx = int(np.argmin(np.linalg.norm(v - np.array([1 / 3, 0.5, 0.5]), axis=1)))
    v = v.copy()
    v[idx] += np.array([0.05, -0.04, 0.03])
    rng = np.random.default_rng(211)
    mesh = synth.Mesh(v, h, rng.integers(1, 4, 12).astype(np.int32), rng.integers(1, 3, 12).astype(np.int32),
                      rng.uniform(1, 4, 12), rng.uniform(1, 2, 12))
    mh = lib.upload(mesh)
    info = lib.stdg.stdg_mesh_info(mh)
    lib.stdg.stdg_mesh_free(mh)
    assert info["n_affine"] == 4 and info["n_nonaffine"] == 8, info
    _check(lib, mesh, 0.05, 0.7, 211, "diss trilinear next to affine", centre=True)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_trilinear_slab_solve_energy_drops(lib, inner, krylov):
    mesh = _trilinear((2, 2, 2), 2, 1, 212)
    mesh.q[:] = np.array([1, 2] * 4, np.int32)
    c, dt = 0.7, 0.12
    d = _disc(mesh, c)
    rng = np.random.default_rng(212)
    s0 = rng.standard_normal(d.state_off[-1])
    note("diss trilinear solve: oracle")
    ref = d.level_state(d.solve_direct(s0, dt), 1)
    mh = lib.upload(mesh)
    try:
        lib.stdg.stdg_mesh_set_dissipation(mh, c)
        st = lib.dev(s0, lib.torch.float64)
        note("diss trilinear solve inner=%d krylov=%d" % (inner, krylov))
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
