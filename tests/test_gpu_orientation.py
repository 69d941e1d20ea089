"""GPU parity on conforming meshes whose neighbours meet in any orientation
(vertex numbers relabelled by seeded cube rotations): stdg_residual_apply in
every mode and precision, with and without D_h, and a slab solve, against
the oracle on the same inputs, through the C ABI; and the same physical
problem numbered two ways gives the same energies on the GPU.

Bars: FP64 <= 1e-12, raw FP32 <= 1e-5, solves <= 1e-10."""
import numpy as np
import pytest

import synth
from oracle import fields
from oracle.dg import Discretisation
from tests.gpu_util import Lib, note, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _check(lib, mesh, dt, seed, name, c=0.0):
    stdg = lib.stdg
    d = Discretisation(mesh.vertices, mesh.hexes, mesh.p, mesh.q, mesh.eps, mesh.mu, c_diss=c)
    assert len(d.fmap) > 0
    mh = lib.upload(mesh)
    if c > 0:
        stdg.stdg_mesh_set_dissipation(mh, c)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(d.unk_off[-1])
    U = rng.standard_normal(d.trial_off[-1])
    L = rng.standard_normal(d.unk_off[-1])
    try:
        for prec in (0, 1):
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
            # the block mass with the element-centre metric (exact on affine elements)
            assert rel_err(got, d.operator(d.precond_centre_solve(xs), dt)) < TOL[prec], (name, prec, "precond")
    finally:
        stdg.stdg_mesh_free(mh)


def _mesh(shape, p, q, seed, hi=(1.0, 1.0, 1.0), perturb=0.0, shear=False):
    v, h = synth.box_mesh(shape, hi=hi)
    if perturb > 0:
        v = synth.perturb_interior(v, shape, perturb, seed=seed, hi=hi)
    if shear:
        v = synth.affine_transform(v, np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]]))
    h = synth.reorient(h, seed=seed)
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    p = np.broadcast_to(np.asarray(p, np.int32), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q, np.int32), (ne,)).copy()
    return synth.Mesh(v, h, p, q, rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


@pytest.mark.parametrize("p,q", [(1, 1), (2, 2), (4, 3), (6, 2)])
def test_uniform_box(lib, p, q):
    _check(lib, _mesh((3, 2, 2), p, q, 40 + p, hi=(0.9, 0.5, 0.7)), 0.06, p, "reoriented p%d q%d" % (p, q))


def test_mixed_degrees(lib):
    rng = np.random.default_rng(41)
    m = _mesh((3, 2, 2), 1, 1, 41)
    m.p[:] = rng.integers(1, 5, m.n_elements)
    m.q[:] = rng.integers(1, 4, m.n_elements)
    _check(lib, m, 0.05, 41, "reoriented mixed")


def test_sheared(lib):
    m = _mesh((2, 2, 2), 2, 2, 42, shear=True)
    m.q[::2] = 1
    _check(lib, m, 0.07, 42, "reoriented sheared")


def test_trilinear(lib):
    m = _mesh((2, 2, 2), 3, 2, 43, perturb=0.15)
    _check(lib, m, 0.05, 43, "reoriented trilinear")


def test_dissipative(lib):
    m = _mesh((3, 2, 1), 3, 2, 44, hi=(0.9, 0.6, 0.4))
    m.q[1] = 3
    _check(lib, m, 0.05, 44, "reoriented D_h", c=0.8)


def test_p8(lib):
    _check(lib, _mesh((2, 2, 1), 8, 2, 45, hi=(0.6, 0.8, 0.5)), 0.05, 45, "reoriented p8")


def test_slab_solve_same_as_canonical_numbering(lib):
    # TE101 on the 4^3 cavity, numbered canonically and reoriented: the GPU
    # solves give the same energies, and the reoriented one matches the oracle
    cfg = synth.cavity_small()
    m0 = cfg["mesh"]
    m1 = synth.Mesh(m0.vertices, synth.reorient(m0.hexes, seed=46), m0.p, m0.q, m0.eps, m0.mu)
    res = []
    for m in (m0, m1):
        d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
        s0 = fields.project(d, fields.te101, 0.0)
        mh = lib.upload(m)
        try:
            st = lib.dev(s0, lib.torch.float64)
            note("reoriented solve: %d permuted faces" % len(d.fmap))
            info = lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=1, rtol=1e-13, max_iters=400,
                                            max_refine=40, krylov_prec=1)
            got = st.cpu().numpy()
        finally:
            lib.stdg.stdg_mesh_free(mh)
        assert info["status"] == 0
        res.append((d, s0, got, info))
    (d0, _, g0, i0), (d1, s1, g1, i1) = res
    assert abs(i0["energy_start"] - i1["energy_start"]) < 1e-13 * i0["energy_start"]
    assert abs(i0["energy_end"] - i1["energy_end"]) < 1e-11 * i0["energy_start"]
    note("reoriented solve: oracle")
    ref = d1.level_state(d1.solve_direct(s1, cfg["dt"]), 1)
    assert rel_err(g1, ref) < 1e-10


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_reoriented_dissipative_sampled(lib, prec):
    """The 32^3, p = 4, q = 3 two-material cavity, every element's numbering
    rotated and D_h on (c = 1), in the benchmark's launch configuration; the
    oracle checks sampled elements (an element's output depends only on it and
    its face neighbours)."""
    stdg = lib.stdg
    cfg = synth.cavity_two_material()
    m0 = cfg["mesh"]
    m = synth.Mesh(m0.vertices, synth.reorient(m0.hexes, seed=0), m0.p, m0.q, m0.eps, m0.mu, shape=m0.shape)
    dt = cfg["dt"]
    note("32^3 reoriented D_h prec=%d: inputs" % prec)
    x = synth.random_vector(m.unknown_size(), 0)
    if prec == 1:
        x = x.astype(np.float32).astype(np.float64)
    d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, c_diss=1.0)
    mh = lib.upload(m)
    try:
        stdg.stdg_mesh_set_dissipation(mh, 1.0)
        n = m.shape[0]
        rng = np.random.default_rng(43)
        sample = [int(e) for e in rng.choice(m.n_elements, 32, replace=False)]
        sample += [0, n - 1, n ** 3 - 1, n // 2 - 1 + n * (n // 2) + n * n * 3, n // 2 + n * 5 + n * n * 7]
        needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
        for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
            note("32^3 reoriented D_h prec=%d mode=%d: apply" % (prec, mode))
            y = lib.apply(mh, dt, prec, mode, x)
            assert np.all(np.isfinite(y))
            xin = d.precond_solve(x, needed) if mode == stdg.STDG_OPERATOR_PRECOND else x
            rows = d.apply_rows(d.embed_unknowns(xin), dt, sample)
            got = np.concatenate([y[d.unk_off[e]:d.unk_off[e + 1]] for e in sample])
            ref = np.concatenate([rows[e] for e in sample])
            note("32^3 reoriented D_h prec=%d mode=%d rel err %.3e" % (prec, mode, rel_err(got, ref)))
            assert rel_err(got, ref) < TOL[prec]
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("p,q", [(2, 2), (3, 1)])
def test_trilinear_dissipation_reoriented(lib, p, q):
    # D_h on trilinear elements met in every orientation: the neighbour's face
    # points and tangential components through the face map
    m = _mesh((3, 2, 2), p, q, 48 + p, hi=(0.9, 0.5, 0.7), perturb=0.15)
    _check(lib, m, 0.05, 48 + p, "reoriented trilinear D_h p%d q%d" % (p, q), c=0.9)
