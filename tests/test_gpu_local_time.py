"""GPU parity with local time steps (Section 2.2: slab intervals bisected into
n = 1, 2, 4, 8 sub-intervals per element; S_h of Section 4.1 couples
neighbours through the projection onto their common temporal test space)
against the FP64 oracle, whose local-time pieces are pinned against the
brute-force assembler and Thm 4.1 (tests/test_oracle_local_time.py), through
the C ABI.

Bars: FP64 <= 1e-12, raw FP32 <= 1e-5 (relative 2-norm and largest entry);
slab solves <= 1e-10 against the oracle's direct solve with the energy
conserved.  Covered: mixed n with mixed p and q, reoriented elements, a
sheared (non-diagonal metric) mesh, a larger mesh where most rows stay in the
kernel groups, p = 6 and 8 (the widest workgroups, FP64 traces gathered per
level), all three modes (the preconditioned one through the P^{-1}
pre-pass that mixes the time levels), the allocation-free entry point, slab
solves in FP64 and FP32 inner precision; refusals of what the path does not
take."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note, oracle_disc, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _mesh(shape=(2, 2, 2), p=2, q=1, nsub=(1, 2), seed=0, reorient=False, shear=False, mixed=False):
    v, h = synth.box_mesh(shape)
    if reorient:
        h = synth.reorient(h, seed=seed)
    if shear:
        v = synth.affine_transform(v, np.array([[1.0, 0.2, -0.1], [0.1, 0.9, 0.15], [-0.05, 0.1, 1.1]]))
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    if mixed:
        p = rng.integers(1, 4, ne)
        q = rng.integers(1, 4, ne)
    p = np.broadcast_to(np.asarray(p, np.int32), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q, np.int32), (ne,)).copy()
    ns = np.asarray(nsub, np.int32)[rng.integers(0, len(nsub), ne)]
    ns = np.where(ns * q > 24, 1, ns).astype(np.int32)
    return synth.Mesh(v, h, p, q, rng.uniform(1, 4, ne), rng.uniform(1, 2, ne), nsub=ns)


def _check(lib, mesh, dt, seed, name):
    stdg = lib.stdg
    d = oracle_disc(mesh)
    assert int(d.nk.max()) > 1
    mh = lib.upload(mesh)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(d.unk_off[-1])
    U = rng.standard_normal(d.trial_off[-1])
    L = rng.standard_normal(d.unk_off[-1])
    try:
        info = stdg.stdg_mesh_info(mh)
        assert info["unknown_size"] == d.unk_off[-1] and info["trial_size"] == d.trial_off[-1]
        for prec in (0, 1):
            cast = (lambda v: v) if prec == 0 else (lambda v: v.astype(np.float32).astype(np.float64))
            xs, Us, Ls = cast(x), cast(U), cast(L)
            note("%s prec=%d operator" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xs)
            assert rel_err(got, d.operator(xs, dt)) < TOL[prec], (name, prec, "operator", rel_err(got, d.operator(xs, dt)))
            note("%s prec=%d residual" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls)
            assert rel_err(got, d.residual(Us, dt, Ls)) < TOL[prec], (name, prec, "residual")
            note("%s prec=%d precond" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs)
            assert rel_err(got, d.operator(d.precond_solve(xs), dt)) < TOL[prec], (name, prec, "precond")
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("q,nsub", [(1, (1, 2)), (2, (1, 2, 4)), (3, (2, 4)), (1, (1, 8))])
def test_uniform_degrees(lib, q, nsub):
    _check(lib, _mesh(p=2, q=q, nsub=nsub, seed=400 + q), 0.06, 400 + q, "local time q%d n%s" % (q, nsub))


def test_mixed_degrees_and_orientations(lib):
    _check(lib, _mesh(nsub=(1, 2, 4), seed=410, reorient=True, mixed=True), 0.05, 410, "local time mixed reoriented")


def test_sheared_prepass(lib):
    _check(lib, _mesh(p=2, q=2, nsub=(1, 2), seed=411, shear=True), 0.05, 411, "local time sheared")


def test_larger_mesh_few_local_rows(lib):
    # 4^3 elements, two with sub-intervals: most rows run in the kernel groups
    m = _mesh((4, 4, 4), p=2, q=2, nsub=(1,), seed=412)
    m.nsub[[5, 42]] = (2, 4)
    _check(lib, m, 0.04, 412, "local time 4^3")


def test_high_degrees(lib):
    # p = 6 and 8 side by side: 384 and 768 threads per workgroup, the own
    # levels read at each use for p = 8, and its FP64 neighbour traces
    # gathered per level (the staged ones exceed 64 KB of LDS)
    v, h = synth.box_mesh((2, 1, 1))
    rng = np.random.default_rng(417)
    m = synth.Mesh(v, h, np.array([6, 8], np.int32), np.array([2, 1], np.int32), rng.uniform(1, 4, 2),
                   rng.uniform(1, 2, 2), nsub=np.array([2, 1], np.int32))
    _check(lib, m, 0.05, 417, "local time p6|p8")


def test_noalloc_entry_point(lib):
    mesh = _mesh(p=2, q=2, nsub=(1, 2), seed=413, shear=True)
    d = oracle_disc(mesh)
    t = lib.torch
    mh = lib.upload(mesh)
    try:
        x = np.random.default_rng(413).standard_normal(d.unk_off[-1])
        xd = lib.dev(x, t.float64)
        yd = t.empty_like(xd)
        note("local time noalloc precond")
        lib.stdg.stdg_residual_apply_noalloc(mh, 0.05, lib.stdg.STDG_FP64, lib.stdg.STDG_OPERATOR_PRECOND, xd, None, yd)
        t.cuda.synchronize()
        assert rel_err(yd.cpu().numpy(), d.operator(d.precond_solve(x), 0.05)) < 1e-12
    finally:
        lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_slab_solve_and_energy(lib, inner, krylov):
    mesh = _mesh(p=2, q=2, nsub=(1, 2, 4), seed=414, mixed=True)
    d = oracle_disc(mesh)
    rng = np.random.default_rng(414)
    s0 = rng.standard_normal(d.state_off[-1])
    dt = 0.1
    note("local time solve: oracle")
    ref = d.level_state(d.solve_direct(s0, dt), 1)
    mh = lib.upload(mesh)
    try:
        st = lib.dev(s0, lib.torch.float64)
        note("local time solve inner=%d krylov=%d" % (inner, krylov))
        info = lib.stdg.stdg_slab_solve(mh, 0.0, dt, None, st, inner_prec=inner, rtol=1e-13, max_iters=800,
                                        max_refine=80, krylov_prec=krylov)
        got = st.cpu().numpy()
    finally:
        lib.stdg.stdg_mesh_free(mh)
    assert info["status"] == 0, info
    assert rel_err(got, ref) < 1e-10
    e0 = d.energy(s0)
    assert abs(d.energy(ref) - e0) < 1e-11 * e0
    assert abs(info["energy_end"] - e0) < 1e-10 * e0


def test_refusals(lib):
    stdg = lib.stdg
    mesh = _mesh(p=1, q=1, nsub=(1, 2), seed=415)
    mh = lib.upload(mesh)
    try:
        with pytest.raises(stdg.StdgError) as ei:
            stdg.stdg_mesh_set_dissipation(mh, 1.0)
        assert ei.value.status == -2  # STDG_E_UNSUPPORTED
    finally:
        stdg.stdg_mesh_free(mh)
    # trilinear elements with sub-intervals
    v, h = synth.box_mesh((2, 2, 2))
    v = synth.perturb_interior(v, (2, 2, 2), 0.15, seed=3)
    tri = synth.Mesh(v, h, np.full(8, 1, np.int32), np.full(8, 1, np.int32), np.ones(8), np.ones(8),
                     nsub=np.array([2, 1, 1, 1, 1, 1, 1, 1], np.int32))
    with pytest.raises(stdg.StdgError) as ei:
        lib.upload(tri)
    assert ei.value.status == -2  # STDG_E_UNSUPPORTED
    bad = _mesh(p=1, q=1, nsub=(1,), seed=416)
    bad.nsub[3] = 3
    with pytest.raises(stdg.StdgError) as ei:
        lib.upload(bad)
    assert ei.value.status == -1  # STDG_E_ARG
