"""GPU parity on 2:1 nonconforming meshes (hanging faces; Section 5.2 sums the
flux terms of a face over the neighbours sharing parts of it) against the
FP64 oracle, whose hanging-face matrices are pinned against the physical-space
brute assembler (tests/test_oracle_hanging.py), through the C ABI.

Bars: FP64 <= 1e-12, raw FP32 <= 1e-5 (relative 2-norm and largest entry);
slab solves <= 1e-10 against the oracle's direct solve with the energy
conserved.  Covered: coarse and fine sides, mixed p and q across the hanging
faces, reoriented elements, a sheared (non-diagonal metric) mesh that takes
P^{-1} as a pre-pass, all three modes, several kernel groups; D_h is refused
on such meshes."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note, oracle_disc, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _mesh(n=2, split=1, p=2, q=1, seed=0, reorient=False, shear=False, mixed=False):
    v, h = synth.hanging_mesh(n, split)
    if reorient:
        h = synth.reorient(h, seed=seed)
    if shear:
        v = synth.affine_transform(v, np.array([[1.0, 0.2, -0.1], [0.1, 0.9, 0.15], [-0.05, 0.1, 1.1]]))
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    if mixed:
        p = rng.integers(1, 4, ne)
        q = rng.integers(1, 3, ne)
    p = np.broadcast_to(np.asarray(p, np.int32), (ne,)).copy()
    q = np.broadcast_to(np.asarray(q, np.int32), (ne,)).copy()
    return synth.Mesh(v, h, p, q, rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))


def _check(lib, mesh, dt, seed, name):
    stdg = lib.stdg
    d = oracle_disc(mesh)
    assert len(d.hang) > 0
    mh = lib.upload(mesh)
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
            assert rel_err(got, d.operator(xs, dt)) < TOL[prec], (name, prec, "operator", rel_err(got, d.operator(xs, dt)))
            note("%s prec=%d residual" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls)
            assert rel_err(got, d.residual(Us, dt, Ls)) < TOL[prec], (name, prec, "residual")
            note("%s prec=%d precond" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs)
            assert rel_err(got, d.operator(d.precond_solve(xs), dt)) < TOL[prec], (name, prec, "precond")
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 1), (3, 2), (4, 3)])
def test_uniform_degrees(lib, p, q):
    _check(lib, _mesh(2, 1, p, q, seed=300 + p), 0.06, 300 + p, "hanging p%d q%d" % (p, q))


def test_mixed_degrees_and_orientations(lib):
    _check(lib, _mesh(2, 1, seed=310, reorient=True, mixed=True), 0.05, 310, "hanging mixed reoriented")


def test_sheared_prepass(lib):
    _check(lib, _mesh(2, 1, 2, 2, seed=311, shear=True), 0.05, 311, "hanging sheared")


def test_larger_mesh_two_interfaces(lib):
    # 3^3 coarse cells, the last two columns refined: 2:1 faces on one plane,
    # conforming fine-fine faces beyond it
    _check(lib, _mesh(3, 1, 2, 1, seed=312), 0.04, 312, "hanging 3^3")


def test_five_cells(lib):
    # a unit cube next to four half-size cubes on its face x = 1
    pts, idx = [], {}

    def vid(x, y, z):
        key = (round(x, 9), round(y, 9), round(z, 9))
        if key not in idx:
            idx[key] = len(pts)
            pts.append(key)
        return idx[key]

    def hexa(x0, y0, z0, hx, hy, hz):
        return [vid(x0 + hx * (v & 1), y0 + hy * ((v >> 1) & 1), z0 + hz * ((v >> 2) & 1)) for v in range(8)]

    hexes = [hexa(0, 0, 0, 1, 1, 1)] + [hexa(1, 0.5 * j, 0.5 * k, 0.5, 0.5, 0.5) for j in range(2) for k in range(2)]
    mesh = synth.Mesh(np.array(pts, dtype=np.float64), np.array(hexes, dtype=np.int64), np.array([3, 2, 2, 2, 2], np.int32),
                      np.array([2, 1, 2, 1, 2], np.int32), np.array([1.0, 2.0, 3.0, 1.5, 2.5]), np.ones(5))
    _check(lib, mesh, 0.08, 313, "hanging five cells")


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_slab_solve_and_energy(lib, inner, krylov):
    mesh = _mesh(2, 1, 2, 1, seed=314, mixed=False)
    mesh.q[:] = np.where(np.arange(mesh.n_elements) % 3 == 0, 2, 1)
    d = oracle_disc(mesh)
    rng = np.random.default_rng(314)
    s0 = rng.standard_normal(d.state_off[-1])
    dt = 0.1
    note("hanging solve: oracle")
    ref = d.level_state(d.solve_direct(s0, dt), 1)
    mh = lib.upload(mesh)
    try:
        st = lib.dev(s0, lib.torch.float64)
        note("hanging solve inner=%d krylov=%d" % (inner, krylov))
        info = lib.stdg.stdg_slab_solve(mh, 0.0, dt, None, st, inner_prec=inner, rtol=1e-13, max_iters=800,
                                        max_refine=80, krylov_prec=krylov)
        got = st.cpu().numpy()
        with pytest.raises(lib.stdg.StdgError) as ei:
            lib.stdg.stdg_mesh_set_dissipation(mh, 1.0)
        assert ei.value.status == -2
    finally:
        lib.stdg.stdg_mesh_free(mh)
    assert info["status"] == 0, info
    assert rel_err(got, ref) < 1e-10
    e0 = d.energy(s0)
    assert abs(d.energy(ref) - e0) < 1e-11 * e0
    assert abs(info["energy_end"] - e0) < 1e-10 * e0
