"""GPU parity on trilinear (non-affine) hexahedra: the residual apply with the
mass integrated by the (p + 2)-point Gauss rule (Section 5.2, non-affine mass),
the load, the energy and the slab solve, against the FP64 oracle on the same
seeded inputs, through the C ABI.

Bars: FP64 <= 1e-12 relative, raw FP32 <= 1e-5, solve <= 1e-10.  Both sides
use the same quadrature rule for the mass, so the comparison is exact up to
rounding; the rule's own error against the exact integral is not a parity
claim."""
import numpy as np
import pytest

import synth
from oracle import fields
from tests.gpu_util import Lib, note, oracle_disc, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _cast(prec):
    return (lambda v: v) if prec == 0 else (lambda v: v.astype(np.float32).astype(np.float64))


def _check(lib, mesh, dt, seed, name, precs=(0, 1), variants=(0,)):
    stdg = lib.stdg
    d = oracle_disc(mesh)
    mh = lib.upload(mesh)
    info = stdg.stdg_mesh_info(mh)
    note("%s: %d affine, %d trilinear elements" % (name, info["n_affine"], info["n_nonaffine"]))
    assert info["n_nonaffine"] > 0
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(d.unk_off[-1])
    U = rng.standard_normal(d.trial_off[-1])
    L = rng.standard_normal(d.unk_off[-1])
    try:
      for variant in variants:
        stdg.stdg_mesh_set_launch(mh, -1, variant)
        for prec in precs:
            c = _cast(prec)
            xs, Us, Ls = c(x), c(U), c(L)
            note("%s variant=%d prec=%d operator" % (name, variant, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xs)
            err = rel_err(got, d.operator(xs, dt))
            assert err < TOL[prec], (name, variant, prec, "operator", err)
            note("%s variant=%d prec=%d residual" % (name, variant, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls)
            err = rel_err(got, d.residual(Us, dt, Ls))
            assert err < TOL[prec], (name, variant, prec, "residual", err)
            note("%s variant=%d prec=%d precond" % (name, variant, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs)
            err = rel_err(got, d.operator(d.precond_centre_solve(xs), dt))
            assert err < TOL[prec], (name, variant, prec, "precond", err)
    finally:
        stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 2), (3, 1), (4, 2), (5, 3), (6, 4), (7, 3), (8, 2)])
def test_trilinear_uniform_degrees(lib, p, q):
    shape = (3, 2, 2) if p <= 6 else (2, 2, 2)  # every element touches an interior vertex
    v, h = synth.box_mesh(shape, hi=(0.9, 0.6, 0.7))
    v = synth.perturb_interior(v, shape, 0.2, 30 + p, hi=(0.9, 0.6, 0.7))
    ne = h.shape[0]
    rng = np.random.default_rng(p * 7 + q)
    mesh = synth.Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                      rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    _check(lib, mesh, 0.043, 200 + p, "trilinear p%d q%d" % (p, q), variants=(0, 1))


def test_trilinear_and_affine_groups_in_one_mesh(lib):
    # only the lattice vertex (1, 1, 1) moves: the 8 elements around it are
    # trilinear, the other 28 stay affine, with random degrees everywhere
    shape = (4, 3, 3)
    v, h = synth.box_mesh(shape)
    vid = 1 + (shape[0] + 1) * (1 + (shape[1] + 1) * 1)
    v = v.copy()
    v[vid] += np.array([0.04, -0.03, 0.05])
    ne = h.shape[0]
    rng = np.random.default_rng(8)
    mesh = synth.Mesh(v, h, rng.integers(1, 6, ne).astype(np.int32), rng.integers(1, 5, ne).astype(np.int32),
                      rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    _check(lib, mesh, 0.05, 9, "trilinear+affine", variants=(0, 1, 2))


def test_graded_hp_mesh_4cubed(lib):
    # the graded workload's recipe at 4^3: rings 1 and 3, p = 5, 3 and q = 3, 1
    cfg = synth.graded_nonaffine(n=4)
    _check(lib, cfg["mesh"], 0.02, 10, "graded 4^3", variants=(0, 1))


def test_trilinear_load_and_energy_graded_4cubed(lib):
    cfg = synth.graded_nonaffine(n=4)
    m = cfg["mesh"]
    d = oracle_disc(m)
    mh = lib.upload(m)
    src = cfg["source"]
    J = fields.gaussian_pulse(src.amp, src.center, src.sigma_x, src.f0, src.t0, src.sigma_t, src.dir)
    t0, dt = 0.08, 0.02
    note("graded 4^3: load")
    Ld = lib.torch.zeros(d.unk_off[-1], dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_load_assemble(mh, src, t0, dt, Ld)
    assert rel_err(Ld.cpu().numpy(), d.load(J, t0, dt)) < 1e-12
    note("graded 4^3: energy")
    s0 = np.random.default_rng(12).standard_normal(d.state_off[-1])
    e = lib.stdg.stdg_energy(mh, lib.dev(s0, lib.torch.float64))
    assert abs(e - d.energy(s0)) < 1e-12 * d.energy(s0)
    lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner", [0, 1])
def test_trilinear_slab_solve_mixed_degrees_with_source(lib, inner):
    shape = (3, 2, 2)
    v, h = synth.box_mesh(shape)
    v = synth.perturb_interior(v, shape, 0.2, 14)
    ne = h.shape[0]
    rng = np.random.default_rng(15)
    m = synth.Mesh(v, h, rng.integers(1, 4, ne).astype(np.int32), rng.integers(1, 4, ne).astype(np.int32),
                   rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    d = oracle_disc(m)
    src = synth.Source(kind=1, amp=2.0, center=(0.4, 0.6, 0.5), sigma_x=0.2, f0=2.0, t0=0.05,
                       sigma_t=0.1, dir=(0.2, 1.0, -0.4))
    J = fields.gaussian_pulse(src.amp, src.center, src.sigma_x, src.f0, src.t0, src.sigma_t, src.dir)
    t0, dt = 0.02, 0.04
    L_ref = d.load(J, t0, dt)
    mh = lib.upload(m)
    Ld = lib.torch.zeros(d.unk_off[-1], dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_load_assemble(mh, src, t0, dt, Ld)
    assert rel_err(Ld.cpu().numpy(), L_ref) < 1e-12
    s0 = rng.standard_normal(d.state_off[-1])
    U_ref = d.solve_direct(s0, dt, L_ref)
    st = lib.dev(s0, lib.torch.float64)
    Ud = lib.torch.zeros(d.trial_off[-1], dtype=lib.torch.float64, device="cuda")
    note("trilinear solve inner=%d" % inner)
    info = lib.stdg.stdg_slab_solve(mh, t0, dt, Ld, st, inner_prec=inner, rtol=1e-13, max_iters=2000,
                                    max_refine=200, slab_U=Ud)
    assert info["status"] == 0, info
    assert rel_err(Ud.cpu().numpy(), U_ref) < 1e-10
    assert rel_err(st.cpu().numpy(), d.level_state(U_ref, 1)) < 1e-10
    lib.stdg.stdg_mesh_free(mh)


def test_trilinear_energy_conserved_without_source(lib):
    cfg = synth.graded_nonaffine(n=4)
    m = cfg["mesh"]
    mh = lib.upload(m)
    info_m = lib.stdg.stdg_mesh_info(mh)
    s0 = np.random.default_rng(13).standard_normal(info_m["state_size"])
    st = lib.dev(s0, lib.torch.float64)
    for n in range(2):
        info = lib.stdg.stdg_slab_solve(mh, n * 0.02, 0.02, None, st, inner_prec=1, rtol=1e-13, max_iters=2000,
                                        max_refine=200)
        assert info["status"] == 0, info
        assert abs(info["energy_end"] - info["energy_start"]) < 1e-10 * info["energy_start"]
    lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("prec,c_diss", [(0, 0.0), (1, 0.0), (0, 1.0), (1, 1.0)])
def test_graded_24cubed_sampled(lib, prec, c_diss):
    """Full-size graded 24^3 trilinear mesh (p 3..6, q 1..4) in the launch
    configuration of a preconditioned operator apply, also with D_h (c = 1);
    the oracle checks sampled elements from every ring."""
    from oracle.dg import Discretisation
    stdg = lib.stdg
    cfg = synth.graded_nonaffine()
    m = cfg["mesh"]
    dt = cfg["dt"]
    x = _cast(prec)(synth.random_vector(m.unknown_size(), 0))
    mh = lib.upload(m)
    if c_diss > 0:
        stdg.stdg_mesh_set_dissipation(mh, c_diss)
    d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, c_diss=c_diss)
    rng = np.random.default_rng(44)
    sample = []
    for p in (6, 5, 4, 3):
        ids = np.nonzero(m.p == p)[0]
        sample += [int(e) for e in rng.choice(ids, 4, replace=False)]
    sample += [0, m.n_elements - 1]
    needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
    for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
        note("graded 24^3 prec=%d c=%g mode=%d: apply" % (prec, c_diss, mode))
        y = lib.apply(mh, dt, prec, mode, x)
        assert np.all(np.isfinite(y))
        xin = d.precond_centre_solve(x, needed) if mode == stdg.STDG_OPERATOR_PRECOND else x
        rows = d.apply_rows(d.embed_unknowns(xin), dt, sample)
        got = np.concatenate([y[d.unk_off[e]:d.unk_off[e + 1]] for e in sample])
        ref = np.concatenate([rows[e] for e in sample])
        err = rel_err(got, ref)
        note("graded 24^3 prec=%d c=%g mode=%d rel err %.3e" % (prec, c_diss, mode, err))
        assert err < TOL[prec]
    stdg.stdg_mesh_free(mh)
