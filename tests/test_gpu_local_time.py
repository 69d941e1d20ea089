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
solves in FP64 and FP32 inner precision, the load per sub-interval with a
source-driven solve, dual norms and an inexact march within eta_it, a
serving request bitwise the plain march, the full-size 32^3 4/2/1 workload
on sampled elements, a march of the manufactured exp solution with the
nodal order 2 q, D_h in every mode and precision with a slab solve;
refusals of what the path does not take."""
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


@pytest.mark.parametrize("q,nsub", [(1, (1, 2)), (2, (1, 2, 4)), (3, (2, 4)), (1, (1, 8)), (5, (1, 2)), (6, (1, 4))])
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


def test_every_element_subdivided(lib):
    # no kernel groups left: every row runs in the local-time kernel; the
    # slab solve equals the oracle's (uniform n = 2 is two half slabs there)
    m = _mesh((2, 2, 1), p=2, q=2, nsub=(2,), seed=421)
    _check(lib, m, 0.05, 421, "local time all n=2")
    d = oracle_disc(m)
    s0 = np.random.default_rng(421).standard_normal(d.state_off[-1])
    ref = d.level_state(d.solve_direct(s0, 0.08), 1)
    mh = lib.upload(m)
    try:
        assert lib.stdg.stdg_mesh_info(mh)["n_groups"] == 0
        st = lib.dev(s0, lib.torch.float64)
        note("local time all n=2: solve")
        r = lib.stdg.stdg_slab_solve(mh, 0.0, 0.08, None, st, inner_prec=1, rtol=1e-13, max_iters=800,
                                     max_refine=80, krylov_prec=1)
        assert r["status"] == 0, r
        assert rel_err(st.cpu().numpy(), ref) < 1e-10
    finally:
        lib.stdg.stdg_mesh_free(mh)


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


def test_load_and_slab_solve_with_source(lib):
    # the load per sub-interval, and a source-driven slab solve
    from oracle import fields
    mesh = _mesh((3, 2, 1), p=2, q=2, nsub=(1, 2, 4), seed=418, mixed=True)
    d = oracle_disc(mesh)
    src = synth.Source(kind=1, amp=2.0, center=(0.4, 0.6, 0.5), sigma_x=0.2, f0=2.0, t0=0.05,
                       sigma_t=0.1, dir=(0.2, 1.0, -0.4))
    J = fields.gaussian_pulse(src.amp, src.center, src.sigma_x, src.f0, src.t0, src.sigma_t, src.dir)
    t0, dt = 0.02, 0.04
    note("local time load: oracle")
    L_ref = d.load(J, t0, dt)
    mh = lib.upload(mesh)
    try:
        t = lib.torch
        Ld = t.zeros(d.unk_off[-1], dtype=t.float64, device="cuda")
        note("local time load")
        lib.stdg.stdg_load_assemble(mh, src, t0, dt, Ld)
        assert rel_err(Ld.cpu().numpy(), L_ref) < 1e-12
        s0 = np.random.default_rng(418).standard_normal(d.state_off[-1])
        U_ref = d.solve_direct(s0, dt, L_ref)
        st = lib.dev(s0, t.float64)
        Ud = t.zeros(d.trial_off[-1], dtype=t.float64, device="cuda")
        note("local time solve with source")
        info = lib.stdg.stdg_slab_solve(mh, t0, dt, Ld, st, inner_prec=1, rtol=1e-13, max_iters=800,
                                        max_refine=80, slab_U=Ud, krylov_prec=1)
        assert info["status"] == 0, info
        assert rel_err(Ud.cpu().numpy(), U_ref) < 1e-10
    finally:
        lib.stdg.stdg_mesh_free(mh)


def test_dual_norm_and_inexact_march(lib):
    # dual norms with test functions on dt / n, and eta_it bounding the
    # iteration error of an inexact march (Section 5.3)
    mesh = _mesh((2, 2, 1), p=2, q=2, nsub=(1, 2, 4), seed=419, mixed=True)
    d = oracle_disc(mesh)
    rng = np.random.default_rng(419)
    dt, n_slabs = 0.05, 3
    mh = lib.upload(mesh)
    try:
        R = rng.standard_normal(d.unk_off[-1])
        note("local time dual norm")
        got = lib.stdg.stdg_residual_dual_norm(mh, dt, lib.dev(R, lib.torch.float64))
        ref = d.dual_norms(R, dt)
        assert np.abs(np.asarray(got) - ref).max() < 1e-12 * ref.max()
        s = rng.standard_normal(d.state_off[-1])
        e0 = d.energy(s)
        eta_tol = 1e-4 * np.sqrt(2 * e0)
        st = lib.dev(s, lib.torch.float64)
        s_ex, eta2 = s.copy(), 0.0
        for n in range(n_slabs):
            note("local time inexact slab %d" % n)
            r = lib.stdg.stdg_slab_solve(mh, n * dt, dt, None, st, inner_prec=1, krylov_prec=1, rtol=1e-12,
                                         max_iters=2000, max_refine=200, eta_tol=eta_tol, eta_t_final=n_slabs * dt)
            assert r["status"] == 0, r
            assert r["eta2"] <= eta_tol ** 2
            eta2 += r["eta2"]
            s_ex = d.level_state(d.solve_direct(s_ex, dt), 1)
        err2 = 2.0 * d.energy(st.cpu().numpy() - s_ex)
        assert err2 <= eta2, (err2, eta2)
    finally:
        lib.stdg.stdg_mesh_free(mh)


def test_serving_request_matches_plain_march(lib):
    # a serving request with local time steps (a source and a mode-free
    # initial state) is bitwise the plain march of the same slabs
    stdg = lib.stdg
    mesh = _mesh((2, 2, 2), p=2, q=2, nsub=(1, 2, 4), seed=420, mixed=True)
    src = synth.Source(kind=1, amp=1.0, center=(0.5, 0.5, 0.5), sigma_x=0.2, f0=2.0, t0=0.05,
                       sigma_t=0.1, dir=(0.0, 0.0, 1.0))
    init = np.random.default_rng(420).standard_normal(mesh.state_size())
    dt, n_slabs = 0.04, 3
    opts = dict(inner_prec=1, rtol=1e-12, max_iters=3000, max_refine=300)
    srv = stdg.stdg_serve_start(lib.ctx, hbm_budget=1 << 28, **opts)
    try:
        note("local time serving request")
        t = stdg.stdg_serve_submit(srv, mesh.vertices, mesh.hexes, mesh.p, mesh.q, mesh.eps, mesh.mu, 0.0, dt,
                                   n_slabs, source=src, init_state=init, nsub=mesh.nsub)
        st_out = np.zeros(mesh.state_size())
        res = None
        for _ in range(60000):
            res = stdg.stdg_serve_poll(srv, t, st_out)
            if res is not None:
                break
            import time
            time.sleep(0.002)
        assert res is not None and res["status"] == 0, res
    finally:
        stdg.stdg_serve_stop(srv)
    mh = lib.upload(mesh)
    try:
        info = stdg.stdg_mesh_info(mh)
        st = lib.dev(init, lib.torch.float64)
        L = lib.torch.zeros(info["unknown_size"], dtype=lib.torch.float64, device="cuda")
        note("local time plain march")
        for n in range(n_slabs):
            stdg.stdg_load_assemble(mh, src, n * dt, dt, L)
            assert stdg.stdg_slab_solve(mh, n * dt, dt, L, st, **opts)["status"] == 0
        ref = st.cpu().numpy()
    finally:
        stdg.stdg_mesh_free(mh)
    assert np.array_equal(ref, st_out)


@pytest.mark.parametrize("prec", [0, 1])
def test_local_time_cavity_32cubed_sampled(lib, prec):
    # the benchmark's local-time workload at full size (32^3, p = 4, q = 3,
    # 4 / 2 / 1 sub-intervals) in the launch configuration it times; the
    # oracle checks sampled elements on both sides of x = 0.25 and x = 0.5
    stdg = lib.stdg
    cfg = synth.local_time_cavity()
    m = cfg["mesh"]
    dt = cfg["dt"]
    note("local time 32^3 prec=%d: inputs" % prec)
    d = oracle_disc(m)
    x = synth.random_vector(d.unk_off[-1], 0)
    if prec == 1:
        x = x.astype(np.float32).astype(np.float64)
    mh = lib.upload(m)
    try:
        rng = np.random.default_rng(43)
        c = synth.centroids(m.vertices, m.hexes)
        near = [int(e) for e in np.flatnonzero((np.abs(c[:, 0] - 0.25) < 0.02) | (np.abs(c[:, 0] - 0.5) < 0.02))]
        sample = sorted(set(int(e) for e in rng.choice(m.n_elements, 24, replace=False)) |
                        set(int(e) for e in rng.choice(near, 24, replace=False)))
        needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
        for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
            note("local time 32^3 prec=%d mode=%d: apply" % (prec, mode))
            y = lib.apply(mh, dt, prec, mode, x)
            assert np.all(np.isfinite(y))
            xin = d.precond_solve(x, needed) if mode == stdg.STDG_OPERATOR_PRECOND else x
            rows = d.apply_rows(d.embed_unknowns(xin, elements=needed), dt, sample)
            got = np.concatenate([y[d.unk_off[e]:d.unk_off[e + 1]] for e in sample])
            ref = np.concatenate([rows[e] for e in sample])
            note("local time 32^3 prec=%d mode=%d rel err %.3e" % (prec, mode, rel_err(got, ref)))
            assert rel_err(got, ref) < TOL[prec]
    finally:
        stdg.stdg_mesh_free(mh)


def test_temporal_order_march(lib):
    # Section 6.1.2 with local time steps: the manufactured exp solution
    # marched by the library (its current integrated by the oracle, since the
    # library's load takes the Gaussian pulse only) equals the oracle's march
    # and keeps the nodal order 2 q
    from oracle import fields
    F, J = fields.exp_solution()
    v, h = synth.box_mesh((2, 1, 1))
    q = 2
    mesh = synth.Mesh(v, h, np.full(2, 2, np.int32), np.full(2, q, np.int32), np.ones(2), np.ones(2),
                      nsub=np.array([1, 2], np.int32))
    d = oracle_disc(mesh)
    mh = lib.upload(mesh)
    T, errs = 0.4, []
    try:
        for nsteps in (2, 4):
            dt = T / nsteps
            s = fields.reference_coefficients(d, F, 0.0)
            st = lib.dev(s, lib.torch.float64)
            for n in range(nsteps):
                L = d.load(J, n * dt, dt, nt=q + 8)
                s = d.level_state(d.solve_direct(s, dt, L), 1)
                note("local time exp march %d/%d" % (n, nsteps))
                r = lib.stdg.stdg_slab_solve(mh, n * dt, dt, lib.dev(L, lib.torch.float64), st, inner_prec=1,
                                             rtol=1e-13, max_iters=800, max_refine=80, krylov_prec=1)
                assert r["status"] == 0, r
            got = st.cpu().numpy()
            assert rel_err(got, s) < 1e-10
            errs.append(np.abs(got - fields.reference_coefficients(d, F, T)).max())
    finally:
        lib.stdg.stdg_mesh_free(mh)
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - 2 * q) < 0.3, (errs, rate)


@pytest.mark.parametrize("shear,big", [(False, False), (True, False), (False, True)])
def test_dissipation(lib, shear, big):
    # D_h with local time steps: the test function projected onto each face
    # pair's common temporal test space (own and neighbour trial), in every
    # mode and precision, and a slab solve with the oracle's energy drop;
    # big: p = 4, q = 4, whose FP64 traces exceed the staged LDS and are
    # gathered per level
    from oracle.dg import Discretisation
    stdg = lib.stdg
    if big:
        mesh = _mesh((2, 1, 1), p=4, q=4, nsub=(1,), seed=424)
        mesh.nsub[:] = (1, 2)
    else:
        mesh = _mesh((2, 2, 2), p=2, q=2, nsub=(1, 2, 4), seed=422 + shear, mixed=True, shear=shear)
    c = 0.7
    d = Discretisation(mesh.vertices, mesh.hexes, mesh.p, mesh.q, mesh.eps, mesh.mu, c_diss=c, nk=mesh.nsub)
    rng = np.random.default_rng(422)
    x = rng.standard_normal(d.unk_off[-1])
    U = rng.standard_normal(d.trial_off[-1])
    L = rng.standard_normal(d.unk_off[-1])
    dt = 0.05
    mh = lib.upload(mesh)
    try:
        stdg.stdg_mesh_set_dissipation(mh, c)
        for prec in (0, 1):
            cast = (lambda v: v) if prec == 0 else (lambda v: v.astype(np.float32).astype(np.float64))
            xs, Us, Ls = cast(x), cast(U), cast(L)
            note("local time D_h shear=%d big=%d prec=%d" % (shear, big, prec))
            assert rel_err(lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xs), d.operator(xs, dt)) < TOL[prec]
            assert rel_err(lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls), d.residual(Us, dt, Ls)) < TOL[prec]
            assert rel_err(lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs),
                           d.operator(d.precond_solve(xs), dt)) < TOL[prec]
        if big:
            return  # (the oracle's direct solve of this one takes half a minute)
        s0 = rng.standard_normal(d.state_off[-1])
        ref = d.level_state(d.solve_direct(s0, dt), 1)
        st = lib.dev(s0, lib.torch.float64)
        note("local time D_h shear=%d big=%d: solve" % (shear, big))
        r = stdg.stdg_slab_solve(mh, 0.0, dt, None, st, inner_prec=1, rtol=1e-13, max_iters=800, max_refine=80,
                                 krylov_prec=1)
        assert r["status"] == 0, r
        assert rel_err(st.cpu().numpy(), ref) < 1e-10
        assert d.energy(ref) < d.energy(s0)
    finally:
        stdg.stdg_mesh_free(mh)


def test_refusals(lib):
    stdg = lib.stdg
    # D_h with local time steps at p = 5, q = 5 (beyond the kernel's registers)
    big = _mesh((2, 1, 1), p=5, q=5, nsub=(2,), seed=415)
    mh = lib.upload(big)
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
