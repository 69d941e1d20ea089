"""GPU parity of the slab solve (Section 3 eq. weakform / Section 4 eq.
weakform_stabilized, GMRES of Section 5.4), the load (eq. bilinearform:C), the
mode projection and the energy (eq. stability:energydef), through the C ABI,
against the oracle.  Bars: FP64 path and FP32+refinement <= 1e-10 relative to
the oracle's direct solve; energy conserved without sources (Thm 3.1, 4.1)."""
import numpy as np
import pytest

import synth
from oracle import fields
from tests.gpu_util import Lib, note, oracle_disc, rel_err, rel_err_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _state_dev(lib, arr):
    return lib.dev(arr, lib.torch.float64)


def test_mode_projection_and_energy_te101(lib):
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = oracle_disc(m)
    mh = lib.upload(m)
    st = lib.torch.zeros(d.state_off[-1], dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_project_modes(mh, [[1, 0, 1]], [[0.0, 1.0, 0.0]], st)
    got = st.cpu().numpy()
    ref = fields.project(d, fields.te101, 0.0)
    assert rel_err(got, ref) < 1e-12
    e = lib.stdg.stdg_energy(mh, st)
    assert abs(e - d.energy(ref)) < 1e-12 * d.energy(ref)
    lib.stdg.stdg_mesh_free(mh)


def test_mode_superposition_projection(lib):
    cfg = synth.cavity_two_material(n=3, p=3, q=2)
    m = cfg["mesh"]
    modes = cfg["init"]
    d = oracle_disc(m)
    mh = lib.upload(m)
    st = lib.torch.zeros(d.state_off[-1], dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_project_modes(mh, modes.mnl, modes.abc, st)
    ref = fields.project(d, fields.mode_superposition(modes.mnl, modes.abc), 0.0)
    assert rel_err(st.cpu().numpy(), ref) < 1e-12
    lib.stdg.stdg_mesh_free(mh)


SOLVE_PATHS = [(0, 0), (1, 0), (1, 1)]  # (inner applies, Krylov basis storage): FP64 = 0, FP32 = 1


@pytest.mark.parametrize("inner,krylov", SOLVE_PATHS)
def test_slab_solve_te101_cavity(lib, inner, krylov):
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = oracle_disc(m)
    s0 = fields.project(d, fields.te101, 0.0)
    U_ref = d.solve_direct(s0, cfg["dt"])
    mh = lib.upload(m)
    st = _state_dev(lib, s0)
    Ud = lib.torch.zeros(d.trial_off[-1], dtype=lib.torch.float64, device="cuda")
    note("te101 solve inner=%d krylov=%d" % (inner, krylov))
    info = lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=inner, rtol=1e-13,
                                    max_iters=400, max_refine=40, slab_U=Ud, krylov_prec=krylov)
    assert info["status"] == 0, info
    assert rel_err(Ud.cpu().numpy(), U_ref) < 1e-10
    assert rel_err(st.cpu().numpy(), d.level_state(U_ref, 1)) < 1e-10
    assert abs(info["energy_end"] - info["energy_start"]) < 1e-10 * info["energy_start"]
    lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("inner,krylov", SOLVE_PATHS)
def test_slab_solve_mixed_degrees_with_source(lib, inner, krylov):
    v, h = synth.box_mesh((3, 2, 2))
    ne = h.shape[0]
    rng = np.random.default_rng(21)
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
    st = _state_dev(lib, s0)
    Ud = lib.torch.zeros(d.trial_off[-1], dtype=lib.torch.float64, device="cuda")
    info = lib.stdg.stdg_slab_solve(mh, t0, dt, Ld, st, inner_prec=inner, rtol=1e-13, max_iters=600,
                                    max_refine=60, slab_U=Ud, krylov_prec=krylov)
    assert info["status"] == 0, info
    assert rel_err(Ud.cpu().numpy(), U_ref) < 1e-10
    lib.stdg.stdg_mesh_free(mh)


def test_slab_solve_bitwise_repeatable_and_option_checks(lib):
    cfg = synth.cavity_two_material(n=4, p=3, q=2)
    m = cfg["mesh"]
    mh = lib.upload(m)
    info_m = lib.stdg.stdg_mesh_info(mh)
    s0 = np.random.default_rng(3).standard_normal(info_m["state_size"])
    outs = []
    for _ in range(2):
        st = lib.dev(s0, lib.torch.float64)
        r = lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=1, rtol=1e-12, max_iters=400,
                                     max_refine=40)
        assert r["status"] == 0
        outs.append(st.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    st = lib.dev(s0, lib.torch.float64)
    with pytest.raises(lib.stdg.StdgError):  # an FP32 basis needs FP32 applies
        lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=0, krylov_prec=1)
    with pytest.raises(lib.stdg.StdgError):  # restart + 1 must fit the basis
        lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=0, restart=40)
    lib.stdg.stdg_mesh_free(mh)


def test_three_slab_march_matches_oracle(lib):
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = oracle_disc(m)
    s = fields.project(d, fields.te101, 0.0)
    mh = lib.upload(m)
    st = _state_dev(lib, s)
    for n in range(3):
        info = lib.stdg.stdg_slab_solve(mh, n * cfg["dt"], cfg["dt"], None, st, inner_prec=1, rtol=1e-13,
                                        max_iters=400, max_refine=40)
        assert info["status"] == 0
        s = d.level_state(d.solve_direct(s, cfg["dt"]), 1)
        assert rel_err(st.cpu().numpy(), s) < 1e-10
    lib.stdg.stdg_mesh_free(mh)


def test_not_converged_reports_and_fills_info(lib):
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = oracle_disc(m)
    mh = lib.upload(m)
    st = _state_dev(lib, fields.project(d, fields.te101, 0.0))
    info = lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=0, rtol=1e-14, max_iters=1)
    assert info["status"] == -5
    assert info["iters"] == 1 and 0 < info["rel_res"] < 1
    lib.stdg.stdg_mesh_free(mh)


def _initial_guess(d, s0, elements):
    """The solver's initial guess on the given elements (others 0): constant
    continuation, m = 1 block := the state at the slab start, higher levels 0."""
    x0 = np.zeros(d.unk_off[-1])
    for e in elements:
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        x0[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)[:, :, 0, :] = \
            s0[d.state_off[e]:d.state_off[e + 1]].reshape(2, 3, a3)
    return d.embed_unknowns(x0, s0, elements)


def _sampled_residual_ratio(d, U, U0, dt, load, sample):
    """||R(U)|| / ||R(U0)|| of the oracle's residual on the sampled elements'
    rows (R = B U - L; the load restricted to those rows)."""
    r = d.residual(U, dt, None, sample)
    r0 = d.residual(U0, dt, None, sample)
    if load is not None:
        for e in sample:
            r[e] = r[e] - load[d.unk_off[e]:d.unk_off[e + 1]]
            r0[e] = r0[e] - load[d.unk_off[e]:d.unk_off[e + 1]]
    num = np.sqrt(sum(np.sum(v ** 2) for v in r.values()))
    den = np.sqrt(sum(np.sum(v ** 2) for v in r0.values()))
    return num / den


def _full_size_slab(lib, m, mh, d, s0, dt, load_dev, load_host, sample, rtol):
    """One slab from s0 with plain FP64 and with FP32 applies inside FP64
    refinement (FP32 basis): the end states match elementwise to 1e-10, the
    slab solutions on the sampled elements and their neighbours too, and both
    satisfy the oracle's equations on the sampled elements to 1e-10 of the
    initial guess's residual.  Only those elements' trial blocks come back
    to the host."""
    t = lib.torch
    needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
    outs = {}
    for name, inner, krylov in (("fp64", 0, 0), ("fp32_refine", 1, 1)):
        st = lib.dev(s0, t.float64)
        Ud = t.zeros(m.trial_size(), dtype=t.float64, device="cuda")
        note("full-size slab %s rtol %g" % (name, rtol))
        info = lib.stdg.stdg_slab_solve(mh, 0.0, dt, load_dev, st, inner_prec=inner, krylov_prec=krylov, rtol=rtol,
                                        slab_U=Ud, max_iters=4000, max_refine=400)
        note("full-size slab %s: %s" % (name, info))
        assert info["status"] == 0 and info["rel_res"] <= rtol
        U = np.zeros(d.trial_off[-1])
        for e in needed:
            U[d.trial_off[e]:d.trial_off[e + 1]] = Ud[d.trial_off[e]:d.trial_off[e + 1]].cpu().numpy()
        outs[name] = (st.cpu().numpy(), U, info)
        del st, Ud
    err = rel_err(outs["fp32_refine"][0], outs["fp64"][0])
    note("full-size slab: FP32+refinement vs FP64 end state %.3e" % err)
    assert err < 1e-10
    blocks = lambda U: np.concatenate([U[d.trial_off[e]:d.trial_off[e + 1]] for e in needed])
    assert rel_err(blocks(outs["fp32_refine"][1]), blocks(outs["fp64"][1])) < 1e-10
    U0 = _initial_guess(d, s0, needed)
    for name in outs:
        ratio = _sampled_residual_ratio(d, outs[name][1], U0, dt, load_host, sample)
        note("full-size slab %s: oracle residual on %d sampled elements %.3e" % (name, len(sample), ratio))
        assert ratio < 1e-10
    return outs


def test_two_material_32cubed_first_slab(lib):
    """Full-size 32^3 p = 4 q = 3 two-material cavity, first slab from the
    projected mode superposition: FP32+refinement and plain FP64 agree to 1e-10
    elementwise, the oracle's residual on sampled elements is below 1e-10 of
    its initial value, and the energy is conserved (Thm 3.1)."""
    cfg = synth.cavity_two_material()
    m = cfg["mesh"]
    modes = cfg["init"]
    mh = lib.upload(m)
    try:
        st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
        lib.stdg.stdg_project_modes(mh, modes.mnl, modes.abc, st)
        s0 = st.cpu().numpy()
        d = oracle_disc(m)
        sample = [int(e) for e in np.random.default_rng(3).choice(m.n_elements, 24, replace=False)]
        outs = _full_size_slab(lib, m, mh, d, s0, cfg["dt"], None, None, sample, 1e-11)
        for name, (_, _, info) in outs.items():
            assert abs(info["energy_end"] - info["energy_start"]) < 1e-10 * info["energy_start"]
    finally:
        lib.stdg.stdg_mesh_free(mh)


def test_two_material_32cubed_march_64_slabs(lib):
    """The benchmark's 64-slab march of the 32^3 cavity at its tolerance (rtol
    1e-10 per slab): on every slab, FP32 applies inside FP64 refinement (FP32
    basis) reach the plain FP64 path's end state to 1e-10, each started from
    the FP64 march's state; the FP64 march conserves the energy (Thm 3.1).
    Two uploads of the mesh keep one cached solver per precision."""
    t = lib.torch
    cfg = synth.cavity_two_material()
    m = cfg["mesh"]
    modes = cfg["init"]
    dt = cfg["dt"]
    mh64 = lib.upload(m)
    mh32 = lib.upload(m)
    try:
        st = t.zeros(m.state_size(), dtype=t.float64, device="cuda")
        lib.stdg.stdg_project_modes(mh64, modes.mnl, modes.abc, st)
        e0 = lib.stdg.stdg_energy(mh64, st)
        worst = 0.0
        for n in range(cfg["n_slabs"]):
            s32 = st.clone()
            r64 = lib.stdg.stdg_slab_solve(mh64, n * dt, dt, None, st, inner_prec=0, rtol=1e-10, max_iters=4000,
                                           max_refine=400)
            r32 = lib.stdg.stdg_slab_solve(mh32, n * dt, dt, None, s32, inner_prec=1, krylov_prec=1, rtol=1e-10,
                                           max_iters=4000, max_refine=400)
            assert r64["status"] == 0 and r32["status"] == 0
            err = rel_err_dev(s32, st)
            worst = max(worst, err)
            if n % 8 == 0 or err >= 1e-10:
                note("64-slab march: slab %d iters %d / %d, FP32+refinement vs FP64 %.3e"
                     % (n, r64["iters"], r32["iters"], err))
            assert err < 1e-10, (n, err)
        e1 = lib.stdg.stdg_energy(mh64, st)
        note("64-slab march: worst slab difference %.3e, energy drift %.3e" % (worst, (e1 - e0) / e0))
        assert abs(e1 - e0) < 1e-8 * e0
    finally:
        lib.stdg.stdg_mesh_free(mh64)
        lib.stdg.stdg_mesh_free(mh32)


def test_graded_trilinear_24cubed_slab_with_source(lib):
    """Full-size graded trilinear 24^3 mesh (p = 3..6, q = p - 2) driven by its
    Gaussian-pulse current, one slab from a random field: FP32+refinement vs
    FP64 to 1e-10 elementwise; the oracle's residual (its own load) on sampled
    elements of every (p, q) ring below 1e-10 of its initial value."""
    cfg = synth.graded_nonaffine()
    m = cfg["mesh"]
    dt = cfg["dt"]
    src = cfg["source"]
    mh = lib.upload(m)
    try:
        t0 = src.t0 - dt
        Ld = lib.torch.zeros(m.unknown_size(), dtype=lib.torch.float64, device="cuda")
        lib.stdg.stdg_load_assemble(mh, src, t0, dt, Ld)
        d = oracle_disc(m)
        rng = np.random.default_rng(24)
        sample = []
        for p in (3, 4, 5, 6):
            ids = np.nonzero(m.p == p)[0]
            sample += [int(e) for e in rng.choice(ids, 3, replace=False)]
        J = fields.gaussian_pulse(src.amp, src.center, src.sigma_x, src.f0, src.t0, src.sigma_t, src.dir)
        Ls = d.load_rows(J, t0, dt, sample)
        Lg = Ld.cpu().numpy()
        L_host = np.zeros(d.unk_off[-1])
        for e in sample:
            assert rel_err(Lg[d.unk_off[e]:d.unk_off[e + 1]], Ls[e]) < 1e-12
            L_host[d.unk_off[e]:d.unk_off[e + 1]] = Ls[e]
        s0 = 1e-3 * synth.random_vector(m.state_size(), 25)
        _full_size_slab(lib, m, mh, d, s0, dt, Ld, L_host, sample, 1e-11)
    finally:
        lib.stdg.stdg_mesh_free(mh)


def test_large_cavity_48cubed_slab_with_source(lib):
    """Full-size 48^3 p = 6 q = 4 cavity (1.1e9 trial DoF) driven by its
    current, one slab from a random field: FP32+refinement vs FP64 to 1e-10
    elementwise and the oracle's residual on sampled elements below 1e-10."""
    cfg = synth.large_cavity()
    m = cfg["mesh"]
    dt = cfg["dt"]
    src = cfg["source"]
    mh = lib.upload(m)
    try:
        t0 = src.t0 - dt
        Ld = lib.torch.zeros(m.unknown_size(), dtype=lib.torch.float64, device="cuda")
        lib.stdg.stdg_load_assemble(mh, src, t0, dt, Ld)
        d = oracle_disc(m)
        rng = np.random.default_rng(48)
        sample = [int(e) for e in rng.choice(m.n_elements, 8, replace=False)] + [0, m.n_elements - 1]
        J = fields.gaussian_pulse(src.amp, src.center, src.sigma_x, src.f0, src.t0, src.sigma_t, src.dir)
        Ls = d.load_rows(J, t0, dt, sample)
        Lg = Ld.cpu().numpy()
        L_host = np.zeros(d.unk_off[-1])
        for e in sample:
            assert rel_err(Lg[d.unk_off[e]:d.unk_off[e + 1]], Ls[e]) < 1e-12
            L_host[d.unk_off[e]:d.unk_off[e + 1]] = Ls[e]
        s0 = 1e-3 * synth.random_vector(m.state_size(), 49)
        _full_size_slab(lib, m, mh, d, s0, dt, Ld, L_host, sample, 1e-11)
    finally:
        lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_iteration_counts_order_of_magnitude(lib, p):
    """Solver realism (the iteration table of Section 5.4.1): an 8^3 cube with
    a T_mm cavity mode, q = p, dt = h / (2p + 1), m = 1, 2, 3 for p in {1, 2},
    {3, 4}, {5, 6}; the paper reports 8 to 25 GMRES iterations per slab for
    exact solves (tolerance unstated).  Checked to an order of magnitude over
    a few slabs at rtol 1e-10."""
    v, h = synth.box_mesh((8, 8, 8))
    ne = h.shape[0]
    m = synth.Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, p, np.int32), np.ones(ne), np.ones(ne),
                   shape=(8, 8, 8))
    mm = (p + 1) // 2
    dt = (1.0 / 8) / (2 * p + 1)
    mh = lib.upload(m)
    try:
        st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
        lib.stdg.stdg_project_modes(mh, [[mm, 0, mm]], [[0.0, 1.0, 0.0]], st)
        its = []
        for n in range(4):
            r = lib.stdg.stdg_slab_solve(mh, n * dt, dt, None, st, inner_prec=0, rtol=1e-10, max_iters=2000,
                                         max_refine=200)
            assert r["status"] == 0
            its.append(r["iters"])
        note("E1 p=%d: iterations per slab %s" % (p, its))
        assert 3 <= np.mean(its) <= 100
    finally:
        lib.stdg.stdg_mesh_free(mh)


def test_resume_from_saved_state_is_bitwise(lib):
    # the method is one-step (each slab starts from the previous end state):
    # saving the FP64 state after two slabs and resuming on a fresh mesh
    # handle gives bitwise the same third slab as the uninterrupted march
    cfg = synth.cavity_two_material(n=3, p=3, q=2)
    m = cfg["mesh"]
    modes = cfg["init"]
    opts = dict(inner_prec=1, rtol=1e-12, max_iters=2000, max_refine=200, krylov_prec=1)
    mh = lib.upload(m)
    st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_project_modes(mh, modes.mnl, modes.abc, st)
    saved = None
    for n in range(3):
        if n == 2:
            saved = st.cpu().numpy().copy()
        assert lib.stdg.stdg_slab_solve(mh, n * cfg["dt"], cfg["dt"], None, st, **opts)["status"] == 0
    straight = st.cpu().numpy()
    lib.stdg.stdg_mesh_free(mh)
    mh = lib.upload(m)
    st2 = _state_dev(lib, saved)
    assert lib.stdg.stdg_slab_solve(mh, 2 * cfg["dt"], cfg["dt"], None, st2, **opts)["status"] == 0
    lib.stdg.stdg_mesh_free(mh)
    assert np.array_equal(st2.cpu().numpy(), straight)


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1), (1, 0)])
def test_graph_replay_several_groups_is_bitwise(lib, inner, krylov):
    """Restart cycles replayed as graphs on a mesh with several kernel groups
    (the side-stream fork and join of the group launches are captured; a
    trilinear mesh with mixed degrees, so the P^{-1} pre-pass too): bitwise the
    direct launches over a march with a dt change."""
    from tests.gpu_util import random_mixed_mesh
    m = random_mixed_mesh((3, 3, 2), 4, 3, 77)
    m = synth.Mesh(synth.perturb_interior(m.vertices, (3, 3, 2), 0.1, 78), m.hexes, m.p, m.q, m.eps, m.mu,
                   shape=m.shape)
    opts = dict(inner_prec=inner, krylov_prec=krylov, rtol=1e-12, max_iters=3000, max_refine=300)
    s0 = synth.random_vector(m.state_size(), 79)
    out = []
    for graph in (False, True):
        mh = lib.upload(m)
        try:
            assert lib.stdg.stdg_mesh_info(mh)["n_groups"] > 3
            st = lib.dev(s0, lib.torch.float64)
            iters = 0
            for n, dt in enumerate((0.02, 0.02, 0.03)):
                note("graph=%d several groups slab %d" % (graph, n))
                r = lib.stdg.stdg_slab_solve(mh, 0.0, dt, None, st, use_graph=graph, **opts)
                assert r["status"] == 0
                iters += r["iters"]
            out.append((st.cpu().numpy(), iters))
        finally:
            lib.stdg.stdg_mesh_free(mh)
    assert out[0][1] == out[1][1] and out[0][1] > 20
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("inner,krylov", [(0, 0), (1, 1)])
def test_graph_replay_is_bitwise(lib, inner, krylov):
    """Arnoldi iterations replayed as captured HIP graphs give bitwise the
    direct launches' result, over a march whose graphs are replayed many
    times with eager work between them, across a change of dt (recapture) and
    on a sheared mesh (preconditioner pre-pass with its scratch)."""
    for shear in (False, True):
        cfg = synth.cavity_two_material(n=4, p=3, q=2)
        m = cfg["mesh"]
        if shear:
            m = synth.Mesh(synth.affine_transform(m.vertices, np.array([[1.0, 0.2, 0.0], [0.0, 1.0, 0.1],
                                                                          [0.1, 0.0, 1.0]])),
                           m.hexes, m.p, m.q, m.eps, m.mu, shape=m.shape)
        modes = cfg["init"]
        opts = dict(inner_prec=inner, krylov_prec=krylov, rtol=1e-12, max_iters=3000, max_refine=300)
        out = []
        for graph in (False, True):
            mh = lib.upload(m)
            st = lib.torch.zeros(m.state_size(), dtype=lib.torch.float64, device="cuda")
            if shear:
                st.copy_(lib.torch.from_numpy(synth.random_vector(m.state_size(), 5)))
            else:
                lib.stdg.stdg_project_modes(mh, modes.mnl, modes.abc, st)
            iters = 0
            for n, dt in enumerate((0.01, 0.01, 0.01, 0.02, 0.02)):
                note("graph=%d shear=%d slab %d" % (graph, shear, n))
                r = lib.stdg.stdg_slab_solve(mh, 0.0, dt, None, st, use_graph=graph, **opts)
                assert r["status"] == 0
                iters += r["iters"]
            out.append((st.cpu().numpy(), iters))
            lib.stdg.stdg_mesh_free(mh)
        assert out[0][1] == out[1][1] and out[0][1] > 20
        assert np.array_equal(out[0][0], out[1][0])


def _march(lib, m, steps, graph, state0):
    """Run `steps` (callables taking (mesh handle, state tensor, graph flag)) on
    a fresh upload of m; returns the states after each step."""
    mh = lib.upload(m)
    st = lib.dev(state0, lib.torch.float64)
    out = []
    try:
        for step in steps:
            step(mh, st, graph)
            out.append(st.cpu().numpy().copy())
    finally:
        lib.stdg.stdg_mesh_free(mh)
    return out


def test_graphs_recaptured_after_mesh_changes(lib):
    """Captured Arnoldi iterations are dropped when the mesh changes what they
    read: the dissipative coefficients switched off between two graph solves,
    and (sheared mesh) an FP64 preconditioned apply between two FP32 graph
    solves.  Each sequence is bitwise the same sequence without graphs."""
    stdg = lib.stdg
    cfg = synth.cavity_two_material(n=4, p=3, q=2)
    m = cfg["mesh"]
    s0 = synth.random_vector(m.state_size(), 8)
    opts = dict(inner_prec=1, krylov_prec=1, rtol=1e-12, max_iters=3000, max_refine=300)

    def solve(mh, st, graph):
        r = stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, use_graph=graph, **opts)
        assert r["status"] == 0 and r["iters"] > 12

    def diss(c):
        return lambda mh, st, graph: stdg.stdg_mesh_set_dissipation(mh, c)
    steps = [diss(0.5), solve, diss(0.0), solve, diss(0.8), solve]
    note("graph epoch: dissipation on / off between graph solves")
    ref = _march(lib, m, steps, False, s0)
    got = _march(lib, m, steps, True, s0)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)

    ms = synth.Mesh(synth.affine_transform(m.vertices, np.array([[1.0, 0.2, 0.0], [0.0, 1.0, 0.1],
                                                                   [0.1, 0.0, 1.0]])),
                    m.hexes, m.p, m.q, m.eps, m.mu, shape=m.shape)
    xr = synth.random_vector(m.unknown_size(), 9)

    def apply64(mh, st, graph):
        x = lib.dev(xr, lib.torch.float64)
        y = lib.torch.empty_like(x)
        stdg.stdg_residual_apply(mh, cfg["dt"], stdg.STDG_FP64, stdg.STDG_OPERATOR_PRECOND, x, None, y)
        lib.torch.cuda.synchronize()
    steps = [solve, apply64, solve, solve]
    note("graph epoch: sheared mesh, FP64 preconditioned apply between FP32 graph solves")
    ref = _march(lib, ms, steps, False, s0)
    got = _march(lib, ms, steps, True, s0)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
