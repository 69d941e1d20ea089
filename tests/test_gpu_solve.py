"""GPU parity of the slab solve (Section 3 eq. weakform / Section 4 eq.
weakform_stabilized, GMRES of Section 5.4), the load (eq. bilinearform:C), the
mode projection and the energy (eq. stability:energydef), through the C ABI,
against the oracle.  Bars: FP64 path and FP32+refinement <= 1e-10 relative to
the oracle's direct solve; energy conserved without sources (Thm 3.1, 4.1)."""
import numpy as np
import pytest

import synth
from oracle import fields
from tests.gpu_util import Lib, note, oracle_disc, rel_err

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


@pytest.mark.parametrize("inner,krylov", [(1, 0), (0, 0), (1, 1)])
def test_two_material_32cubed_first_slab_properties(lib, inner, krylov):
    """Full-size 32^3 p = 4 q = 3 solve of the first slab: energy conserved and
    the oracle's residual on sampled elements of the GPU solution is small."""
    cfg = synth.cavity_two_material()
    m = cfg["mesh"]
    modes = cfg["init"]
    mh = lib.upload(m)
    info_m = lib.stdg.stdg_mesh_info(mh)
    st = lib.torch.zeros(info_m["state_size"], dtype=lib.torch.float64, device="cuda")
    lib.stdg.stdg_project_modes(mh, modes.mnl, modes.abc, st)
    s0 = st.cpu().numpy()
    Ud = lib.torch.zeros(info_m["trial_size"], dtype=lib.torch.float64, device="cuda")
    note("32^3 solve inner=%d krylov=%d" % (inner, krylov))
    info = lib.stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, st, inner_prec=inner, rtol=1e-10, slab_U=Ud,
                                    krylov_prec=krylov, max_iters=2000, max_refine=300)
    note("32^3 solve inner=%d krylov=%d: %s" % (inner, krylov, info))
    assert info["status"] == 0
    assert abs(info["energy_end"] - info["energy_start"]) < 1e-9 * info["energy_start"]
    d = oracle_disc(m)
    U = Ud.cpu().numpy()
    x0 = np.zeros(d.unk_off[-1])
    for e in range(d.ne):
        a3 = int(d.a[e]) ** 3
        qe = int(d.q[e])
        x0[d.unk_off[e]:d.unk_off[e + 1]].reshape(2, 3, qe, a3)[:, :, 0, :] = \
            s0[d.state_off[e]:d.state_off[e + 1]].reshape(2, 3, a3)
    U0 = d.embed_unknowns(x0, s0)   # the solver's initial guess: constant continuation
    rng = np.random.default_rng(3)
    sample = [int(e) for e in rng.choice(m.n_elements, 24, replace=False)]
    r = d.residual(U, cfg["dt"], None, sample)
    r0 = d.residual(U0, cfg["dt"], None, sample)
    num = np.sqrt(sum(np.sum(v ** 2) for v in r.values()))
    den = np.sqrt(sum(np.sum(v ** 2) for v in r0.values()))
    assert num / den < 1e-8, num / den
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
