"""GPU parity of stdg_residual_apply (the slab residual, Section 5 eq. residual)
against the FP64 oracle on the same seeded inputs, through the C ABI.

Bars: FP64 <= 1e-12, raw FP32 apply <= 1e-5, each for the relative 2-norm
error and for the largest entry error relative to the largest reference entry
(the FP32 inputs are the float32 roundings of the FP64 ones and the oracle is
run on exactly those values)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note, oracle_disc, random_mixed_mesh, rel_err

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _check_all_modes(lib, mesh, dt, seed, name, precs=(0, 1), with_precond=True, elements=None):
    stdg = lib.stdg
    d = oracle_disc(mesh)
    mh = lib.upload(mesh)
    rng = np.random.default_rng(seed)
    nu, nt = d.unk_off[-1], d.trial_off[-1]
    x = rng.standard_normal(nu)
    U = rng.standard_normal(nt)
    L = rng.standard_normal(nu)
    try:
        for prec in precs:
            cast = (lambda v: v) if prec == 0 else (lambda v: v.astype(np.float32).astype(np.float64))
            xs, Us, Ls = cast(x), cast(U), cast(L)
            note("%s prec=%d operator" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xs)
            ref = d.operator(xs, dt)
            assert rel_err(got, ref) < TOL[prec], (name, prec, "operator", rel_err(got, ref))
            note("%s prec=%d residual" % (name, prec))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, Ls)
            ref = d.residual(Us, dt, Ls)
            assert rel_err(got, ref) < TOL[prec], (name, prec, "residual", rel_err(got, ref))
            got = lib.apply(mh, dt, prec, stdg.STDG_RESIDUAL, Us, None)
            ref = d.residual(Us, dt)
            assert rel_err(got, ref) < TOL[prec], (name, prec, "residual-noload", rel_err(got, ref))
            if with_precond:
                note("%s prec=%d precond" % (name, prec))
                got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR_PRECOND, xs)
                ref = d.operator(d.precond_solve(xs), dt)
                assert rel_err(got, ref) < TOL[prec], (name, prec, "precond", rel_err(got, ref))
    finally:
        stdg.stdg_mesh_free(mh)


def test_cavity_4cubed_p2_q1(lib):
    cfg = synth.cavity_small()
    _check_all_modes(lib, cfg["mesh"], cfg["dt"], 0, "cavity4")


def test_operator_on_seed0_vector_cavity_4cubed(lib):
    # the small workload's apply on N(0,1) coefficients, seed 0, full trial vector
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = oracle_disc(m)
    U = synth.random_vector(d.trial_off[-1], 0)
    mh = lib.upload(m)
    got = lib.apply(mh, cfg["dt"], 0, lib.stdg.STDG_RESIDUAL, U)
    lib.stdg.stdg_mesh_free(mh)
    assert rel_err(got, d.residual(U, cfg["dt"])) < 1e-12


@pytest.mark.parametrize("p,q", [(1, 1), (3, 2), (4, 3), (5, 4), (6, 4), (7, 5), (8, 6)])
def test_uniform_degrees_ragged_count(lib, p, q):
    # 3 x 2 x 2 = 12 elements: not a multiple of the 8-way block interleave
    v, h = synth.box_mesh((3, 2, 2), hi=(0.9, 0.5, 0.7))
    ne = h.shape[0]
    rng = np.random.default_rng(p * 10 + q)
    mesh = synth.Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32),
                      rng.uniform(1, 4, ne), rng.uniform(1, 2, ne))
    _check_all_modes(lib, mesh, 0.037, 100 + p, "uniform p%d q%d" % (p, q))


def test_mixed_p_and_q(lib):
    mesh = random_mixed_mesh((3, 3, 2), 5, 4, seed=5)
    _check_all_modes(lib, mesh, 0.05, 6, "mixed")


def test_single_element(lib):
    v, h = synth.box_mesh((1, 1, 1))
    mesh = synth.Mesh(v, h, np.array([3], np.int32), np.array([2], np.int32), np.array([2.0]), np.array([0.5]))
    _check_all_modes(lib, mesh, 0.1, 7, "single")


def test_sheared_affine_nondiagonal_metric(lib):
    v, h = synth.box_mesh((2, 2, 3))
    A = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    v = synth.affine_transform(v, A)
    ne = h.shape[0]
    rng = np.random.default_rng(11)
    mesh = synth.Mesh(v, h, rng.integers(1, 4, ne).astype(np.int32), rng.integers(1, 4, ne).astype(np.int32),
                      rng.uniform(1, 3, ne), rng.uniform(1, 3, ne))
    _check_all_modes(lib, mesh, 0.08, 12, "sheared")


def test_deterministic_bitwise(lib):
    cfg = synth.cavity_two_material(n=6, p=4, q=3)
    m = cfg["mesh"]
    mh = lib.upload(m)
    x = synth.random_vector(m.unknown_size(), 3)
    for prec in (0, 1):
        a = lib.apply(mh, 0.01, prec, lib.stdg.STDG_OPERATOR, x)
        b = lib.apply(mh, 0.01, prec, lib.stdg.STDG_OPERATOR, x)
        assert np.array_equal(a, b)
    lib.stdg.stdg_mesh_free(mh)


@pytest.mark.parametrize("prec", [0, 1])
def test_two_material_32cubed_sampled(lib, prec):
    """Full-size 32^3, p = 4, q = 3 two-material cavity, in the launch
    configuration the benchmark times; the oracle checks sampled elements
    (an element's output depends only on it and its face neighbours)."""
    stdg = lib.stdg
    cfg = synth.cavity_two_material()
    m = cfg["mesh"]
    dt = cfg["dt"]
    note("32^3 prec=%d: generating inputs" % prec)
    x = synth.random_vector(m.unknown_size(), 0)
    if prec == 1:
        x = x.astype(np.float32).astype(np.float64)
    mh = lib.upload(m)
    d = oracle_disc(m)
    n = m.shape[0]
    rng = np.random.default_rng(42)
    sample = [int(e) for e in rng.choice(m.n_elements, 48, replace=False)]
    # corners, both sides of the material interface x = 0.5
    sample += [0, n - 1, n * n - 1, n ** 3 - 1, n // 2 - 1 + n * (n // 2) + n * n * 3, n // 2 + n * 5 + n * n * 7]
    needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
    for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
        note("32^3 prec=%d mode=%d: apply" % (prec, mode))
        y = lib.apply(mh, dt, prec, mode, x)
        assert np.all(np.isfinite(y))
        xin = d.precond_solve(x, needed) if mode == stdg.STDG_OPERATOR_PRECOND else x
        U = d.embed_unknowns(xin)
        rows = d.apply_rows(U, dt, sample)
        got = np.concatenate([y[d.unk_off[e]:d.unk_off[e + 1]] for e in sample])
        ref = np.concatenate([rows[e] for e in sample])
        note("32^3 prec=%d mode=%d rel err %.3e" % (prec, mode, rel_err(got, ref)))
        assert rel_err(got, ref) < TOL[prec]
    stdg.stdg_mesh_free(mh)


def test_binding_checks_device_buffers(lib):
    # the binding refuses vectors of the wrong size, dtype or device before
    # their addresses reach the kernels
    stdg, t = lib.stdg, lib.torch
    cfg = synth.cavity_small()
    mh = lib.upload(cfg["mesh"])
    try:
        info = stdg.stdg_mesh_info(mh)
        nu, nt = info["unknown_size"], info["trial_size"]
        x = t.zeros(nu, dtype=t.float64, device="cuda")
        y = t.zeros(nu, dtype=t.float64, device="cuda")
        bad = [(t.zeros(nu - 1, dtype=t.float64, device="cuda"), y, stdg.STDG_OPERATOR),
               (x, t.zeros(nu, dtype=t.float32, device="cuda"), stdg.STDG_OPERATOR),
               (x.cpu(), y, stdg.STDG_OPERATOR),
               (x, y, stdg.STDG_RESIDUAL)]          # RESIDUAL reads the full trial vector
        for xx, yy, mode in bad:
            with pytest.raises(ValueError):
                stdg.stdg_residual_apply(mh, 0.1, stdg.STDG_FP64, mode, xx, None, yy)
        stdg.stdg_residual_apply(mh, 0.1, stdg.STDG_FP64, stdg.STDG_RESIDUAL,
                                 t.zeros(nt, dtype=t.float64, device="cuda"), None, y)
        with pytest.raises(ValueError):
            stdg.stdg_energy(mh, t.zeros(info["state_size"] - 6, dtype=t.float64, device="cuda"))
    finally:
        stdg.stdg_mesh_free(mh)


def test_work_order_launch_variants_and_autotune(lib, tmp_path):
    # every element order and every launch variant gives bitwise the same
    # apply; the autotuner returns one of its candidate orders and a variant
    # per group, stores them in the cache and reuses them
    stdg = lib.stdg
    cfg = synth.cavity_two_material(n=8, p=3, q=2)
    m = cfg["mesh"]
    mh = lib.upload(m)
    try:
        assert stdg.stdg_mesh_info(mh)["work_order"] == 8
        x = synth.random_vector(m.unknown_size(), 9)
        ref = {}
        for order in (0, 4, 8, 16, 3):
            stdg.stdg_mesh_set_order(mh, order)
            assert stdg.stdg_mesh_info(mh)["work_order"] == order
            for variant in (0, 1, 2):
                stdg.stdg_mesh_set_launch(mh, -1, variant)
                assert stdg.stdg_mesh_group(mh, 0)["variant"] == variant
                for prec in (0, 1):
                    for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
                        y = lib.apply(mh, cfg["dt"], prec, mode, x)
                        ref.setdefault((prec, mode), y)
                        assert np.array_equal(y, ref[(prec, mode)]), (order, variant, prec, mode)
        with pytest.raises(stdg.StdgError):
            stdg.stdg_mesh_set_order(mh, 1)
        with pytest.raises(stdg.StdgError):
            stdg.stdg_mesh_set_launch(mh, -1, 3)
        with pytest.raises(stdg.StdgError):
            stdg.stdg_mesh_set_launch(mh, 1, 0)
        cache = str(tmp_path / "tune.json")
        got = stdg.stdg_mesh_autotune(mh, stdg.STDG_FP32, cfg["dt"], reps=5, cache=cache)
        assert got["order"] in (0, 4, 8, 16) and stdg.stdg_mesh_info(mh)["work_order"] == got["order"]
        assert len(got["variants"]) == 1 and got["variants"][0] in (0, 1, 2)
        assert stdg.stdg_mesh_group(mh, 0)["variant"] == got["variants"][0]
        import json
        table = json.load(open(cache))
        assert list(table.values()) == [got]
        stdg.stdg_mesh_set_order(mh, 0 if got["order"] else 4)
        stdg.stdg_mesh_set_launch(mh, -1, (got["variants"][0] + 1) % 3)
        assert stdg.stdg_mesh_autotune(mh, stdg.STDG_FP32, cfg["dt"], cache=cache) == got
        assert stdg.stdg_mesh_info(mh)["work_order"] == got["order"]
        assert stdg.stdg_mesh_group(mh, 0)["variant"] == got["variants"][0]
        for prec in (0, 1):
            assert np.array_equal(lib.apply(mh, cfg["dt"], prec, stdg.STDG_OPERATOR_PRECOND, x),
                                  ref[(prec, stdg.STDG_OPERATOR_PRECOND)])
    finally:
        stdg.stdg_mesh_free(mh)


def test_launch_variants_mixed_groups_match_oracle(lib):
    # mixed degrees (several groups, staged and gathered neighbour paths,
    # p-truncated faces) in every variant against the oracle
    stdg = lib.stdg
    m = random_mixed_mesh((3, 3, 2), 5, 3, 41)
    d = oracle_disc(m)
    mh = lib.upload(m)
    try:
        n_groups = stdg.stdg_mesh_info(mh)["n_groups"]
        assert n_groups > 4
        assert {stdg.stdg_mesh_group(mh, g)["affine"] for g in range(n_groups)} == {1}
        x = synth.random_vector(m.unknown_size(), 42)
        dt = 0.03
        for prec in (0, 1):
            xin = x.astype(np.float32).astype(np.float64) if prec == 1 else x
            ref = d.operator(xin, dt)
            for variant in (0, 1, 2):
                stdg.stdg_mesh_set_launch(mh, -1, variant)
                got = lib.apply(mh, dt, prec, stdg.STDG_OPERATOR, xin)
                assert rel_err(got, ref) < TOL[prec], (prec, variant)
    finally:
        stdg.stdg_mesh_free(mh)


def test_upload_refuses_invalid_meshes(lib):
    # the library's own checks (STDG_E_ARG), each naming what is wrong; a
    # valid mesh uploads after every refusal
    stdg = lib.stdg
    v, h = synth.box_mesh((2, 1, 1))
    base = dict(v=v, h=h, p=np.full(2, 2, np.int32), q=np.full(2, 1, np.int32), eps=np.ones(2), mu=np.ones(2))

    def upload(**kw):
        a = dict(base)
        a.update(kw)
        return stdg.stdg_mesh_upload(lib.ctx, a["v"], a["h"], a["p"], a["q"], a["eps"], a["mu"])

    inverted = h.copy()
    inverted[1] = inverted[1][[1, 0, 3, 2, 5, 4, 7, 6]]       # mirrored along x-hat: negative Jacobian
    far = h.copy()
    far[1, 0] = v.shape[0]
    cases = [("empty mesh", dict(h=h[:0], p=base["p"][:0], q=base["q"][:0], eps=base["eps"][:0], mu=base["mu"][:0])),
             ("p must", dict(p=np.array([2, 9], np.int32))), ("p must", dict(p=np.array([0, 2], np.int32))),
             ("q must", dict(q=np.array([7, 1], np.int32))), ("q must", dict(q=np.array([1, 0], np.int32))),
             ("eps and mu", dict(eps=np.array([1.0, 0.0]))), ("eps and mu", dict(mu=np.array([1.0, np.nan]))),
             ("vertex id", dict(h=far)), ("inverted", dict(h=inverted))]
    for fragment, kw in cases:
        note("refusal: %s" % fragment)
        with pytest.raises(stdg.StdgError) as ei:
            upload(**kw)
        assert ei.value.status == -1 and fragment in str(ei.value), (fragment, str(ei.value))
    mh = upload()
    assert stdg.stdg_mesh_info(mh)["n_elements"] == 2
    stdg.stdg_mesh_free(mh)


@pytest.fixture(scope="module")
def large_cavity():
    cfg = synth.large_cavity()
    note("48^3: oracle set-up")
    return cfg, oracle_disc(cfg["mesh"])


@pytest.mark.parametrize("prec", [0, 1])
def test_large_cavity_48cubed_sampled(lib, large_cavity, prec):
    """Full-size 48^3, p = 6, q = 4 cavity with eps drawn per element (1.1e9
    trial DoF), in the launch configuration the benchmark times.  The input is
    seeded N(0,1) on the sampled elements and their face neighbours and zero
    elsewhere, so a read of any other element's block shows up as a mismatch;
    the oracle evaluates the sampled elements' rows."""
    stdg, t = lib.stdg, lib.torch
    cfg, d = large_cavity
    m, dt = cfg["mesh"], cfg["dt"]
    rng = np.random.default_rng(4800 + prec)
    n = 48
    sample = [int(e) for e in rng.choice(m.n_elements, 12, replace=False)]
    sample += [0, n - 1, n * n - 1, n ** 3 - 1, n // 2 + n * (n // 2) + n * n * (n // 2)]
    needed = sorted(set(sample) | {int(k) for e in sample for k in d.nb[e] if k >= 0})
    x = np.zeros(d.unk_off[-1])
    for e in needed:
        blk = rng.standard_normal(d.unk_off[e + 1] - d.unk_off[e])
        x[d.unk_off[e]:d.unk_off[e + 1]] = blk.astype(np.float32) if prec == 1 else blk
    dtype = t.float64 if prec == 0 else t.float32
    mh = lib.upload(m)
    try:
        nu = stdg.stdg_mesh_info(mh)["unknown_size"]
        assert nu == d.unk_off[-1]
        xd = t.zeros(nu, dtype=dtype, device="cuda")
        for e in needed:
            xd[d.unk_off[e]:d.unk_off[e + 1]] = t.from_numpy(x[d.unk_off[e]:d.unk_off[e + 1]]).to(dtype)
        for mode in (stdg.STDG_OPERATOR, stdg.STDG_OPERATOR_PRECOND):
            note("48^3 prec=%d mode=%d: apply" % (prec, mode))
            yd = t.full((nu,), float("nan"), dtype=dtype, device="cuda")
            stdg.stdg_residual_apply(mh, dt, prec, mode, xd, None, yd)
            t.cuda.synchronize()
            got = np.concatenate([yd[d.unk_off[e]:d.unk_off[e + 1]].double().cpu().numpy() for e in sample])
            xin = d.precond_solve(x, needed) if mode == stdg.STDG_OPERATOR_PRECOND else x
            rows = d.apply_rows(d.embed_unknowns(xin, elements=needed), dt, sample)
            ref = np.concatenate([rows[e] for e in sample])
            note("48^3 prec=%d mode=%d rel err %.3e" % (prec, mode, rel_err(got, ref)))
            assert rel_err(got, ref) < TOL[prec]
        del xd, yd
    finally:
        stdg.stdg_mesh_free(mh)
