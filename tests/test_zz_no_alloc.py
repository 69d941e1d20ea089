"""The allocation-free apply (stdg_residual_apply_noalloc) against
stdg_residual_apply on the same inputs, through the C ABI: two calls in a row
on meshes that need the static scratch (sheared, so P^{-1} is a pre-pass),
the second smaller than the first, in both precisions and all modes; a mesh
with several kernel groups; the size limit."""
import numpy as np
import pytest

import synth
from tests.gpu_util import Lib, note

pytestmark = pytest.mark.gpu

SHEAR = np.array([[1.0, 0.2, 0.0], [0.0, 1.0, 0.1], [0.1, 0.0, 1.0]])


@pytest.fixture(scope="module")
def lib():
    return Lib()


def _sheared(shape, p, q, seed):
    v, h = synth.box_mesh(shape)
    v = synth.affine_transform(v, SHEAR)
    ne = h.shape[0]
    rng = np.random.default_rng(seed)
    return synth.Mesh(v, h, np.full(ne, p, np.int32), np.full(ne, q, np.int32), rng.uniform(1, 4, ne),
                      rng.uniform(1, 2, ne), shape=tuple(shape))


def _both(lib, mh, m, prec, mode, seed, dt=0.03):
    t = lib.torch
    stdg = lib.stdg
    dtype = t.float64 if prec == stdg.STDG_FP64 else t.float32
    n_in = m.trial_size() if mode == stdg.STDG_RESIDUAL else m.unknown_size()
    x = lib.dev(synth.random_vector(n_in, seed), dtype)
    load = lib.dev(synth.random_vector(m.unknown_size(), seed + 1), dtype) if mode == stdg.STDG_RESIDUAL else None
    y_ref = t.full((m.unknown_size(),), float("nan"), dtype=dtype, device="cuda")
    y_na = t.full((m.unknown_size(),), float("nan"), dtype=dtype, device="cuda")
    stdg.stdg_residual_apply(mh, dt, prec, mode, x, load, y_ref)
    stdg.stdg_residual_apply_noalloc(mh, dt, prec, mode, x, load, y_na)
    t.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_apply_two_calls_second_smaller(lib, prec):
    stdg = lib.stdg
    big = _sheared((4, 4, 3), 3, 2, 1)
    small = _sheared((2, 2, 1), 2, 1, 2)
    assert small.unknown_size() < big.unknown_size()
    for mode in (stdg.STDG_OPERATOR_PRECOND, stdg.STDG_OPERATOR, stdg.STDG_RESIDUAL):
        for k, m in enumerate((big, small)):
            note("noalloc prec=%d mode=%d call %d (%d unknowns)" % (prec, mode, k, m.unknown_size()))
            mh = lib.upload(m)
            try:
                ref, got = _both(lib, mh, m, prec, mode, 10 + k)
            finally:
                stdg.stdg_mesh_free(mh)
            assert np.all(np.isfinite(ref))
            assert np.array_equal(ref, got)


def test_noalloc_several_groups_and_trilinear(lib):
    # mixed degrees on a perturbed mesh: several kernel groups run one after
    # another on the caller's stream; the trilinear elements need the pre-pass
    stdg = lib.stdg
    v, h = synth.box_mesh((3, 2, 2))
    v = synth.perturb_interior(v, (3, 2, 2), 0.15, 3)
    ne = h.shape[0]
    rng = np.random.default_rng(4)
    m = synth.Mesh(v, h, rng.integers(1, 4, ne).astype(np.int32), rng.integers(1, 3, ne).astype(np.int32),
                   rng.uniform(1, 3, ne), np.ones(ne), shape=(3, 2, 2))
    mh = lib.upload(m)
    try:
        assert stdg.stdg_mesh_info(mh)["n_groups"] > 1
        for prec in (0, 1):
            note("noalloc trilinear mixed prec=%d" % prec)
            ref, got = _both(lib, mh, m, prec, stdg.STDG_OPERATOR_PRECOND, 20 + prec)
            assert np.all(np.isfinite(ref))
            assert np.array_equal(ref, got)
    finally:
        stdg.stdg_mesh_free(mh)


def test_noalloc_refuses_inputs_beyond_the_scratch(lib):
    stdg = lib.stdg
    cap = stdg.stdg_noalloc_scratch_bytes()
    assert cap == 64 << 20
    m = _sheared((14, 14, 14), 4, 3, 5)          # 6.2 M unknowns: 49 MB in FP64
    m2 = _sheared((16, 16, 16), 4, 3, 6)         # 9.2 M unknowns: 74 MB in FP64, 37 MB in FP32
    assert m.unknown_size() * 8 <= cap < m2.unknown_size() * 8
    mh = lib.upload(m2)
    try:
        x = lib.torch.zeros(m2.unknown_size(), dtype=lib.torch.float64, device="cuda")
        y = lib.torch.empty_like(x)
        with pytest.raises(stdg.StdgError) as ei:
            stdg.stdg_residual_apply_noalloc(mh, 0.01, stdg.STDG_FP64, stdg.STDG_OPERATOR_PRECOND, x, None, y)
        assert ei.value.status == -7 and "scratch" in str(ei.value)
        # FP32 fits; and plain operator applies need no scratch at all
        ref, got = _both(lib, mh, m2, stdg.STDG_FP32, stdg.STDG_OPERATOR_PRECOND, 30)
        assert np.array_equal(ref, got)
        ref, got = _both(lib, mh, m2, stdg.STDG_FP64, stdg.STDG_OPERATOR, 31)
        assert np.array_equal(ref, got)
    finally:
        stdg.stdg_mesh_free(mh)
    mh = lib.upload(m)
    try:
        note("noalloc near the limit")
        ref, got = _both(lib, mh, m, stdg.STDG_FP64, stdg.STDG_OPERATOR_PRECOND, 32)
        assert np.array_equal(ref, got)
    finally:
        stdg.stdg_mesh_free(mh)
