"""The C-ABI library loads and exports every entry point include/stdg.h declares
(no compute calls: runs without a GPU), and fails cleanly without a device."""
import ctypes

import pytest

import paper_1307_5310_amd as stdg


def test_library_exports_every_declared_symbol():
    L = stdg.lib()
    names = stdg.exported_symbols()
    assert "stdg_residual_apply" in names and "stdg_slab_solve" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_error_string():
    assert stdg.stdg_version() >> 16 >= 1
    assert isinstance(stdg.lib().stdg_last_error(), bytes)


def test_init_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(stdg.StdgError) as ei:
        stdg.stdg_init(0, 0)
    assert ei.value.status == -4


def test_null_arguments_rejected():
    L = stdg.lib()
    assert L.stdg_residual_apply(None, 0.1, 0, 0, None, None, None, None) == -1
    assert L.stdg_mesh_info(None, None) == -1
    assert L.stdg_finalize(None) == -1
    assert b"NULL" in L.stdg_last_error()


def test_mesh_arrays_checked_before_the_library_reads_them():
    # the library reads n_elements entries of each per-element array: the
    # binding refuses arrays of other shapes before passing their addresses
    import numpy as np
    import synth
    v, h = synth.box_mesh((2, 1, 1))
    ok = [v, h, np.full(2, 2), np.full(2, 1), np.ones(2), np.ones(2)]
    d, _keep = stdg._mesh_desc(*ok)
    assert d.n_elements == 2 and d.n_vertices == v.shape[0]
    bad = [(0, v[:, :2]), (0, v.ravel()), (1, h[:, :6]), (1, h.ravel()),
           (2, np.full(1, 2)), (3, np.full(3, 1)), (4, np.ones((2, 1))), (5, np.ones(1))]
    for k, arr in bad:
        args = list(ok)
        args[k] = arr
        with pytest.raises(ValueError):
            stdg._mesh_desc(*args)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback path: without the built library every entry point raises
    from paper_1307_5310_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libstdg.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError, match="no fallback"):
        _lib.lib()
    with pytest.raises(ImportError):
        stdg.stdg_version()


def test_tune_cache_read_and_write(tmp_path):
    # a missing or damaged cache reads as empty; writes replace the file whole
    path = str(tmp_path / "tune.json")
    assert stdg._tune_cache_read(path) == {}
    a = {"order": 8, "variants": [0, 2]}
    stdg._tune_cache_write(path, {"a": a})
    assert stdg._tune_cache_read(path) == {"a": a}
    for junk in ("{not json", "[1, 2]", '{"a": "x"}', '{"a": 8}', '{"a": {"order": 8}}',
                 '{"a": {"order": 8, "variants": ["x"]}}'):
        with open(path, "w") as f:
            f.write(junk)
        assert stdg._tune_cache_read(path) == {}
    b = {"order": 0, "variants": [1]}
    stdg._tune_cache_write(path, {"a": a, "b": b})
    assert stdg._tune_cache_read(path) == {"a": a, "b": b}
    assert sorted(p.name for p in tmp_path.iterdir()) == ["tune.json"]


def test_struct_layouts_match_the_library():
    from paper_1307_5310_amd import _lib
    L = stdg.lib()
    for which, st in enumerate(_lib.STRUCTS):
        assert L.stdg_struct_size(which) == ctypes.sizeof(st), st.__name__
    assert L.stdg_struct_size(99) == 0


def test_serving_buffers_checked_before_the_library_reads_them():
    # poll copies the final state into state_out: only a writeable C-contiguous
    # float64 array is accepted; submit reads init_state's declared length,
    # which must be the mesh's state size (both refused before any call)
    import numpy as np
    import synth
    for bad in (np.zeros(10, dtype=np.float32), np.zeros((10, 2))[:, 0], [0.0] * 10):
        with pytest.raises(ValueError):
            stdg.stdg_serve_poll(None, 1, state_out=bad)
    v, h = synth.box_mesh((2, 1, 1))
    n_state = 2 * 6 * 3 ** 3
    for size in (n_state - 1, n_state + 5):
        with pytest.raises(ValueError):
            stdg.stdg_serve_submit(None, v, h, np.full(2, 2), np.full(2, 1), np.ones(2), np.ones(2), 0.0, 0.1, 1,
                                   init_state=np.zeros(size))
