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
