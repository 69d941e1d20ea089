"""The library's streaming copy (measurement utility: the practical HBM
ceiling the memory-bound kernels are compared with): exact copies at sizes
with a ragged tail, and its argument refusals."""
import pytest

from tests.gpu_util import Lib, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return Lib()


@pytest.mark.parametrize("n16", [1, 255, 256 * 2 + 1, 256 * 256 * 32 * 2 + 17, (64 << 20) // 16 + 3])
def test_stream_copy_exact(lib, n16):
    torch = lib.torch
    note("stream copy of %d 16-byte chunks" % n16)
    g = torch.Generator(device="cuda").manual_seed(n16)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (4 * n16,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    lib.stdg.stdg_stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_copy_refusals(lib):
    torch, stdg = lib.torch, lib.stdg
    buf = torch.zeros(1024, dtype=torch.int32, device="cuda")
    base = buf.data_ptr()
    raw = stdg.lib().stdg_stream_copy
    import ctypes
    E_ARG = -1
    # misaligned pointer, ragged size, overlap, NULL; nothing is launched
    assert raw(ctypes.c_void_p(base + 4), ctypes.c_void_p(base + 2048), ctypes.c_size_t(64), None) == E_ARG
    assert raw(ctypes.c_void_p(base), ctypes.c_void_p(base + 2048), ctypes.c_size_t(40), None) == E_ARG
    assert raw(ctypes.c_void_p(base), ctypes.c_void_p(base + 1024), ctypes.c_size_t(2048), None) == E_ARG
    assert raw(None, ctypes.c_void_p(base), ctypes.c_size_t(64), None) == E_ARG
    assert raw(None, None, ctypes.c_size_t(0), None) == 0
    with pytest.raises(ValueError):
        stdg.stdg_stream_copy(buf, torch.zeros(1023, dtype=torch.int32, device="cuda"))
