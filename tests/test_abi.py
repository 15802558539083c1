"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its pure-host calls (sizes, error strings, argument
validation that fails before any device work) behave as documented."""
import ctypes

import pytest

from paper_2106_03452_amd import _lib


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_header_symbol_is_exported(L):
    names = _lib.header_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_and_version(L):
    assert L.psr_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.psr_strerror(code)
    assert b"unknown" in L.psr_strerror(12345)


def test_stage_names(L):
    n = L.psr_num_stages()
    names = [L.psr_stage_name(i).decode() for i in range(n)]
    assert len(set(names)) == n and "P3_fft_j0_spectral_ifft_j0" in names
    assert L.psr_stage_name(n) == b"unknown"


@pytest.mark.parametrize("res", [8, 16, 32, 64, 128, 256, 512])
def test_workspace_sizes(res):
    P = 12345
    ws = _lib.workspace_bytes(res, P)
    H = res // 2 + 1
    assert ws >= 2 * 3 * H * res * res * 8 + P * 32
    assert ws % 256 == 0
    sv = _lib.saved_bytes(res, P)
    assert sv >= P * 48 + 256


@pytest.mark.parametrize("res,P", [(0, 10), (7, 10), (1024, 10), (4, 10), (96, 10), (64, 0), (64, -5)])
def test_size_queries_reject_bad_arguments(L, res, P):
    out = ctypes.c_size_t(0)
    assert L.psr_workspace_bytes(res, P, 1, ctypes.byref(out)) == _lib.PSR_EINVAL
    assert L.psr_saved_bytes(res, P, ctypes.byref(out)) == _lib.PSR_EINVAL


@pytest.mark.parametrize("res,slabs", [(16, 1), (16, 16), (64, 64), (256, 8), (1024, 8), (1024, 64)])
def test_slab_workspace_sizes(L, res, slabs):
    P = 1000
    out = ctypes.c_size_t(0)
    assert L.psr_slab_workspace_bytes(res, P, slabs, ctypes.byref(out)) == _lib.PSR_OK
    hp = res // 2 + 1
    # three splat channels, two exchange channels, one returned channel
    assert out.value >= (3 + 2 + 1) * res * res * hp * 8 + P * 80
    assert out.value % 256 == 0
    zero = ctypes.c_size_t(0)
    assert L.psr_slab_workspace_bytes(res, 0, slabs, ctypes.byref(zero)) == _lib.PSR_OK
    assert zero.value < out.value


@pytest.mark.parametrize("res,slabs,P", [(8, 1, 10), (2048, 8, 10), (96, 2, 10), (64, 3, 10), (64, 128, 10),
                                         (32, 64, 10), (64, 0, 10), (64, 4, -1)])
def test_slab_size_query_rejects_bad_arguments(L, res, slabs, P):
    out = ctypes.c_size_t(0)
    assert L.psr_slab_workspace_bytes(res, P, slabs, ctypes.byref(out)) == _lib.PSR_EINVAL


def test_null_arguments_rejected_without_device_work(L):
    # every check below fails before any HIP call is made
    assert L.psr_forward(None, None, None, 10, 64, 2.0, None, None, None, 0, None) == _lib.PSR_EINVAL
    assert L.psr_backward(None, 10, 64, 2.0, None, None, None, None, None, None, 0, None) == _lib.PSR_EINVAL
    assert L.psr_ctx_create(None, 0) == _lib.PSR_EINVAL
    assert L.psr_ctx_destroy(None) == _lib.PSR_EINVAL
    assert L.psr_ctx_set(None, b"m", 0.5) == _lib.PSR_EINVAL
    assert L.psr_run_batched(None, 1, None, None) == _lib.PSR_EINVAL
    assert L.psr_debug_spectral(None, None, 64, 2.0, None, None, 0, None) == _lib.PSR_EINVAL
    assert L.psr_saved_status(None, None, None) == _lib.PSR_EINVAL
    assert L.psr_slab_forward(None, None, None, 10, 64, 2.0, 4, None, None, None, 0, None) == _lib.PSR_EINVAL
    assert L.psr_slab_debug_spectral(None, None, 64, 2.0, 4, None, None, 0, None) == _lib.PSR_EINVAL


def test_opt_step_size_query_and_argument_checks(L):
    out = ctypes.c_size_t(0)
    assert L.psr_opt_step_workspace_bytes(32, 20000, 20000, 20000, 8192, 16384, ctypes.byref(out)) == _lib.PSR_OK
    small = out.value
    assert small > 0 and small % 256 == 0
    assert L.psr_opt_step_workspace_bytes(64, 20000, 20000, 20000, 8192, 16384, ctypes.byref(out)) == _lib.PSR_OK
    assert out.value > small  # the grids grow with res
    for args in ((33, 10, 10, 10, 10, 10), (32, 0, 10, 10, 10, 10), (32, 10, 0, 10, 10, 10),
                 (32, 10, 10, 0, 10, 10), (32, 10, 10, 10, 0, 10), (32, 10, 10, 10, 10, 0),
                 (32, 10, 1 << 31, 10, 10, 10)):
        assert L.psr_opt_step_workspace_bytes(*args, ctypes.byref(out)) == _lib.PSR_EINVAL
    assert L.psr_opt_step_workspace_bytes(32, 10, 10, 10, 10, 10, None) == _lib.PSR_EINVAL
    # argument checks fail before any device work
    assert L.psr_opt_step(None, None, None, 10, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None, 10, None,
                          10, 32, 2.0, 100, 100, None, None, None, 0, None) == _lib.PSR_EINVAL


def test_mc_case_table_matches_the_oracle(L):
    """The library builds its Marching Cubes table at compile time from the
    same face rule the oracle implements in Python: both must agree entry by
    entry (host only, no GPU)."""
    import ctypes
    from oracle import mc
    ntri = (ctypes.c_int8 * 256)()
    edges = (ctypes.c_int8 * (256 * 15))()
    L.psr_mc_case_table.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert L.psr_mc_case_table(ctypes.cast(ntri, ctypes.c_void_p), ctypes.cast(edges, ctypes.c_void_p)) == 0
    table = mc.case_table()
    for c in range(256):
        got = [tuple(edges[c * 15 + 3 * i: c * 15 + 3 * i + 3]) for i in range(ntri[c])]
        assert got == [tuple(t) for t in table[c]], c
