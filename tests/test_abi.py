"""The C-ABI library loads and exports every symbol include/tc.h declares; host-side
argument checks (no GPU needed, no kernels launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")
LIB = os.path.join(ROOT, "paper_2403_02997_amd", "libtc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tc_count", "tc_count_batch", "tc_count_ex", "tc_count_per_vertex",
                     "tc_validate_csr", "tc_count_batch_workspace_size"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    import paper_2403_02997_amd.tc as b
    assert sorted(b.EXPORTS) == declared_functions()


def test_status_strings_and_version(lib):
    lib.tc_status_string.restype = ctypes.c_char_p
    for code in range(0, -7, -1):
        s = lib.tc_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.tc_status_string(-99).decode() == "unknown status"
    # the limits named in the message are the ones check_args applies
    assert "2^30" in lib.tc_status_string(-5).decode()
    assert "2^32 - 2^20" in lib.tc_status_string(-5).decode()
    assert lib.tc_version() >= 10000


def test_argument_errors_without_gpu(lib):
    u64 = ctypes.c_uint64
    lib.tc_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_void_p, ctypes.POINTER(u64)]
    out = u64(7)
    # null count pointer
    assert lib.tc_count(None, None, 0, 0, None, None) == -1
    # n >= 2^30 and m >= 2^32 are refused before any device work
    assert lib.tc_count(None, None, 0x80000000, 0, None, ctypes.byref(out)) == -5
    assert lib.tc_count(None, None, 0x40000000, 0, None, ctypes.byref(out)) == -5
    assert lib.tc_count(None, None, 10, 1 << 32, None, ctypes.byref(out)) == -5
    # entry offsets keep 2^20 of headroom below 2^32 for the tile arithmetic
    assert lib.tc_count(None, None, 10, (1 << 32) - (1 << 20) + 1, None, ctypes.byref(out)) == -5
    # data required when m > 0
    assert lib.tc_count(None, None, 10, 4, None, ctypes.byref(out)) == -1
    assert out.value == 7  # untouched on error
    # batch: null inputs with graphs
    lib.tc_count_batch.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_uint64,
                                                          ctypes.c_uint64, ctypes.c_void_p,
                                                          ctypes.c_size_t, ctypes.c_void_p,
                                                          ctypes.c_void_p]
    assert lib.tc_count_batch(None, None, None, None, 3, 10, 20, None, 0, None, None) == -1
    assert lib.tc_count_batch(None, None, None, None, 0, 0, 0, None, 0, None, None) == 0
    # totals above 2^32 - 2^20 are refused before the workspace or any launch
    dummy = (ctypes.c_uint64 * 4)()
    p = ctypes.cast(dummy, ctypes.c_void_p)
    assert lib.tc_count_batch(p, p, p, p, 1, 2, (1 << 32) - (1 << 20) + 1, None, 0, None,
                              p) == -5
    # the allocation-free batch: the same argument checks, and a batch whose workspace
    # exceeds the fixed scratch array is refused before any device call
    lib.tc_count_batch_noalloc.argtypes = [ctypes.c_void_p] * 4 + [
        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.tc_count_batch_noalloc(None, None, None, None, 3, 10, 20, None, None) == -1
    assert lib.tc_count_batch_noalloc(None, None, None, None, 0, 0, 0, None, None) == 0
    assert lib.tc_count_batch_noalloc(p, p, p, p, 1, 2, (1 << 32) - (1 << 20) + 1, None, p) == -5
    lib.tc_count_batch_workspace_size.argtypes = [ctypes.c_uint32, ctypes.c_uint64,
                                                  ctypes.c_uint64]
    lib.tc_count_batch_workspace_size.restype = ctypes.c_size_t
    cap = 64 << 20
    rows = 1 << 20
    cols = (cap - lib.tc_count_batch_workspace_size(4, rows, 0)) // 8 + 64
    assert lib.tc_count_batch_workspace_size(4, rows, cols) > cap
    assert lib.tc_count_batch_noalloc(p, p, p, p, 4, rows, cols, None, p) == -5
    # CETC-Seq-FE's threshold: 2.0 (off) by default, negative and NaN refused
    lib.tc_get_forward_threshold.restype = ctypes.c_double
    lib.tc_set_forward_threshold.argtypes = [ctypes.c_double]
    assert lib.tc_get_forward_threshold() == 2.0
    assert lib.tc_set_forward_threshold(-0.5) == -1
    assert lib.tc_set_forward_threshold(float("nan")) == -1
    assert lib.tc_get_forward_threshold() == 2.0
    assert lib.tc_set_forward_threshold(0.7) == 0 and lib.tc_get_forward_threshold() == 0.7
    assert lib.tc_set_forward_threshold(2.0) == 0
    # clustering coefficients: checked before the launch
    lib.tc_local_clustering.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p]
    assert lib.tc_local_clustering(None, None, 0, None, None) == 0
    assert lib.tc_local_clustering(None, None, 5, None, None) == -1
    assert lib.tc_local_clustering(None, None, 0x40000000, None, None) == -5


def test_workspace_size_grows_with_rows(lib):
    lib.tc_count_batch_workspace_size.argtypes = [ctypes.c_uint32, ctypes.c_uint64,
                                                  ctypes.c_uint64]
    lib.tc_count_batch_workspace_size.restype = ctypes.c_size_t
    a = lib.tc_count_batch_workspace_size(10, 1000, 5000)
    b = lib.tc_count_batch_workspace_size(10, 100000, 5000)
    c = lib.tc_count_batch_workspace_size(10, 100000, 500000)
    assert c > b > a >= 21 * 1000 + 8 * 5000


def test_isect_params_validation(lib):
    arr = (ctypes.c_uint32 * 4)()
    assert lib.tc_get_isect_params(arr) == 0
    saved = tuple(arr)
    assert lib.tc_set_isect_params(16, 4096, 4096, 256) == -1  # wavefront tables hold 512
    assert lib.tc_set_isect_params(16, 512, 32768, 256) == -1  # workgroup table holds 16384
    assert lib.tc_set_isect_params(16, 512, 4096, 2048) == -1  # one partner per thread
    assert lib.tc_set_isect_params(16, 512, 0, 256) == -1
    assert lib.tc_set_isect_params(600, 512, 4096, 256) == -1  # lane class inside wave class
    assert lib.tc_set_isect_params(8, 256, 2048, 128) == 0
    assert lib.tc_get_isect_params(arr) == 0 and tuple(arr) == (8, 256, 2048, 128)
    assert lib.tc_set_isect_params(*saved) == 0


def test_serve_argument_errors_without_gpu(lib):
    vp = ctypes.c_void_p
    lib.tc_serve_submit.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.c_uint64, vp]
    lib.tc_serve_poll.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_int32]
    lib.tc_serve_get_stats.argtypes = [vp, vp]
    lib.tc_serve_destroy.argtypes = [vp]
    lib.tc_serve_create.argtypes = [vp, vp]
    t = ctypes.c_uint64(0)
    assert lib.tc_serve_create(None, None) == -1
    assert lib.tc_serve_submit(None, None, None, 0, 0, ctypes.byref(t)) == -1
    assert lib.tc_serve_poll(None, None, 0, None, 0) == -1
    assert lib.tc_serve_get_stats(None, None) == -1
    assert lib.tc_serve_destroy(None) == -1
