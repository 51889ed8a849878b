"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device. CPU only:
none of the calls below reaches a kernel launch."""
import ctypes
import os
import re

import pytest

from paper_1012_2273_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gemm_mi355x.h")
TUNING_HEADER = os.path.join(ROOT, "include", "gemm_mi355x_tuning.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def _declared(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gemm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("gemm_plain", "gemm_split", "gemm_grouped", "gemm_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    tuning = _declared(TUNING_HEADER)
    assert set(tuning) == set(_lib.TUNING_EXPORTS)
    for n in names + tuning:
        assert hasattr(lib, n), n


def test_every_header_is_covered():
    """Each header under include/ is one of the two whose symbols are checked."""
    hs = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert hs == ["gemm_mi355x.h", "gemm_mi355x_tuning.h"]


def test_tuning_knobs_are_per_thread(lib):
    """A forced shape or chunk count on one thread leaves another thread's
    choice alone (the workspace query reads the calling thread's setting)."""
    import threading
    F64 = _lib.GEMM_F64
    size = lib.gemm_plain_ksplit_workspace_size
    auto = size(F64, 64, 64, 1000)
    seen = {}
    assert lib.gemm_tuning_force_ksplit_parts(3) == _lib.GEMM_OK
    try:
        assert size(F64, 64, 64, 1000) == 2 * 64 * 64 * 8
        t = threading.Thread(target=lambda: seen.update(other=size(F64, 64, 64, 1000)))
        t.start()
        t.join()
    finally:
        assert lib.gemm_tuning_force_ksplit_parts(-1) == _lib.GEMM_OK
    assert seen["other"] == auto
    assert size(F64, 64, 64, 1000) == auto


def test_strerror_texts(lib):
    for code in range(9):
        assert lib.gemm_strerror(code)
    assert lib.gemm_strerror(99) == b"unknown status"


def test_tile_config_names(lib):
    n = lib.gemm_tile_config_count()
    names = [lib.gemm_tile_config_name(i).decode() for i in range(n)]
    assert names[0] == "128x128" and len(set(names)) == n
    assert lib.gemm_tile_config_name(n) == b""
    assert lib.gemm_tuning_force_tile_config(n) == _lib.GEMM_EINVAL
    assert lib.gemm_tuning_force_tile_config(-2) == _lib.GEMM_EINVAL
    assert lib.gemm_tuning_force_tile_config(-1) == _lib.GEMM_OK


def _plain(lib, dtype=0, m=4, n=4, k=4, A=16, lda=4, B=16, ldb=4, C=16, ldc=4):
    v = lambda x: ctypes.c_void_p(x) if x else None
    return lib.gemm_plain(dtype, m, n, k, v(A), lda, v(B), ldb, v(C), ldc, None)


def test_plain_validation(lib):
    assert _plain(lib, dtype=7) == _lib.GEMM_EUNSUPPORTED
    assert _plain(lib, m=-1) == _lib.GEMM_EINVAL
    assert _plain(lib, k=-3) == _lib.GEMM_EINVAL
    assert _plain(lib, A=0) == _lib.GEMM_ENULL
    assert _plain(lib, C=0) == _lib.GEMM_ENULL
    assert _plain(lib, lda=3) == _lib.GEMM_ELD
    assert _plain(lib, ldb=2) == _lib.GEMM_ELD
    assert _plain(lib, ldc=1) == _lib.GEMM_ELD
    assert b"leading dimension" in lib.gemm_last_error()
    # empty output: no work, no device call
    assert _plain(lib, m=0, A=0, C=0) == _lib.GEMM_OK
    assert _plain(lib, n=0, B=0, C=0, ldb=0, ldc=0) == _lib.GEMM_OK


def test_split_one_launch_query_without_device(lib):
    """Empty, null or misaligned operands report the two-step form (0)
    before the library looks at the device."""
    v = ctypes.c_void_p
    assert lib.gemm_split_one_launch(0, 8, 8, v(256), 8, v(256), 8) == 0
    assert lib.gemm_split_one_launch(8, 8, 8, None, 8, v(256), 8) == 0
    assert lib.gemm_split_one_launch(8, 8, 8, v(256), 8, None, 8) == 0
    assert lib.gemm_split_one_launch(8, 8, 8, v(260), 8, v(256), 8) == 0   # base not 16-byte aligned
    assert lib.gemm_split_one_launch(8, 8, 8, v(256), 9, v(256), 8) == 0   # row pitch 36 bytes
    assert lib.gemm_split_one_launch(8, 8, 6, v(256), 8, v(256), 8) == 0   # k not a multiple of 4
    assert lib.gemm_split_one_launch(8, 8, 2048, v(256), 2048, v(256), 8) == 0   # long K loop


def test_split_workspace_size(lib):
    assert lib.gemm_split_workspace_size(-1, 2, 2) == 0
    s = lib.gemm_split_workspace_size(2000, 2000, 2000)
    assert s >= 2 * 2 * 2000 * 2000 * 2 and s % 256 == 0
    # plane rows padded to a 64-element (128-byte) pitch, planes to 256 bytes
    assert lib.gemm_split_workspace_size(1, 1, 1) == 4 * 256
    assert lib.gemm_split_workspace_size(3, 5, 65) == 2 * 768 + 2 * 1280
    assert lib.gemm_split_workspace_size(2000, 2000, 2000) == 4 * 2000 * 2048 * 2


def test_row_pitch_limit(lib):
    """Tile offsets are 32-bit: row pitches of 8 MiB or more are rejected
    before any launch (a 256-row tile must span less than 2^31 bytes)."""
    v = ctypes.c_void_p
    assert _plain(lib, 0, 4, 4, 4, lda=1 << 20) == _lib.GEMM_EINVAL          # 8 MiB binary64 rows
    assert _plain(lib, 1, 4, 4, 4, ldb=1 << 21) == _lib.GEMM_EINVAL          # 8 MiB binary32 rows
    k = 1 << 22                                                              # split planes: 8 MiB rows
    assert lib.gemm_split(4, 4, k, v(16), k, v(16), 4, v(16), 4, v(256), 1 << 40, None) == _lib.GEMM_EINVAL
    assert lib.gemm_split3(4, 4, k, v(16), k, v(16), 4, v(16), 4, v(256), 1 << 40, None) == _lib.GEMM_EINVAL


def test_split3_workspace_and_validation(lib):
    v = ctypes.c_void_p
    assert lib.gemm_split3_workspace_size(-1, 2, 2) == 0
    # six planes, rows padded to a 64-element pitch, planes to 256 bytes
    assert lib.gemm_split3_workspace_size(1, 1, 1) == 6 * 256
    assert lib.gemm_split3_workspace_size(3, 5, 65) == 3 * 768 + 3 * 1280
    ws = lib.gemm_split3_workspace_size(8, 8, 8)
    assert lib.gemm_split3(8, 8, 8, v(16), 8, v(16), 8, v(16), 8, None, ws, None) == _lib.GEMM_EWORKSPACE
    assert lib.gemm_split3(8, 8, 8, v(16), 8, v(16), 8, v(16), 8, v(256), ws - 1, None) == _lib.GEMM_EWORKSPACE
    assert lib.gemm_split3(8, 8, 8, v(16), 7, v(16), 8, v(16), 8, v(256), ws, None) == _lib.GEMM_ELD
    assert lib.gemm_split3(8, 8, -1, v(16), 8, v(16), 8, v(16), 8, v(256), ws, None) == _lib.GEMM_EINVAL
    assert lib.gemm_split3(8, 8, 8, None, 8, v(16), 8, v(16), 8, v(256), ws, None) == _lib.GEMM_ENULL
    assert lib.gemm_split3_convert(4, 4, v(16), 4, 2, v(16), v(16), v(16), 4, None) == _lib.GEMM_EINVAL
    assert lib.gemm_split3_convert(4, 5, v(16), 5, 1, v(16), v(16), v(16), 3, None) == _lib.GEMM_ELD
    assert lib.gemm_split3_convert(4, 5, v(16), 5, 0, v(16), None, v(16), 5, None) == _lib.GEMM_ENULL


def test_split_validation(lib):
    v = ctypes.c_void_p
    ws = lib.gemm_split_workspace_size(8, 8, 8)
    assert lib.gemm_split(8, 8, 8, v(16), 8, v(16), 8, v(16), 8, None, ws, None) == _lib.GEMM_EWORKSPACE
    assert lib.gemm_split(8, 8, 8, v(16), 8, v(16), 8, v(16), 8, v(256), ws - 1, None) == _lib.GEMM_EWORKSPACE
    assert lib.gemm_split(8, 8, 8, v(16), 8, v(16), 8, v(16), 8, v(8), ws, None) == _lib.GEMM_EWORKSPACE
    assert lib.gemm_split(8, 8, 8, v(16), 7, v(16), 8, v(16), 8, v(256), ws, None) == _lib.GEMM_ELD
    assert lib.gemm_split(8, -8, 8, v(16), 8, v(16), 8, v(16), 8, v(256), ws, None) == _lib.GEMM_EINVAL
    assert lib.gemm_split_convert(4, 4, v(16), 4, 2, v(16), v(16), 4, None) == _lib.GEMM_EINVAL
    assert lib.gemm_split_convert(4, 5, v(16), 5, 1, v(16), v(16), 3, None) == _lib.GEMM_ELD
    assert lib.gemm_split_convert(4, 5, v(16), 5, 0, None, v(16), 5, None) == _lib.GEMM_ENULL


def test_ksplit_workspace_and_validation(lib):
    """Workspace query (the device's CU count falls back to 256 without a
    device) and argument checks of the K-split product."""
    v = ctypes.c_void_p
    F64, F32 = _lib.GEMM_F64, _lib.GEMM_F32
    size = lib.gemm_plain_ksplit_workspace_size
    # binary64 256 x 256 x 65536: 4 tiles of 128 x 128 on 256 CUs, 64 chunks of 1024: 63 planes
    assert size(F64, 256, 256, 65536) == 63 * 256 * 256 * 8
    # binary32: 4 tiles of 128 x 128, two per CU: 128 chunks of 512: 127 planes
    assert size(F32, 256, 256, 65536) == 127 * 256 * 256 * 4
    # binary32 1000 x 1000 x 1000: 64 tiles of 128 x 128 would give 8 chunks of 125; 256
    # tiles of 64 x 64, more than one per two CUs: unsplit
    assert size(F32, 1000, 1000, 1000) == 0
    # binary64 128 x 2048 x 4096: 16 chunks of 128 x 128 would be 256 deep: 64 x 64 rule,
    # 64 tiles, 12 chunks asked, 342 rounded up to 384 indices each, so 11 chunks (the last
    # 256 deep): 10 planes
    assert size(F64, 128, 2048, 4096) == 10 * 128 * 2048 * 8
    assert size(F64, 4096, 4096, 4096) == 0      # enough tiles: unsplit
    assert size(F64, 512, 512, 64) == 0          # K too short for two 128-deep chunks
    assert size(7, 256, 256, 65536) == 0 and size(F64, -1, 8, 8) == 0
    assert lib.gemm_tuning_force_ksplit_parts(0) == _lib.GEMM_EINVAL
    assert lib.gemm_tuning_force_ksplit_parts(-2) == _lib.GEMM_EINVAL
    assert lib.gemm_tuning_force_ksplit_parts(3) == _lib.GEMM_OK
    try:
        assert size(F64, 64, 64, 1000) == 2 * 64 * 64 * 8   # 3 chunks of 384
        assert size(F64, 64, 64, 100) == 1 * 64 * 64 * 8    # 2 chunks of 64
    finally:
        assert lib.gemm_tuning_force_ksplit_parts(-1) == _lib.GEMM_OK
    m = n = 256
    k = 65536
    ws = size(F64, m, n, k)

    def call(**kw):
        a = dict(dtype=F64, m=m, n=n, k=k, A=v(256), lda=k, B=v(256), ldb=n, C=v(256), ldc=n,
                 W=v(256), wb=ws)
        a.update(kw)
        return lib.gemm_plain_ksplit(a["dtype"], a["m"], a["n"], a["k"], a["A"], a["lda"], a["B"],
                                     a["ldb"], a["C"], a["ldc"], a["W"], a["wb"], None)

    assert call(W=None) == _lib.GEMM_EWORKSPACE
    assert call(wb=ws - 1) == _lib.GEMM_EWORKSPACE
    assert call(W=v(264)) == _lib.GEMM_EWORKSPACE        # not 16-byte aligned
    assert call(dtype=9) == _lib.GEMM_EUNSUPPORTED
    assert call(m=-1) == _lib.GEMM_EINVAL
    assert call(A=None) == _lib.GEMM_ENULL
    assert call(lda=k - 1) == _lib.GEMM_ELD
    assert call(m=0, A=None, C=None) == _lib.GEMM_OK


def test_ksplit_noalloc_validation(lib):
    """The allocation-free K split checks its arguments like the workspace
    call and refuses, before touching a device, a product whose K split needs
    more than the per-device scratch array holds."""
    v = ctypes.c_void_p
    F64 = _lib.GEMM_F64
    size = lib.gemm_plain_ksplit_workspace_size

    def call(dtype=F64, m=1024, n=1024, k=8192, A=v(256), lda=8192, B=v(256), ldb=1024,
             C=v(256), ldc=1024):
        return lib.gemm_plain_ksplit_noalloc(dtype, m, n, k, A, lda, B, ldb, C, ldc, None)

    assert lib.gemm_tuning_force_ksplit_parts(20) == _lib.GEMM_OK
    try:
        # 20 chunks asked: 410 rounded up to 448 indices, so 19 chunks and 18 planes
        assert size(F64, 1024, 1024, 8192) == 18 * 1024 * 1024 * 8 > _lib.NOALLOC_SCRATCH_BYTES
        assert call() == _lib.GEMM_EWORKSPACE
        assert b"scratch" in lib.gemm_last_error()
    finally:
        assert lib.gemm_tuning_force_ksplit_parts(-1) == _lib.GEMM_OK
    assert call(dtype=9) == _lib.GEMM_EUNSUPPORTED
    assert call(k=-1) == _lib.GEMM_EINVAL
    assert call(B=None) == _lib.GEMM_ENULL
    assert call(ldc=1000) == _lib.GEMM_ELD
    assert call(m=0, A=None, C=None) == _lib.GEMM_OK


def test_backward_validation(lib):
    v = ctypes.c_void_p
    assert lib.gemm_backward(5, 4, 4, 4, v(16), 4, v(16), 4, v(16), 4, v(16), 4, v(16), 4, None) == _lib.GEMM_EUNSUPPORTED
    assert lib.gemm_backward(0, 4, 4, 4, v(16), 4, v(16), 4, None, 4, v(16), 4, v(16), 4, None) == _lib.GEMM_ENULL
    assert lib.gemm_backward(0, 4, 4, 4, v(16), 4, v(16), 3, v(16), 4, v(16), 4, None, 0, None) == _lib.GEMM_ELD
    assert lib.gemm_backward(0, 4, 4, 4, v(16), 3, v(16), 4, v(16), 4, None, 0, v(16), 4, None) == _lib.GEMM_ELD
    assert lib.gemm_backward(0, 4, -1, 4, v(16), 4, v(16), 4, v(16), 4, v(16), 4, v(16), 4, None) == _lib.GEMM_EINVAL


def test_grouped_validation(lib):
    h = ctypes.c_void_p()
    P = _lib.GemmProblem
    arr = (P * 2)(P(4, 4, 4, 16, 16, 16, 4, 4, 4), P(4, 4, 4, 16, 16, 16, 3, 4, 4))
    assert lib.gemm_grouped_plan_create(ctypes.byref(h), 0, arr, 2, None, 0, None) == _lib.GEMM_ELD
    assert b"problem 1" in lib.gemm_last_error()
    assert lib.gemm_grouped_plan_create(ctypes.byref(h), 2, arr, 2, None, 0, None) == _lib.GEMM_EUNSUPPORTED
    assert lib.gemm_grouped_plan_create(ctypes.byref(h), 0, arr, -1, None, 0, None) == _lib.GEMM_EINVAL
    assert lib.gemm_grouped_plan_create(ctypes.byref(h), 0, arr, 1, None, 8, None) == _lib.GEMM_EINVAL
    assert lib.gemm_grouped_plan_create(None, 0, arr, 1, None, 0, None) == _lib.GEMM_ENULL
    arr2 = (P * 1)(P(4, 4, 4, 16, None, 16, 4, 4, 4))
    assert lib.gemm_grouped_plan_create(ctypes.byref(h), 0, arr2, 1, None, 0, None) == _lib.GEMM_ENULL
    assert lib.gemm_grouped_run(None, None) == _lib.GEMM_ENULL
    assert lib.gemm_grouped_plan_destroy(None) == _lib.GEMM_OK


def test_product_path_has_no_oracle_dependency():
    """The package never imports, links or reads the oracle."""
    pkg = os.path.join(ROOT, "paper_1012_2273_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "oracle.c" not in text, f
