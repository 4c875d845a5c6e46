"""The C-ABI library loads, exports every symbol include/rpca.h declares, and
rejects invalid arguments on the host before touching a device.  No compute
call runs here (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2506_10257_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpca.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpca_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rpca_solve_f64", "rpca_solve_f32", "rpca_solve_many",
                 "rpca_footprint_bytes", "rpca_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) <= set(_declared())


def test_strerror_and_version(lib):
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.rpca_strerror(code)
    assert lib.rpca_strerror(99) == b"unknown status"
    assert lib.rpca_version().startswith(b"rpca_mi355x")


def test_footprint(lib):
    f32 = lib.rpca_footprint_bytes(262144, 20, _lib.RPCA_F32)
    f64 = lib.rpca_footprint_bytes(262144, 20, _lib.RPCA_F64)
    mat32 = 262144 * 20 * 4
    assert 4 * mat32 <= f32 < 4 * mat32 + (4 << 20)
    assert 8 * mat32 <= f64 < 8 * mat32 + (8 << 20)
    assert lib.rpca_footprint_bytes(0, 20, _lib.RPCA_F32) == 0
    assert lib.rpca_footprint_bytes(100, 0, _lib.RPCA_F32) == 0
    assert lib.rpca_footprint_bytes(100, 145, _lib.RPCA_F32) == 0
    assert lib.rpca_footprint_bytes(100, 20, 7) == 0


def _call(lib, M, m, n, L, S, maxit=10, fn="rpca_solve_f32"):
    it = ctypes.c_int32(-7)
    rc = getattr(lib, fn)(M, m, n, -1.0, -1.0, 1e-6, maxit, L, S, ctypes.byref(it), None)
    return rc, it.value


def test_invalid_arguments_rejected_on_host(lib):
    A, B, C = 1 << 40, 2 << 40, 3 << 40       # disjoint fake device ranges
    assert _call(lib, None, 100, 4, B, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 4, None, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 4, B, None)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 0, 4, B, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 0, B, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 145, B, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 4, B, C, maxit=0)[0] == _lib.RPCA_ERR_ARG
    # overlapping M / L / S
    assert _call(lib, A, 100, 4, A + 16, C)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 4, B, B + 1596)[0] == _lib.RPCA_ERR_ARG
    assert _call(lib, A, 100, 4, B, B, fn="rpca_solve_f64")[0] == _lib.RPCA_ERR_ARG
    # iterations is written as 0 on failure
    assert _call(lib, None, 100, 4, B, C)[1] == 0


def test_batch_argument_checks(lib):
    P = _lib.RpcaProblem
    arr = (P * 1)()
    assert lib.rpca_solve_many(arr, 0, _lib.RPCA_F32, 0, None) == _lib.RPCA_ERR_ARG
    assert lib.rpca_solve_many(arr, 1, 5, 0, None) == _lib.RPCA_ERR_ARG
    assert lib.rpca_solve_many(arr, 1, _lib.RPCA_F32, 9, None) == _lib.RPCA_ERR_ARG
    assert lib.rpca_solve_many(arr, 1, _lib.RPCA_F32, 0, None) == _lib.RPCA_ERR_ARG  # NULL M


def test_tuning_knobs(lib):
    import paper_2506_10257_amd as rp
    K = rp.RPCA_KNOB_EIG_THREADS
    for dt in (rp.RPCA_F32, rp.RPCA_F64):
        for cls in (16, 32, 64):
            assert rp.rpca_tune_get(K, dt, cls) in (256, 512, 1024)
    old = rp.rpca_tune_get(K, rp.RPCA_F32, 64)
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 64, 512) == rp.RPCA_OK
    assert rp.rpca_tune_get(K, rp.RPCA_F32, 64) == 512
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 64, old) == rp.RPCA_OK
    # invalid class, value, dtype and knob leave the table unchanged
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 24, 256) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 16, 1024) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 32, 300) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, 7, 32, 256) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(99, rp.RPCA_F32, 32, 256) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_get(99, rp.RPCA_F32, 32) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_get(K, rp.RPCA_F32, 64) == old


def test_frame_limits(lib):
    A, B, C = 1 << 40, 2 << 40, 3 << 40
    assert _lib.RPCA_N_MAX == 144
    assert _call(lib, A, 100, 145, B, C)[0] == _lib.RPCA_ERR_ARG
    # FP64 solves stop at 128 frames (RPCA_N_MAX_F64), FP32 solves at 144
    assert _lib.RPCA_N_MAX_F64 == 128
    assert _call(lib, A, 100, 129, B, C, fn="rpca_solve_f64")[0] == _lib.RPCA_ERR_UNSUPPORTED
    for n in (112, 113, 128, 132, 144):
        assert lib.rpca_footprint_bytes(4096, n, _lib.RPCA_F32) > 0
    for n in (33, 64, 65, 100, 112, 113, 128):
        assert lib.rpca_footprint_bytes(4096, n, _lib.RPCA_F64) > 0
    assert lib.rpca_footprint_bytes(4096, 145, _lib.RPCA_F32) == 0
    assert lib.rpca_footprint_bytes(4096, 129, _lib.RPCA_F64) == 0
    # the 144-frame class holds a 144 x 144 FP64 scratch for the eigensolver's
    # warm start beside its V, P and partials
    assert (lib.rpca_footprint_bytes(4096, 132, _lib.RPCA_F32)
            > lib.rpca_footprint_bytes(4096, 112, _lib.RPCA_F32) + 144 * 144 * 8)
    # the split-BF16 mode is FP32 only
    p = _lib.RpcaProblem()
    p.M, p.L, p.S, p.m, p.n, p.maxit = A, B, C, 100, 4, 10
    assert lib.rpca_solve_ex(ctypes.byref(p), _lib.RPCA_F64, _lib.RPCA_GRAM_BF16X3, None) == _lib.RPCA_ERR_ARG
    assert lib.rpca_solve_ex(ctypes.byref(p), _lib.RPCA_F64, _lib.RPCA_GRAM_BF16X6, None) == _lib.RPCA_ERR_ARG
    assert lib.rpca_solve_ex(ctypes.byref(p), _lib.RPCA_F32, 3, None) == _lib.RPCA_ERR_ARG


def test_stream_kernel_knob(lib):
    import paper_2506_10257_amd as rp
    K = rp.RPCA_KNOB_STREAM_KERNEL
    for cls in (4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60, 64):
        assert rp.rpca_tune_get(K, rp.RPCA_F32, cls) in (0, 1)
    old = rp.rpca_tune_get(K, rp.RPCA_F32, 40)
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 40, 1) == rp.RPCA_OK
    assert rp.rpca_tune_get(K, rp.RPCA_F32, 40) == 1
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 40, old) == rp.RPCA_OK
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 44, 1) == rp.RPCA_ERR_ARG   # not a class
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 80, 0) == rp.RPCA_ERR_ARG   # tile kernel only
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 40, 2) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, rp.RPCA_F64, 20, 1) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_get(K, rp.RPCA_F64, 20) == rp.RPCA_ERR_ARG


def test_tile_rows_knob(lib):
    import paper_2506_10257_amd as rp
    K = rp.RPCA_KNOB_TILE_ROWS
    for nb in range(16, 145, 16):
        assert rp.rpca_tune_get(K, rp.RPCA_F32, nb) == 1024
    old = rp.rpca_tune_get(K, rp.RPCA_F32, 64)
    try:
        for rows in (64, 256, 512, 768, 1024, 2048, 4096, 8192):
            assert rp.rpca_tune_set(K, rp.RPCA_F32, 64, rows) == rp.RPCA_OK
            assert rp.rpca_tune_get(K, rp.RPCA_F32, 64) == rows
    finally:
        assert rp.rpca_tune_set(K, rp.RPCA_F32, 64, old) == rp.RPCA_OK
    for bad in (0, 32, 100, 8256):
        assert rp.rpca_tune_set(K, rp.RPCA_F32, 64, bad) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 40, 512) == rp.RPCA_ERR_ARG   # not a tile class
    assert rp.rpca_tune_set(K, rp.RPCA_F32, 160, 512) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_set(K, rp.RPCA_F64, 64, 512) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_get(K, rp.RPCA_F64, 64) == rp.RPCA_ERR_ARG
    assert rp.rpca_tune_get(K, rp.RPCA_F32, 64) == old


def test_tile_rows_change_the_footprint(lib):
    """Fewer rows per workgroup mean more partial slots in the workspace."""
    import paper_2506_10257_amd as rp
    K = rp.RPCA_KNOB_TILE_ROWS
    old = rp.rpca_tune_get(K, rp.RPCA_F32, 112)
    try:
        big = lib.rpca_footprint_bytes(262144, 100, rp.RPCA_F32)
        assert rp.rpca_tune_set(K, rp.RPCA_F32, 112, 256) == rp.RPCA_OK
        small = lib.rpca_footprint_bytes(262144, 100, rp.RPCA_F32)
    finally:
        rp.rpca_tune_set(K, rp.RPCA_F32, 112, old)
    assert small > big
    assert lib.rpca_footprint_bytes(262144, 100, rp.RPCA_F32) == big
    # a 65536-row window is capped at 256 rows per workgroup (256 workgroups),
    # whatever the knob says
    try:
        capped = lib.rpca_footprint_bytes(65536, 100, rp.RPCA_F32)
        assert rp.rpca_tune_set(K, rp.RPCA_F32, 112, 256) == rp.RPCA_OK
        assert lib.rpca_footprint_bytes(65536, 100, rp.RPCA_F32) == capped
    finally:
        rp.rpca_tune_set(K, rp.RPCA_F32, 112, old)


def test_autotune_save_load_roundtrip(lib, tmp_path):
    import paper_2506_10257_amd as rp
    K, S = rp.RPCA_KNOB_EIG_THREADS, rp.RPCA_KNOB_STREAM_KERNEL
    before = rp.tuning_choices()
    path = tmp_path / "tune.txt"
    assert rp.rpca_autotune_save(str(path)) == rp.RPCA_OK
    try:
        rp.rpca_tune_set(K, rp.RPCA_F32, 64, 256)
        rp.rpca_tune_set(S, rp.RPCA_F32, 40, 1 - before["stream_kernel"][40])
        rp.rpca_tune_set(rp.RPCA_KNOB_TILE_ROWS, rp.RPCA_F32, 96, 512)
        assert rp.tuning_choices() != before
        assert rp.rpca_autotune_load(str(path)) == rp.RPCA_OK
        assert rp.tuning_choices() == before
        # a bad line is reported, the valid ones are still applied
        bad = tmp_path / "bad.txt"
        bad.write_text(f"{S} {rp.RPCA_F32} 40 {1 - before['stream_kernel'][40]}\n9 9 9 9\n")
        assert rp.rpca_autotune_load(str(bad)) == rp.RPCA_ERR_ARG
        assert rp.rpca_tune_get(S, rp.RPCA_F32, 40) == 1 - before["stream_kernel"][40]
        assert rp.rpca_autotune_load(str(tmp_path / "missing.txt")) == rp.RPCA_ERR_ARG
        assert lib.rpca_autotune(7, 4096, None) == rp.RPCA_ERR_ARG
        assert lib.rpca_autotune(rp.RPCA_F32, 10, None) == rp.RPCA_ERR_ARG
    finally:
        rp.rpca_autotune_load(str(path))
    assert rp.tuning_choices() == before


def test_noalloc_rejects_what_does_not_fit(lib):
    """rpca_solve_noalloc refuses a solve larger than its static scratch, and
    invalid arguments, before any device call."""
    A, B, C = 1 << 40, 2 << 40, 3 << 40
    it = ctypes.c_int32(7)
    f = lib.rpca_solve_noalloc
    m = 1 << 22                                   # 4 x 16 MiB x 20 frames of iterates
    assert lib.rpca_footprint_bytes(m, 20, _lib.RPCA_F32) > _lib.RPCA_NOALLOC_MAX_BYTES
    assert f(A, m, 20, _lib.RPCA_F32, -1.0, -1.0, 1e-6, 10, B, C, ctypes.byref(it), None) \
        == _lib.RPCA_ERR_ARG
    assert it.value == 0
    assert b"RPCA_NOALLOC_MAX_BYTES" in lib.rpca_last_error()
    assert f(A, 100, 4, 7, -1.0, -1.0, 1e-6, 10, B, C, None, None) == _lib.RPCA_ERR_ARG
    assert f(A, 100, 4, _lib.RPCA_F32, -1.0, -1.0, 1e-6, 0, B, C, None, None) == _lib.RPCA_ERR_ARG
    assert f(A, 100, 4, _lib.RPCA_F32, -1.0, -1.0, 1e-6, 10, A, C, None, None) == _lib.RPCA_ERR_ARG
    # the 512 x 512 x 20 window fits in both precisions
    for dt in (_lib.RPCA_F32, _lib.RPCA_F64):
        assert lib.rpca_footprint_bytes(262144, 20, dt) + 4096 <= _lib.RPCA_NOALLOC_MAX_BYTES
