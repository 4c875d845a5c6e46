"""Tuning knobs: every eigensolver workgroup size gives bitwise-identical
results (same arithmetic in the same order); the tile kernel's rows per
workgroup regroup the partial sums, so they keep results within the FP32 bar
of the oracle, and bitwise the same alone or in a batch."""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro
from synth import batch_window
from tests.gpu_helpers import device, to_dev, to_host, report

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,cls", [(12, 16), (20, 32), (40, 64)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_eig_threads_bitwise(n, cls, dtype):
    device()
    X = batch_window(64, 64, n, 3100 + n).X()
    M = to_dev(X, dtype)
    dt = rp.RPCA_F64 if dtype == np.float64 else rp.RPCA_F32
    K = rp.RPCA_KNOB_EIG_THREADS
    old = rp.rpca_tune_get(K, dt, cls)
    outs = []
    try:
        for nt in (256, 512, 1024):
            if rp.rpca_tune_set(K, dt, cls, nt) != rp.RPCA_OK:
                continue
            r = rp.solve(M, tol=1e-6, maxit=60)
            outs.append((nt, r))
    finally:
        rp.rpca_tune_set(K, dt, cls, old)
    assert len(outs) >= 2
    _, r0 = outs[0]
    for nt, r in outs[1:]:
        assert r.iterations == r0.iterations, nt
        assert bool((r.L == r0.L).all()) and bool((r.S == r0.S).all()), nt


def test_autotune_runs_and_keeps_valid_choices(tmp_path):
    device()
    saved = tmp_path / "before.txt"
    assert rp.rpca_autotune_save(str(saved)) == rp.RPCA_OK
    try:
        assert rp.rpca_autotune(rp.RPCA_F32, 65536) == rp.RPCA_OK, rp.rpca_last_error()
        assert rp.rpca_autotune(rp.RPCA_F64, 65536) == rp.RPCA_OK, rp.rpca_last_error()
        ch = rp.tuning_choices()
        assert all(v in (256, 512, 1024) for v in ch["eig_threads"].values())
        assert all(v in (0, 1) for v in ch["stream_kernel"].values())
        assert all(v % 64 == 0 and 64 <= v <= 8192 for v in ch["tile_rows"].values())
        print("[tuning]", ch, flush=True)
    finally:
        rp.rpca_autotune_load(str(saved))


def test_tile_rows_knob_parity_and_batch():
    """40-frame windows on the tile kernel with 256 and 512 rows per
    workgroup (a 131072-row window allows up to 512): the k-th iterate meets
    the oracle's, and a batch at the non-default setting is bitwise equal to
    its solves alone."""
    import torch
    device()
    K, S = rp.RPCA_KNOB_TILE_ROWS, rp.RPCA_KNOB_STREAM_KERNEL
    w = batch_window(256, 512, 40, 7700)
    X = w.X()
    ref = rpca(X, tol=0.0, maxit=3)
    old_rows = rp.rpca_tune_get(K, rp.RPCA_F32, 48)
    old_kind = rp.rpca_tune_get(S, rp.RPCA_F32, 40)
    try:
        assert rp.rpca_tune_set(S, rp.RPCA_F32, 40, 1) == rp.RPCA_OK
        for rows in (256, 512):
            assert rp.rpca_tune_set(K, rp.RPCA_F32, 48, rows) == rp.RPCA_OK
            r = rp.solve(to_dev(X, np.float32), tol=0.0, maxit=3)
            eL, eS = rel_fro(to_host(r.L), ref.L), rel_fro(to_host(r.S), ref.S)
            report(f"tile rows {rows}", relL=eL, relS=eS)
            assert r.iterations == 3 and eL <= 1e-5 and eS <= 1e-5
        shapes = [(256, 512, 40), (128, 128, 40), (64, 96, 20)]
        Ms = [to_dev(batch_window(H, W_, n, 7710 + i).X(), np.float32) for i, (H, W_, n) in enumerate(shapes)]
        alone = [rp.solve(M, tol=1e-6, maxit=150) for M in Ms]
        many = rp.solve_many(Ms, tol=1e-6, maxit=150)
        torch.cuda.synchronize()
        for a, b in zip(alone, many):
            assert a.iterations == b.iterations
            assert torch.equal(a.L, b.L) and torch.equal(a.S, b.S)
    finally:
        rp.rpca_tune_set(K, rp.RPCA_F32, 48, old_rows)
        rp.rpca_tune_set(S, rp.RPCA_F32, 40, old_kind)
