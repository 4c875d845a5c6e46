"""Tuning knobs change speed only: every eigensolver workgroup size gives
bitwise-identical results (same arithmetic in the same order)."""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from synth import batch_window
from tests.gpu_helpers import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,cls", [(12, 16), (20, 32), (40, 64)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_eig_threads_bitwise(n, cls, dtype):
    device()
    if dtype == np.float64 and n > 32:
        pytest.skip("FP64 streaming classes stop at 32 frames")
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
        print("[tuning]", ch, flush=True)
    finally:
        rp.rpca_autotune_load(str(saved))
