"""Serving loop on the device: continuous batching with footprint admission.

Every result must be bitwise the same as the same window solved alone, and
the FP32 results must match the FP64 oracle within the FP32 bar.
"""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from paper_2506_10257_amd.server import Server, request_bytes
from synth import batch_window
from tests.gpu_helpers import device, to_dev, report

pytestmark = pytest.mark.gpu

# up to 60 frames the small eigensolver classes; 100 and 132 frames the wide
# eigensolver (132: FP32 only, its FP32 increment path)
SHAPES = [(64, 64, 10), (96, 64, 20), (64, 128, 40), (128, 128, 20), (48, 80, 12),
          (64, 64, 60), (80, 96, 33), (128, 64, 10), (40, 48, 100), (36, 40, 132)]


def _windows(dtype):
    out = []
    for i, (H, W, n) in enumerate(SHAPES):
        if dtype == np.float64 and n > 128:
            continue
        out.append((i, to_dev(batch_window(H, W, n, 6000 + i).X(), dtype)))
    return out


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("max_active,quantum,budget_of", [(3, 7, None), (16, 16, None), (8, 5, 2)])
def test_server_results_bitwise_equal_alone(dtype, max_active, quantum, budget_of):
    import torch
    device()
    tol, maxit = (1e-6, 300) if dtype == np.float32 else (1e-7, 300)
    wins = _windows(dtype)
    alone = {i: rp.solve(M, tol=tol, maxit=maxit) for i, M in wins}
    dt = rp.RPCA_F32 if dtype == np.float32 else rp.RPCA_F64
    if budget_of is None:
        budget = 1 << 40
    else:  # room for about two of the largest requests at a time
        budget = budget_of * max(request_bytes(M.shape[0], M.shape[1], dt) for _, M in wins)
    srv = Server(dt, hbm_budget=budget, max_active=max_active, quantum=quantum)
    got = {}
    # half the requests arrive first, the rest while those are running
    first, later = wins[: len(wins) // 2], wins[len(wins) // 2:]
    for i, M in first:
        srv.submit(M, tag=i, tol=tol, maxit=maxit)
    steps = 0
    while srv.pending()[0] > 0 or later:
        if steps == 2:
            for i, M in later:
                srv.submit(M, tag=i, tol=tol, maxit=maxit)
            later = []
        for c in srv.step():
            got[c.tag] = c
        steps += 1
        assert steps < 10000
    assert srv.peak_bytes() <= budget
    srv.close()
    torch.cuda.synchronize()
    assert sorted(got) == sorted(alone)
    for i, r in alone.items():
        c = got[i]
        assert c.status == r.status and c.iterations == r.iterations, i
        assert torch.equal(c.L, r.L) and torch.equal(c.S, r.S), i
    report("server_bitwise", dtype=str(np.dtype(dtype)), max_active=max_active, quantum=quantum,
           requests=len(alone), steps=steps)


def test_server_fp32_matches_oracle():
    """A served FP32 window against the FP64 oracle (relative Frobenius error
    <= 1e-4 in L and S, iterations within one)."""
    import torch
    from oracle import rpca
    device()
    w = batch_window(96, 64, 20, 6101)
    X = w.X()
    M = to_dev(X, np.float32)
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 34, max_active=4, quantum=9)
    srv.submit(M, tag=1, tol=1e-6, maxit=500)
    other = to_dev(batch_window(64, 64, 10, 6102).X(), np.float32)
    srv.submit(other, tag=2, tol=1e-6, maxit=500)
    got = {}
    while srv.pending()[0] > 0:
        for c in srv.step():
            got[c.tag] = c
    srv.close()
    ref = rpca(X, tol=1e-6, maxit=500)
    c = got[1]
    L = c.L.t().contiguous().cpu().numpy().T.astype(np.float64)
    S = c.S.t().contiguous().cpu().numpy().T.astype(np.float64)
    eL = np.linalg.norm(L - ref.L) / np.linalg.norm(ref.L)
    eS = np.linalg.norm(S - ref.S) / np.linalg.norm(ref.S)
    report("server_vs_oracle", relL=eL, relS=eS, it=c.iterations, it_ref=ref.iterations)
    assert eL <= 1e-4 and eS <= 1e-4
    assert abs(c.iterations - ref.iterations) <= 1


def test_submit_async_background_bitwise_alone():
    """Futures from a server stepped by its background thread: each result is
    bitwise the window solved alone."""
    import torch
    device()
    wins = _windows(np.float32)[:5]
    alone = {i: rp.solve(M, tol=1e-6, maxit=300) for i, M in wins}
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=3, quantum=8, background=True)
    futs = {i: srv.submit_async(M, tol=1e-6, maxit=300) for i, M in wins}
    got = {i: f.result(timeout=120) for i, f in futs.items()}
    srv.close()
    torch.cuda.synchronize()
    for i, r in alone.items():
        c = got[i]
        assert c.status == r.status and c.iterations == r.iterations
        assert torch.equal(c.L, r.L) and torch.equal(c.S, r.S)
    report("server_async", requests=len(got))
