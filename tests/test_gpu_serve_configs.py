"""Serving at the sizes of the Poisson request workload (square windows of
256-1024 px sides, 10/20/40/100 frames, device-built from the request seeds).

* For every cell (side bucket x frame count) the smallest request of the 60 s
  trace in that cell; all 16 are served together and their k = 3 iterates
  (tol = 0) are compared element-wise with the FP64 oracle (<= 1e-4).
* The first 24 requests of the trace arrive a few per server step and are
  served to tol 1e-6; each result is bitwise the same window solved alone.
"""
import numpy as np
import pytest

import paper_2506_10257_amd as rp
from oracle import rpca, rel_fro
from paper_2506_10257_amd.server import Server
from synth import serve_trace, SERVE_FRAMES
from synth.device import device_window
from tests.gpu_helpers import device, to_host, report

pytestmark = pytest.mark.gpu

BUCKETS = ((256, 448), (448, 640), (640, 832), (832, 1025))


def _trace():
    return serve_trace(rate_hz=50.0, duration_s=60.0, seed=5)


def _cells(trace):
    """Smallest request (side, then arrival) of each (side bucket x n) cell."""
    out = []
    for lo, hi in BUCKETS:
        for n in SERVE_FRAMES:
            cand = [(side, i) for i, (_, side, nn, _) in enumerate(trace) if lo <= side < hi and nn == n]
            side, i = min(cand)
            out.append(i)
    return out


def _window(req, dev):
    _, side, n, seed = req
    x = device_window(side, side, n, seed, dev)
    return x.view(n, side * side).t()


def _serve(srv, items, first, per_step, **kw):
    """Submit `first` requests, then `per_step` more before each step."""
    got = {}
    pending = list(items)
    for tag, M in pending[:first]:
        srv.submit(M, tag=tag, **kw)
    pending = pending[first:]
    steps = 0
    while srv.pending()[0] > 0 or pending:
        for tag, M in pending[:per_step]:
            srv.submit(M, tag=tag, **kw)
        pending = pending[per_step:]
        for c in srv.step():
            got[c.tag] = c
        steps += 1
        assert steps < 100000
    return got, steps


@pytest.mark.timeout(1200)
def test_served_cells_iterate_parity():
    import torch
    dev = device()
    trace = _trace()
    cells = _cells(trace)
    K = 3
    items = [(i, _window(trace[i], dev)) for i in cells]
    torch.cuda.synchronize()
    srv = Server(rp.RPCA_F32, hbm_budget=160 << 30, max_active=8, quantum=2)
    got, steps = _serve(srv, items, first=6, per_step=2, tol=0.0, maxit=K)
    srv.close()
    torch.cuda.synchronize()
    worst = 0.0
    for i, M in items:
        _, side, n, _ = trace[i]
        c = got[i]
        X = to_host(M)
        ref = rpca(X, tol=0.0, maxit=K)
        relL, relS = rel_fro(to_host(c.L), ref.L), rel_fro(to_host(c.S), ref.S)
        report(f"served cell {side}x{side}x{n} k={K}", tag=i, it=c.iterations, relL=relL, relS=relS)
        assert c.status == rp.RPCA_NOT_CONVERGED and c.iterations == K
        assert relL <= 1e-4 and relS <= 1e-4
        worst = max(worst, relL, relS)
    report("served cells", cells=len(items), steps=steps, worst=worst)


@pytest.mark.timeout(900)
def test_served_trace_head_bitwise_alone():
    import torch
    dev = device()
    trace = _trace()[:24]
    items = [(i, _window(req, dev)) for i, req in enumerate(trace)]
    torch.cuda.synchronize()
    kw = dict(tol=1e-6, maxit=400)
    srv = Server(rp.RPCA_F32, hbm_budget=160 << 30, max_active=12, quantum=16)
    got, steps = _serve(srv, items, first=4, per_step=3, **kw)
    srv.close()
    torch.cuda.synchronize()
    for i, M in items:
        a = rp.solve(M, **kw)
        torch.cuda.synchronize()
        c = got[i]
        same = torch.equal(a.L, c.L) and torch.equal(a.S, c.S)
        _, side, n, _ = trace[i]
        report(f"served {side}x{side}x{n}", tag=i, it=c.iterations, it_alone=a.iterations,
               bitwise=int(same))
        assert c.status == a.status and c.iterations == a.iterations
        assert same
    report("served trace head", requests=len(items), steps=steps)
