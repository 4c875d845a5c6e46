"""Admission and retirement logic of the serving loop, run without a device
(RPCA_SERVER_SIMULATE: no HIP call is made; a request finishes after maxit
iterations counted in quanta)."""
import ctypes

import pytest

import paper_2506_10257_amd as rp
from paper_2506_10257_amd import _lib
from paper_2506_10257_amd.server import Server, request_bytes


def _prob(m, n, maxit, base):
    """Problem with placeholder device addresses (never dereferenced here)."""
    p = _lib.RpcaProblem()
    span = m * n * 4
    p.M, p.L, p.S = base, base + 2 * span, base + 4 * span
    p.m, p.n = m, n
    p.lam, p.mu, p.tol, p.maxit = -1.0, -1.0, 1e-6, maxit
    return p


def _drain(srv, max_steps=1000):
    order, trace = [], []
    for _ in range(max_steps):
        left, q, a, used = srv.pending()
        if left == 0:
            break
        trace.append((q, a, used))
        order += [(c.tag, c.status, c.iterations) for c in srv.step()]
    return order, trace


def test_fifo_and_max_active():
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=2, quantum=16, simulate=True)
    for t in range(6):
        assert srv.submit_raw(_prob(4096, 20, 32, (t + 1) << 32), t) == 0
    order, trace = _drain(srv)
    assert [t for t, _, _ in order] == list(range(6))
    assert all(st == rp.RPCA_NOT_CONVERGED and it == 32 for _, st, it in order)
    assert max(a for _, a, _ in trace) <= 2
    srv.close()


def test_budget_and_head_of_line():
    big = request_bytes(65536, 40, rp.RPCA_F32)
    small = request_bytes(4096, 10, rp.RPCA_F32)
    assert big > 2 * small > 0
    srv = Server(rp.RPCA_F32, hbm_budget=big, max_active=8, quantum=10, simulate=True)
    srv.submit_raw(_prob(65536, 40, 30, 1 << 36), 0)  # needs 3 steps
    srv.submit_raw(_prob(4096, 10, 10, 2 << 36), 1)
    srv.submit_raw(_prob(4096, 10, 10, 3 << 36), 2)
    order, trace = _drain(srv)
    # the small requests do not overtake the big one at the head of the queue
    assert [t for t, _, _ in order] == [0, 1, 2]
    assert srv.peak_bytes() <= big
    assert all(used <= big for _, _, used in trace)
    srv.close()


def test_oversized_request_rejected_with_nomem():
    small = request_bytes(4096, 10, rp.RPCA_F32)
    srv = Server(rp.RPCA_F32, hbm_budget=small, max_active=4, quantum=8, simulate=True)
    srv.submit_raw(_prob(65536, 40, 8, 1 << 36), 5)
    srv.submit_raw(_prob(4096, 10, 8, 2 << 36), 6)
    order, _ = _drain(srv)
    assert order[0] == (5, rp.RPCA_ERR_NOMEM, 0)
    assert order[1][0] == 6 and order[1][1] == rp.RPCA_NOT_CONVERGED
    srv.close()


def test_continuous_admission():
    """A request submitted while others run joins without waiting for them."""
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=4, quantum=10, simulate=True)
    srv.submit_raw(_prob(4096, 20, 100, 1 << 36), 0)  # 10 steps
    srv.step()
    srv.step()
    srv.submit_raw(_prob(4096, 20, 20, 2 << 36), 1)  # 2 steps
    assert srv.pending()[2] == 1
    got = srv.step()
    assert got == [] and srv.pending()[2] == 2
    got = srv.step()
    assert [c.tag for c in got] == [1]
    order, _ = _drain(srv)
    assert [t for t, _, _ in order] == [0]
    srv.close()


def test_submit_rejects_what_a_solve_rejects():
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 30, max_active=2, quantum=4, simulate=True)
    assert srv.submit_raw(_prob(4096, 0, 10, 1 << 36), 0) == rp.RPCA_ERR_ARG
    assert srv.submit_raw(_prob(4096, rp.RPCA_N_MAX + 1, 10, 1 << 36), 0) == rp.RPCA_ERR_ARG
    assert srv.submit_raw(_prob(4096, 10, 0, 1 << 36), 0) == rp.RPCA_ERR_ARG
    p = _prob(4096, 10, 10, 1 << 36)
    p.S = p.M  # aliasing
    assert srv.submit_raw(p, 0) == rp.RPCA_ERR_ARG
    assert srv.pending()[0] == 0
    srv.close()


@pytest.mark.parametrize("args", [
    dict(dtype=7), dict(hbm_budget=0), dict(max_active=0), dict(quantum=0)])
def test_create_rejects_bad_arguments(args):
    kw = dict(dtype=rp.RPCA_F32, hbm_budget=1 << 30, max_active=2, quantum=4, simulate=True)
    kw.update(args)
    with pytest.raises(ValueError):
        Server(**kw)


def test_timeout_of_queued_and_active_requests():
    """A request past its timeout completes with RPCA_ERR_TIMEOUT, queued or
    active; the others are unaffected (simulated clock: 1 ms per step)."""
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=1, quantum=10, simulate=True)
    srv.set_timeout(0.0035)                               # 3.5 steps
    srv.submit_raw(_prob(4096, 20, 10000, 1 << 36), 0)  # "hangs": would need 1000 steps
    srv.submit_raw(_prob(4096, 20, 20, 2 << 36), 1)     # queued behind it
    srv.set_timeout(0.0)
    srv.submit_raw(_prob(4096, 20, 20, 3 << 36), 2)     # no timeout
    order, _ = _drain(srv)
    got = {t: (st, it) for t, st, it in order}
    assert got[0][0] == rp.RPCA_ERR_TIMEOUT and 0 < got[0][1] < 10000
    assert got[1] == (rp.RPCA_ERR_TIMEOUT, 0)             # timed out while queued
    assert got[2] == (rp.RPCA_NOT_CONVERGED, 20)
    # the queued request expires first in the step where both pass 3.5 ms
    assert [t for t, _, _ in order] == [1, 0, 2]
    assert srv.pending() == (0, 0, 0, 0)
    srv.close()


def test_set_timeout_rejects_bad_values():
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 30, max_active=2, quantum=4, simulate=True)
    for bad in (-1.0, float("nan")):
        with pytest.raises(ValueError):
            srv.set_timeout(bad)
    srv.close()


@pytest.mark.parametrize("code", [rp.RPCA_ERR_NOMEM, rp.RPCA_ERR_DEVICE])
def test_failed_init_releases_requests(code):
    """A failure while admitted requests are set up completes them with the
    failure's code and gives their footprint back; later requests still run."""
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=4, quantum=8, simulate=True)
    srv.submit_raw(_prob(4096, 20, 16, 1 << 36), 0)
    srv.submit_raw(_prob(8192, 10, 16, 2 << 36), 1)
    assert srv.inject_failure(code) == rp.RPCA_OK
    got = srv.step()
    assert sorted((c.tag, c.status) for c in got) == [(0, code), (1, code)]
    assert srv.pending() == (0, 0, 0, 0)      # nothing queued, active or held
    srv.submit_raw(_prob(4096, 20, 16, 3 << 36), 2)
    order, _ = _drain(srv)
    assert order == [(2, rp.RPCA_NOT_CONVERGED, 16)]
    assert srv.inject_failure(5) == rp.RPCA_ERR_ARG          # codes are negative
    assert srv._lib.rpca_server_inject_failure(srv._h, 9, -2) == rp.RPCA_ERR_ARG  # unknown stage
    srv.close()


def test_duplicate_tag_rejected_until_reported():
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=1, quantum=8, simulate=True)
    assert srv.submit_raw(_prob(4096, 20, 8, 1 << 36), 7) == 0
    assert srv.submit_raw(_prob(4096, 20, 8, 2 << 36), 7) == rp.RPCA_ERR_ARG   # queued
    n = ctypes.c_int32(0)
    buf = (_lib.RpcaCompletion * 4)()
    assert srv._lib.rpca_server_step(srv._h, buf, 0, ctypes.byref(n)) == 0  # done, not reported
    assert srv.submit_raw(_prob(4096, 20, 8, 2 << 36), 7) == rp.RPCA_ERR_ARG   # still held
    got = srv.step()
    assert [c.tag for c in got] == [7]
    assert srv.submit_raw(_prob(4096, 20, 8, 2 << 36), 7) == 0                 # free again
    srv.close()


def test_python_submit_checks():
    """Server.submit refuses a repeated tag, a dtype other than the server's
    and a host tensor before anything reaches the library."""
    import torch
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=2, quantum=8, simulate=True)
    assert srv.submit_raw(_prob(4096, 20, 8, 1 << 36), 3, keep=()) == 0
    M32 = torch.zeros(64, 4, dtype=torch.float32).t().contiguous().t()
    with pytest.raises(ValueError, match="tag"):
        srv.submit(M32, tag=3)
    with pytest.raises(ValueError, match="dtype"):
        srv.submit(M32.double(), tag=4)
    with pytest.raises(ValueError, match="device"):
        srv.submit(M32, tag=4)
    assert srv.pending()[1] == 1
    srv.close()


def _future_request(srv, p):
    """What Server.submit_async does once its device checks passed (the
    simulated server takes placeholder addresses instead of tensors)."""
    import concurrent.futures
    fut = concurrent.futures.Future()
    with srv._mu:
        tag = next(srv._tags)
        srv._futures[tag] = fut
        assert srv.submit_raw(p, tag) == 0
    srv._wake.set()
    return fut


def test_submit_async_futures_resolve_on_step():
    """A future-backed request is resolved by the step that reports it;
    requests submitted with plain tags are returned by step()."""
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=4, quantum=8, simulate=True)
    srv.submit_raw(_prob(4096, 20, 16, 1 << 36), 5)
    futs = [_future_request(srv, _prob(4096, 10, 8 * (i + 1), (i + 2) << 36)) for i in range(3)]
    plain = []
    for _ in range(10):
        plain += srv.step()
    assert [c.tag for c in plain] == [5]
    assert all(f.done() for f in futs)
    assert [f.result().iterations for f in futs] == [8, 16, 24]
    srv.close()


def test_background_server_resolves_futures_and_closes():
    import concurrent.futures
    import time
    srv = Server(rp.RPCA_F32, hbm_budget=1 << 40, max_active=2, quantum=4, simulate=True,
                 background=True)
    futs = [_future_request(srv, _prob(4096, 10, 4 * (i + 1), (i + 1) << 36)) for i in range(5)]
    done, _ = concurrent.futures.wait(futs, timeout=30)
    assert len(done) == 5
    assert sorted(f.result().iterations for f in futs) == [4, 8, 12, 16, 20]
    # a request still running when the server closes gets its future cancelled
    fut = _future_request(srv, _prob(4096, 10, 10 ** 6, 9 << 36))
    time.sleep(0.05)
    srv.close()
    assert fut.cancelled()
