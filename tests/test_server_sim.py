"""CPU tests of the request server's scheduler, driven through the C ABI on the simulated executor
(fge_server_create_simulated): admission order, the HBM budget, max_active, cancellation,
injected launch and device failures, and the threaded mode.  Nothing runs on a GPU; the request
buffers are fake device addresses that the simulated executor only stores.

In manual mode the caller's thread runs the scheduler (fge_server_sim_step) and the clock only
moves when told, so every schedule below is exact: a request takes one tick per fine level
(its first tick also runs the coarse block), ticks complete in launch order.
"""
import threading

import pytest

from paper_2006_14970_amd import fge as fge_mod

# Fake device addresses: request k's I, alpha, F, B at 2^40 + (4k + i) 2^32, far from each other
# and from the simulated arena (at 2^46).
BASE = 1 << 40


def ptrs(k):
    return [BASE + ((4 * k + i) << 32) for i in range(4)]


@pytest.fixture(scope="module")
def fge():
    fge_mod.load()
    return fge_mod


def ticks_of(fge, H, W, p=None):
    info = fge.plan(H, W, p)
    n, nc = len(info.levels), info.n_coarse
    return n - nc if nc < n else 1


def submit(server, k, H, W):
    I, A, F, B = ptrs(k)
    server.submit_ptrs(k, I, A, H, W, F, B)


def run_all(server, max_steps=10000):
    """Complete one tick per step until nothing is in flight; returns the polled results."""
    out = []
    for _ in range(max_steps):
        out += server.poll()
        if server.inflight() == 0:
            server.step(0, 0.0)
            if server.inflight() == 0:
                break
        server.step(1, 0.0)
    out += server.poll()
    return out


def test_single_request_ticks_and_latency(fge):
    p = fge.default_params(storage=fge.F16)
    s = fge.Server.simulated(p, sim=fge.server_sim(us_per_launch=3.0, us_per_mpx=10.0))
    H, W = 768, 1024
    submit(s, 0, H, W)
    assert s.step() == 2                  # two tick slots: the request's first two levels
    assert s.inflight() == 2
    res = run_all(s)
    assert len(res) == 1 and res[0].status == fge.FGE_OK
    assert res[0].ticks == ticks_of(fge, H, W, p)
    assert res[0].submit_ms == 0.0 and res[0].latency_ms == res[0].ready_ms > 0.0
    st = s.stats()
    assert st["ticks"] == res[0].ticks and st["completed"] == 1 and st["failed"] == 0
    s.close()


def test_admission_is_fifo_under_the_budget(fge):
    """The budget fits one large request: a small request queued behind the first large one waits
    for it (strict arrival order), and the second large one waits for both."""
    p = fge.default_params(storage=fge.F16)
    big, small = (1500, 2000), (100, 100)
    budget = fge.server_request_bytes(*big, p)
    assert fge.server_request_bytes(*small, p) < budget
    s = fge.Server.simulated(p, fge.server_config(budget_bytes=budget), arena_bytes=8 << 30)
    submit(s, 0, *big)
    submit(s, 1, *small)
    submit(s, 2, *big)
    s.step()
    st = s.stats()
    assert st["peak_active"] == 1 and st["peak_charged_bytes"] == budget
    res = run_all(s)
    assert [r.id for r in res] == [0, 1, 2]
    assert all(r.status == fge.FGE_OK for r in res)
    assert [r.ticks for r in res] == [ticks_of(fge, *big, p), ticks_of(fge, *small, p),
                                      ticks_of(fge, *big, p)]
    assert res[1].admit_ms >= res[0].ready_ms   # admitted only once the first left the device
    assert s.stats()["peak_charged_bytes"] <= budget
    s.close()


def test_max_active_and_budget_over_a_stream(fge):
    import numpy as np
    rng = np.random.default_rng(3)
    p = fge.default_params(storage=fge.F16)
    sizes = [(int(rng.integers(1, 1200)), int(rng.integers(1, 1200))) for _ in range(120)]
    budget = 3 * max(fge.server_request_bytes(h, w, p) for h, w in sizes)
    s = fge.Server.simulated(p, fge.server_config(budget_bytes=budget, max_active=5),
                             arena_bytes=8 << 30)
    for k, (h, w) in enumerate(sizes):
        submit(s, k, h, w)
    res = run_all(s)
    assert sorted(r.id for r in res) == list(range(len(sizes)))
    assert all(r.status == fge.FGE_OK for r in res)
    for r in res:
        assert r.ticks == ticks_of(fge, *sizes[r.id], p), r.id
    st = s.stats()
    assert st["peak_active"] == 5 and st["peak_charged_bytes"] <= budget
    assert st["mixed_ticks"] > 0 and st["admitted_while_busy"] > 0
    assert st["completed"] == st["submitted"] == len(sizes)
    s.close()


def test_cancel_queued_requests_only(fge):
    p = fge.default_params()
    budget = fge.server_request_bytes(768, 1024, p)
    s = fge.Server.simulated(p, fge.server_config(budget_bytes=budget), arena_bytes=4 << 30)
    for k in range(3):
        submit(s, k, 768, 1024)
    assert s.cancel(2)                    # not taken in yet
    s.step()                              # request 0 admitted, 1 queued behind the budget
    assert s.cancel(1)                    # queued in the scheduler
    assert not s.cancel(0)                # admitted: runs to completion
    assert not s.cancel(1)                # already cancelled
    assert not s.cancel(77)               # unknown
    res = run_all(s)
    by_id = {r.id: r for r in res}
    assert by_id[2].status == fge.FGE_ECANCELED and by_id[1].status == fge.FGE_ECANCELED
    assert by_id[0].status == fge.FGE_OK and by_id[2].ticks == 0
    st = s.stats()
    assert st["cancelled"] == 2 and st["completed"] == 3 and st["failed"] == 0
    s.drain()
    s.close()


def test_launch_failure_fails_only_that_ticks_requests(fge):
    """The 2nd tick's launch fails: the two requests in it fail with FGE_EHIP, their memory and
    budget are released, and the server goes on serving new requests."""
    p = fge.default_params()
    budget = 2 * fge.server_request_bytes(768, 1024, p)
    s = fge.Server.simulated(p, fge.server_config(budget_bytes=budget), arena_bytes=4 << 30,
                             sim=fge.server_sim(fail_launch_tick=2))
    submit(s, 0, 768, 1024)
    submit(s, 1, 768, 1024)
    s.step()
    res = run_all(s)
    assert sorted((r.id, r.status) for r in res) == [(0, fge.FGE_EHIP), (1, fge.FGE_EHIP)]
    assert s.stats()["failed"] == 2
    # the budget was given back: two more requests of the same size are admitted together
    submit(s, 2, 768, 1024)
    submit(s, 3, 768, 1024)
    s.step()
    assert s.stats()["peak_active"] == 2
    res = run_all(s)
    assert sorted((r.id, r.status) for r in res) == [(2, fge.FGE_OK), (3, fge.FGE_OK)]
    assert all(r.ticks == ticks_of(fge, 768, 1024, p) for r in res)
    st = s.stats()
    assert st["completed"] == 4 and st["failed"] == 2
    s.close()


def test_device_failure_ends_the_server(fge):
    p = fge.default_params()
    s = fge.Server.simulated(p, arena_bytes=4 << 30, sim=fge.server_sim(fail_device_tick=1))
    for k in range(3):
        submit(s, k, 300 + 50 * k, 400)
    s.step()
    with pytest.raises(fge.FgeError):
        s.step(1, 0.0)                    # the first tick reports its error: the server fails
    res = s.poll()
    assert sorted(r.id for r in res) == [0, 1, 2]
    assert all(r.status == fge.FGE_EHIP for r in res)
    with pytest.raises(fge.FgeError):
        submit(s, 9, 64, 64)
    with pytest.raises(fge.FgeError):
        s.poll()                          # nothing left to report: the server's error
    assert s.stats()["failed"] == 3
    s.close()


def test_threaded_mode_with_concurrent_submitters(fge):
    """The simulated executor with its own scheduler thread and the host clock: four threads
    submit, one cancels, the caller drains; every request completes exactly once."""
    p = fge.default_params(storage=fge.F16)
    s = fge.Server.simulated(p, fge.server_config(max_active=16), arena_bytes=16 << 30,
                             sim=fge.server_sim(manual=0, us_per_launch=1.0, us_per_mpx=2.0))
    per, nthreads = 40, 4
    errors = []

    def work(t):
        try:
            for i in range(per):
                k = t * per + i
                submit(s, k, 64 + (k * 37) % 900, 64 + (k * 53) % 700)
        except Exception as e:   # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(t,)) for t in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    s.cancel(nthreads * per - 1)          # may or may not still be queued
    s.drain()
    res = s.poll()
    assert not errors
    assert sorted(r.id for r in res) == list(range(nthreads * per))
    assert all(r.status in (fge.FGE_OK, fge.FGE_ECANCELED) for r in res)
    assert all(r.latency_ms >= 0.0 for r in res if r.status == fge.FGE_OK)
    st = s.stats()
    assert st["completed"] == st["submitted"] == nthreads * per and st["failed"] == 0
    s.close()


def test_simulated_argument_errors(fge):
    lib = fge.load()
    import ctypes
    out = ctypes.c_void_p()
    bad = fge.server_sim(manual=2)
    assert lib.fge_server_create_simulated(None, None, 1 << 30, ctypes.byref(bad),
                                           ctypes.byref(out)) == fge.FGE_EINVAL
    bad = fge.server_sim(us_per_mpx=-1.0)
    assert lib.fge_server_create_simulated(None, None, 1 << 30, ctypes.byref(bad),
                                           ctypes.byref(out)) == fge.FGE_EINVAL
    assert lib.fge_server_create_simulated(None, None, 1024, None,
                                           ctypes.byref(out)) == fge.FGE_EWORKSPACE
    s = fge.Server.simulated(sim=fge.server_sim(manual=0))
    assert lib.fge_server_sim_step(s._h, 0, 0.0) == fge.FGE_EINVAL   # not in manual mode
    s.close()
    s = fge.Server.simulated()
    assert lib.fge_server_sim_step(s._h, -1, 0.0) == fge.FGE_EINVAL
    with pytest.raises(fge.FgeError):
        submit(s, 0, 0, 10)
    with pytest.raises(fge.FgeError):     # a request larger than the whole budget
        s2 = fge.Server.simulated(config=fge.server_config(budget_bytes=1 << 20))
        submit(s2, 0, 2000, 2000)
    s.close()
