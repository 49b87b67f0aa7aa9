"""Serving scheduler on the simulated executor (no GPU): queueing, continuous
batching, memory admission, FIFO order and latency statistics, with a fake
clock.  A batch started at t finishes at t + launch + rays * per_ray."""
import pytest

import paper_2602_03002_amd as m

LAUNCH, PER_RAY = 1e-3, 1e-9   # 1 ms + 1 ns per ray
PX = 64 * 48


def server(**kw):
    cfg = dict(n_streams=1, max_batch_rays=1 << 24, out_pixels=1 << 24, scratch_bytes=1 << 28)
    cfg.update(kw)
    return m.Server.simulated(LAUNCH, PER_RAY, **cfg)


def drain(s):
    out = []
    while True:
        r = s.next_result()
        if r is None:
            return out
        out.append(r)


def test_single_request_latency():
    s = server()
    rid = s.submit(0.0, 16, 2, 64, 48)
    assert s.poll(0.0) == 0
    done_at = LAUNCH + 16 * 2 * PX * PER_RAY
    assert s.poll(done_at * 0.5) == 0
    assert s.poll(done_at) == 1
    r = drain(s)[0]
    assert r["id"] == rid and r["status"] == 0 and r["n_pixels"] == 16 * 2 * PX
    assert r["launch_s"] == 0.0 and r["done_s"] == pytest.approx(done_at)
    st = s.stats()
    assert st["completed"] == 1 and st["batches"] == 1
    assert st["p50_s"] == pytest.approx(done_at)


def test_requests_arriving_while_busy_are_batched_together():
    s = server()
    a = s.submit(0.0, 64, 1, 64, 48)
    s.poll(0.0)                      # A starts alone
    b = s.submit(1e-4, 32, 2, 32, 24)
    c = s.submit(2e-4, 16, 4, 106, 60)
    s.poll(2e-4)                     # the only stream is busy: B, C wait
    assert s.stats()["queued"] == 2
    t_a = LAUNCH + 64 * PX * PER_RAY
    s.poll(t_a)                      # A done; B and C start together
    assert s.stats()["batches"] == 2 and s.stats()["in_flight"] == 2
    rays_bc = 32 * 2 * 32 * 24 + 16 * 4 * 106 * 60
    s.poll(t_a + LAUNCH + rays_bc * PER_RAY)
    res = drain(s)
    assert [r["id"] for r in res] == [a, b, c]
    assert res[1]["launch_s"] == res[2]["launch_s"] == pytest.approx(t_a)


def test_batch_ray_cap_splits_batches_and_streams_overlap():
    s = server(n_streams=2, max_batch_rays=40 * PX)
    ids = [s.submit(0.0, 32, 1, 64, 48) for _ in range(3)]
    s.poll(0.0)                      # 2 streams: two batches of one request each
    st = s.stats()
    assert st["batches"] == 2 and st["in_flight"] == 2 and st["queued"] == 1
    t1 = LAUNCH + 32 * PX * PER_RAY
    s.poll(t1)
    s.poll(2 * t1)
    assert [r["id"] for r in drain(s)] == ids


def test_memory_admission_waits_for_release():
    s = server(n_streams=2, out_pixels=100 * PX)
    a = s.submit(0.0, 60, 1, 64, 48)
    b = s.submit(0.0, 60, 1, 64, 48)
    s.poll(0.0)
    assert s.stats()["in_flight"] == 1 and s.stats()["queued"] == 1  # B has no room
    t = LAUNCH + 60 * PX * PER_RAY
    s.poll(t)
    r = drain(s)
    assert [x["id"] for x in r] == [a]
    s.poll(t)
    assert s.stats()["queued"] == 1, "outputs of A are still held by the client"
    s.release(a)
    s.poll(t)
    assert s.stats()["in_flight"] == 1 and s.stats()["queued"] == 0
    s.poll(2 * t)
    assert [x["id"] for x in drain(s)] == [b]
    with pytest.raises(m.RcError):
        s.release(a)                 # twice


def test_request_that_can_never_fit_is_rejected():
    s = server(out_pixels=10 * PX)
    with pytest.raises(m.RcError) as e:
        s.submit(0.0, 11, 1, 64, 48)
    assert e.value.status == -2
    assert s.stats()["rejected"] == 1
    with pytest.raises(m.RcError):
        s.submit(0.0, 0, 1, 64, 48)


def test_fifo_order_under_memory_pressure():
    s = server(n_streams=4, out_pixels=100 * PX)
    big = s.submit(0.0, 90, 1, 64, 48)
    s.poll(0.0)
    blocked = s.submit(1e-5, 50, 1, 64, 48)   # needs memory the big one holds
    small = s.submit(2e-5, 5, 1, 64, 48)      # would fit, but may not overtake
    s.poll(2e-5)
    assert s.stats()["queued"] == 2
    t = LAUNCH + 90 * PX * PER_RAY
    s.poll(t)
    s.release(drain(s)[0]["id"])
    s.poll(t)                                 # both start now, in arrival order
    s.poll(1.0)
    assert [r["id"] for r in drain(s)] == [blocked, small]
    del big


def test_latency_percentiles_nearest_rank():
    s = server(n_streams=16)
    # 100 requests arriving together with distinct sizes: latencies are the sizes' run times
    for k in range(1, 101):
        s.submit(0.0, k, 1, 64, 48)
    s.poll(0.0)
    s.poll(100.0)
    st = s.stats()
    assert st["completed"] == 100
    assert st["p50_s"] == pytest.approx(100.0) and st["p99_s"] == pytest.approx(100.0)
    # a poll exactly at each completion gives the model's latencies
    s2 = server(n_streams=1)
    times = []
    t = 0.0
    for k in range(1, 11):
        s2.submit(t, k, 1, 64, 48)
        s2.poll(t)
        t += LAUNCH + k * PX * PER_RAY
        s2.poll(t)
        times.append(LAUNCH + k * PX * PER_RAY)
    st2 = s2.stats()
    times.sort()
    assert st2["p50_s"] == pytest.approx(times[4]) and st2["p99_s"] == pytest.approx(times[9])


def test_injected_failure_fails_only_that_batch():
    """rc_server_fail_next: the requests of the next batch report a device
    error; the batch's memory comes back and later batches succeed."""
    s = server(out_pixels=4 * PX)
    a = s.submit(0.0, 1, 2, 64, 48)
    s.poll(0.0)                       # A starts
    s.fail_next(1)
    b = s.submit(1e-4, 1, 2, 64, 48)  # waits: the only stream is busy
    t_a = LAUNCH + 2 * PX * PER_RAY
    s.poll(t_a)                       # A completes (reported failed), B starts
    assert b"injected" in m.lib().rc_last_error()
    r = drain(s)
    assert [x["id"] for x in r] == [a] and r[0]["status"] == -3
    s.release(a)
    s.poll(t_a + LAUNCH + 2 * PX * PER_RAY)
    r = drain(s)
    assert [x["id"] for x in r] == [b] and r[0]["status"] == 0
    s.release(b)
    c = s.submit(1.0, 2, 2, 64, 48)   # all output memory is free again
    s.poll(1.0)
    s.poll(1.0 + LAUNCH + 4 * PX * PER_RAY)
    r = drain(s)
    assert [x["id"] for x in r] == [c] and r[0]["status"] == 0
    st = s.stats()
    assert st["completed"] == 3 and st["in_flight"] == 0 and st["queued"] == 0
