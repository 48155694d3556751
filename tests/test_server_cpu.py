"""Streaming server scheduling, admission and failure handling, on the CPU
(SDD_SERVER_FAKE: no device memory, batches sleep and yield empty results)."""
import time

import numpy as np
import pytest

import paper_2605_03531_amd as sdd
from paper_2605_03531_amd import _capi as A


def _plan(nchan=64, dec_ranges=False):
    f = np.linspace(750.0, 550.0, nchan)
    if dec_ranges:
        return sdd.Plan(f, 81.92e-6, ranges=[(0.0, 10.0, 1.0, 1), (10.0, 20.0, 1.0, 4)],
                        widths=[1, 2], layout="time")
    return sdd.Plan(f, 81.92e-6, dm_list=np.linspace(0.0, 50.0, 16), widths=[1, 2, 4],
                    layout="time")


def _drain(srv, want, timeout_s=10.0):
    got = []
    t0 = time.time()
    while len(got) < want and time.time() - t0 < timeout_s:
        got += srv.poll(64, timeout_us=20000)
    return got


def test_results_for_every_ready_chunk_in_order():
    p = _plan()
    N = 1024
    srv = sdd.Server(hbm_budget=1 << 40, nstreams=2, max_batch=4, fake_exec_us=2000)
    streams = [srv.open(p, N, tag=10 + b) for b in range(5)]
    chunks = 6
    for k in range(chunks):
        for s in streams:
            assert s.submit(None) == 0
    # output chunk k needs (k+1)N + O samples
    per = (chunks * N - p.overlap) // N
    res = _drain(srv, per * 5)
    assert len(res) == per * 5
    for b in range(5):
        ks = [r["chunk"] for r in res if r["tag"] == 10 + b]
        assert ks == list(range(per))
    st = srv.stats()
    assert st["chunks"] == per * 5 and st["batches"] < st["chunks"]  # chunks were batched
    for r in res:
        assert r["t_ready_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
    srv.close()


def test_admission_by_hbm_footprint_and_beam_limit():
    p = _plan(nchan=256)
    N = 4096
    probe = sdd.Server(hbm_budget=1 << 40, fake_exec_us=10)
    ring = probe.footprint(p, N)
    probe.close()
    assert ring == ((p.overlap + N - 1) // N + 2) * N * 256
    # budget for the slot buffers and exactly two rings
    srv = sdd.Server(hbm_budget=1 << 40, max_beams=3, fake_exec_us=10)
    a = srv.open(p, N)
    used = srv.stats()["hbm_used"]
    srv.close()
    srv = sdd.Server(hbm_budget=used + ring, max_beams=3, fake_exec_us=10)
    srv.open(p, N)
    srv.open(p, N)
    with pytest.raises(sdd.SddError) as ei:
        srv.open(p, N)
    assert ei.value.status == A.SDD_EAGAIN
    srv.close()
    srv = sdd.Server(hbm_budget=1 << 40, max_beams=2, fake_exec_us=10)
    srv.open(p, N)
    srv.open(p, N)
    with pytest.raises(sdd.SddError) as ei:
        srv.open(p, N)
    assert ei.value.status == A.SDD_EAGAIN
    srv.close()


def test_backpressure_sequence_gap_and_bad_chunks():
    p = _plan()
    N = 1024
    srv = sdd.Server(hbm_budget=1 << 40, nstreams=1, max_batch=1, ring_chunks=2,
                     fake_exec_us=200000)
    s = srv.open(p, N)
    rc = [s.submit(None) for _ in range(12)]
    assert A.SDD_EAGAIN in rc  # ring full while the slow batch holds its chunk
    k = rc.index(A.SDD_EAGAIN)
    assert all(r == 0 for r in rc[:k])
    with pytest.raises(sdd.SddError) as ei:
        s.submit(None, seq=s.seq + 5)
    assert ei.value.status == A.SDD_ESTATE
    with pytest.raises(sdd.SddError) as ei:
        A.check(A.lib().sdd_stream_submit(s._h, None, N + 1, s.seq, 0), "submit")
    assert ei.value.status == A.SDD_EINVAL
    # results free ring slots again
    assert _drain(srv, 1, 5.0)
    t0 = time.time()
    while s.submit(None) == A.SDD_EAGAIN and time.time() - t0 < 5:
        srv.poll(8, timeout_us=10000)
    srv.close()


def test_poll_timeout_and_close_mid_flight():
    p = _plan(dec_ranges=True)
    N = 1024
    srv = sdd.Server(hbm_budget=1 << 40, nstreams=1, max_batch=2, fake_exec_us=100000)
    t0 = time.time()
    assert srv.poll(4, timeout_us=50000) == []
    assert time.time() - t0 >= 0.04
    s = srv.open(p, N)
    for _ in range((p.overlap + N - 1) // N + 2):
        assert s.submit(None) == 0
    time.sleep(0.02)           # a batch is now in flight
    s.close()                  # waits for it, drops the rest
    res = _drain(srv, 1, 2.0)
    assert 1 <= len(res) <= 2 and srv.stats()["open_streams"] == 0
    with pytest.raises(sdd.SddError):
        A.check(A.lib().sdd_stream_open(srv.handle, _plan(dec_ranges=True).handle, N + 1, 0,
                                        A.C.byref(A.C.c_void_p())), "open")
    srv.close()


def test_stream_rejects_channel_major_plans_and_bad_desc():
    f = np.linspace(750.0, 550.0, 8)
    p = sdd.Plan(f, 81.92e-6, dm_list=[0.0, 1.0], widths=[1], layout="chan")
    srv = sdd.Server(hbm_budget=1 << 30, fake_exec_us=10)
    with pytest.raises(sdd.SddError) as ei:
        srv.open(p, 1024)
    assert ei.value.status == A.SDD_EINVAL
    srv.close()
    with pytest.raises(sdd.SddError):
        sdd.Server(hbm_budget=0, fake_exec_us=10)
    with pytest.raises(sdd.SddError):
        sdd.Server(hbm_budget=1 << 30, nstreams=0, fake_exec_us=10)


def test_snapshot_and_restore_resume_the_sequence():
    """A checkpoint holds the next sequence number, the next unscheduled
    output chunk and the spectra still needed; a stream restored from it
    (on another server) continues the numbering and the output chunks, and
    malformed or mismatched checkpoints are refused."""
    import ctypes as C
    p = _plan()
    N = 1024
    srv = sdd.Server(hbm_budget=1 << 40, nstreams=2, max_batch=4, fake_exec_us=500)
    s = srv.open(p, N, tag=1)
    got = []
    for _ in range(4):
        while s.submit(None) != 0:      # ring full: results first
            got += srv.poll(64, timeout_us=2000)
    ready = max(0, (4 * N - p.overlap) // N)
    got += _drain(srv, ready - len(got))
    assert sorted(r["chunk"] for r in got) == list(range(ready))
    snap = s.snapshot()
    h = np.frombuffer(snap[:64], dtype="<i8")
    submitted, next_out, first, count = int(h[4]), int(h[5]), int(h[6]), int(h[7])
    assert (submitted, next_out, first, count) == (4, ready, ready * N, (4 - ready) * N)
    assert len(snap) == 64 + count * 64
    s.close()
    srv2 = sdd.Server(hbm_budget=1 << 40, nstreams=2, max_batch=4, fake_exec_us=500)
    s2 = srv2.restore(p, snap, tag=2)
    assert s2.seq == 4
    with pytest.raises(sdd.SddError):
        s2.submit(None, seq=3)          # the numbering continues at 4
    got2 = []
    for _ in range(3):
        while s2.submit(None) != 0:
            got2 += srv2.poll(64, timeout_us=2000)
    more = max(0, (7 * N - p.overlap) // N) - ready
    got2 += _drain(srv2, more - len(got2))
    assert sorted(r["chunk"] for r in got2) == list(range(ready, ready + more))
    assert all(r["tag"] == 2 for r in got2)
    # refused: another channel count, a corrupted magic, a truncated buffer
    L = A.lib()
    h2 = C.c_void_p()
    assert L.sdd_stream_restore(srv2.handle, _plan(nchan=32).handle, snap, len(snap), 3,
                                C.byref(h2)) == A.SDD_EINVAL
    bad = b"X" + snap[1:]
    assert L.sdd_stream_restore(srv2.handle, p.handle, bad, len(bad), 3,
                                C.byref(h2)) == A.SDD_EINVAL
    assert L.sdd_stream_restore(srv2.handle, p.handle, snap, len(snap) - 1, 3,
                                C.byref(h2)) == A.SDD_EINVAL
    need = C.c_int64()
    assert L.sdd_stream_snapshot(s2._h, None, 0, C.byref(need)) == A.SDD_OK
    small = C.create_string_buffer(8)
    assert L.sdd_stream_snapshot(s2._h, small, 8, C.byref(need)) == A.SDD_ENOMEM
    s2.close()


def test_injected_batch_failures_are_reported_and_the_streams_go_on():
    """A fake server whose every third batch fails as a device error would:
    the failed output chunks come back with SDD_EDEVICE, every other chunk
    with SDD_OK, each exactly once, and the beams keep streaming."""
    p = _plan()
    N = 1024
    srv = sdd.Server(hbm_budget=1 << 40, nstreams=2, max_batch=2, fake_exec_us=300,
                     fake_fail_every=3)
    streams = [srv.open(p, N, tag=b) for b in range(3)]
    got = []
    for k in range(8):
        for s in streams:
            while s.submit(None) != 0:
                got += srv.poll(64, timeout_us=2000)
    per = (8 * N - p.overlap) // N
    got += _drain(srv, 3 * per - len(got))
    keys = [(r["tag"], r["chunk"]) for r in got]
    assert sorted(keys) == sorted((b, k) for b in range(3) for k in range(per))
    status = [r["status"] for r in got]
    assert A.SDD_EDEVICE in status and A.SDD_OK in status
    assert set(status) <= {A.SDD_OK, A.SDD_EDEVICE}
    assert srv.stats()["batches"] >= 3
    for s in streams:
        s.close()


def test_concurrent_opens_cannot_overrun_the_budget():
    """Two beams opened at once while a batch holds the only slot: both need
    the slots grown, which waits for the slot; the budget fits one of them,
    so exactly one open succeeds and the other gets SDD_EAGAIN (every limit is
    checked again after the wait), and the server never counts more than its
    budget."""
    import threading
    small, big = _plan(nchan=64), _plan(nchan=512)
    N = 1024
    probe = sdd.Server(hbm_budget=1 << 40, nstreams=1, max_batch=1, fake_exec_us=10)
    probe.open(big, N)
    used_big = probe.stats()["hbm_used"]        # slots sized for the big plan + its ring
    ring_small = probe.footprint(small, N)
    probe.close()
    budget = used_big + ring_small
    srv = sdd.Server(hbm_budget=budget, nstreams=1, max_batch=1, fake_exec_us=400000)
    s = srv.open(small, N)
    for _ in range((small.overlap + N - 1) // N + 1):
        assert s.submit(None) == 0
    time.sleep(0.05)                             # the one slot is now busy
    out, gate = [], threading.Barrier(2)

    def opener():
        gate.wait()
        try:
            srv.open(big, N)
            out.append(0)
        except sdd.SddError as e:
            out.append(e.status)

    th = [threading.Thread(target=opener) for _ in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(10.0)
    assert sorted(out) == sorted([0, A.SDD_EAGAIN])
    st = srv.stats()
    assert st["open_streams"] == 2 and st["hbm_used"] <= budget
    srv.close()
