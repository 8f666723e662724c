"""The server's admission and batching policy, run on the host by the
library's discrete-event simulator (the same policy code the live server
uses).  No GPU needed."""
import numpy as np
import pytest

from paper_2606_22423_amd import _lib, serve

OK, BUSY = _lib.SCAN_OK, _lib.SCAN_EBUSY


def cfg(**kw):
    base = dict(hbm_budget_bytes=1 << 30, max_inflight=256, n_streams=2, max_batch=64, batch_window_us=200)
    base.update(kw)
    return serve.config(**base)


def test_idle_server_launches_at_once_and_busy_streams_batch():
    c = cfg(n_streams=1)
    arr = [0.0, 10.0, 20.0, 30.0]
    launch, done, st, nb = serve.simulate(c, arr, batch_fixed_us=1000.0, per_query_us=1.0)
    assert list(st) == [OK] * 4
    assert launch[0] == 0.0 and done[0] == 1001.0
    # the stream frees at 1001: the three waiting queries go together
    assert list(launch[1:]) == [1001.0] * 3 and nb == 2
    assert np.all(done[1:] == 1001.0 + 1000.0 + 3.0)


def test_window_expiry_launches_on_a_free_stream():
    c = cfg(n_streams=2, batch_window_us=200)
    launch, done, st, nb = serve.simulate(c, [0.0, 10.0], batch_fixed_us=5000.0, per_query_us=0.0)
    assert launch[0] == 0.0
    # stream 1 is free but stream 0 is busy: the second waits for its window
    assert launch[1] == pytest.approx(210.0)
    assert nb == 2


def test_full_batch_launches_without_waiting():
    c = cfg(n_streams=2, max_batch=4, batch_window_us=10_000)
    arr = [0.0] + [1.0 + 0.1 * i for i in range(4)]
    launch, done, st, nb = serve.simulate(c, arr, batch_fixed_us=5000.0, per_query_us=0.0)
    assert launch[0] == 0.0
    assert launch[4] == pytest.approx(1.3)  # the fourth waiting query fills the batch
    assert np.all(launch[1:] == launch[4])


def test_admission_by_slots_and_by_budget():
    arr = [0.0] * 10
    _, _, st, _ = serve.simulate(cfg(max_inflight=4), arr, 100.0, 1.0)
    assert list(st) == [OK] * 4 + [BUSY] * 6
    _, _, st, _ = serve.simulate(cfg(hbm_budget_bytes=2 * 184 + 10), arr, 100.0, 1.0)
    assert list(st) == [OK] * 2 + [BUSY] * 8


def test_poisson_load_invariants():
    rng = np.random.default_rng(3)
    n = 5000
    arr = np.cumsum(rng.exponential(20.0, size=n))  # 50k queries/s
    c = cfg(n_streams=2, max_batch=32, batch_window_us=200, max_inflight=128)
    launch, done, st, nb = serve.simulate(c, arr, batch_fixed_us=300.0, per_query_us=8.0)
    ok = st == OK
    assert ok.sum() > 0.9 * n
    assert np.all(launch[ok] >= arr[ok]) and np.all(done[ok] > launch[ok])
    # FIFO: admitted queries launch in arrival order
    assert np.all(np.diff(launch[ok]) >= 0)
    # no batch exceeds max_batch; every admitted query finished
    _, counts = np.unique(launch[ok], return_counts=True)
    assert counts.max() <= c.max_batch * c.n_streams
    assert nb >= int(np.ceil(ok.sum() / c.max_batch))
    # a query that found a free stream never waited longer than the window
    wait = launch[ok] - arr[ok]
    assert np.percentile(wait, 50) <= 200.0 + 300.0 + 32 * 8.0


def test_invalid_configs_are_rejected():
    for bad in (cfg(max_inflight=0), cfg(n_streams=0), cfg(n_streams=17), cfg(max_batch=0)):
        with pytest.raises(_lib.ScanError):
            serve.simulate(bad, [0.0], 1.0, 1.0)
    with pytest.raises(_lib.ScanError):
        serve.simulate(cfg(), [5.0, 1.0], 1.0, 1.0)  # arrivals must not decrease
    launch, done, st, nb = serve.simulate(cfg(), [], 1.0, 1.0)
    assert len(st) == 0 and nb == 0
