"""Continuous-batching server on the simulated backend (no device): admission
by the memory budget, batching of requests that arrive while others run,
overlap of batches, arrival order, cancellation, queue time-outs and the
latency statistics.  The device backend runs the same scheduler; its results
are checked against the oracle in test_gpu_server.py."""
import time

import pytest

import paper_2605_17222_amd as H



@pytest.fixture(autouse=True, scope="module")
def _library_built():
    # Built here if missing (a clean tree): these tests must run, not skip.
    if not H.os.path.exists(H.LIB_PATH):
        from paper_2605_17222_amd import build
        build.build()
    yield

MiB = 1 << 20


def _server(budget=64 * MiB, batch=4, inflight=2, service=0.2, timeout=0.0):
    S = H.Server(budget, max_batch=batch, max_inflight=inflight, simulated=True, queue_timeout_s=timeout,
                 simulated_service_s=service)
    ring = H.ckks_server_add_ring(S, None, {})
    return S, ring


def _submit(S, ring, ws=MiB):
    return H.ckks_server_submit(S, ring, level=1, sim_ws_bytes=ws)


def _wait_status(S, rid, want, limit=5.0):
    t0 = time.time()
    while time.time() - t0 < limit:
        st, _ = H.ckks_server_poll(S, rid)
        if st == want:
            return True
        time.sleep(0.002)
    return False


def test_request_larger_than_budget_is_refused():
    S, ring = _server(budget=4 * MiB)
    with pytest.raises(H.CkksError) as e:
        _submit(S, ring, ws=5 * MiB)
    assert e.value.code == H.CKKS_E_WORKSPACE
    rid = _submit(S, ring, ws=4 * MiB)
    H.ckks_server_wait_all(S)
    assert H.ckks_server_poll(S, rid)[0] == H.CKKS_OK
    st = H.ckks_server_stats(S)
    assert st["rejected"] == 1 and st["completed"] == 1
    S.close()


def test_arrivals_during_a_batch_start_on_a_free_stream():
    # Continuous batching: a request that arrives while a batch runs is
    # admitted on the other stream without waiting for that batch.
    S, ring = _server(inflight=2, service=0.6)
    a = _submit(S, ring)
    assert _wait_status(S, a, H.CKKS_RUNNING)
    time.sleep(0.05)
    b = _submit(S, ring)
    assert _wait_status(S, b, H.CKKS_RUNNING, limit=0.3)
    assert H.ckks_server_poll(S, a)[0] == H.CKKS_RUNNING
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    assert st["max_inflight"] == 2 and st["completed"] == 2
    S.close()


def test_queued_requests_join_the_next_batch():
    S, ring = _server(batch=4, inflight=1, service=0.3)
    first = _submit(S, ring)
    assert _wait_status(S, first, H.CKKS_RUNNING)
    rest = [_submit(S, ring) for _ in range(6)]
    assert all(H.ckks_server_poll(S, r)[0] == H.CKKS_PENDING for r in rest)
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    # 1 alone, then 4, then the remaining 2 (arrival order)
    assert st["batches"] == 3 and st["max_batch"] == 4 and st["completed"] == 7
    lat = [H.ckks_server_poll(S, r)[1] for r in rest]
    assert max(lat[:4]) < min(lat[4:]) + 0.3  # the first four finished one batch earlier
    assert lat[0] < lat[4]
    S.close()


def test_memory_budget_limits_what_runs_at_once():
    # Each request needs 0.6 of the budget: never two at once, whatever the
    # stream and batch limits allow.
    S, ring = _server(budget=10 * MiB, batch=8, inflight=4, service=0.05)
    ids = [_submit(S, ring, ws=6 * MiB) for _ in range(5)]
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    assert st["max_inflight"] == 1 and st["max_batch"] == 1 and st["batches"] == 5
    assert st["arena_peak"] <= 10 * MiB and st["arena_in_use"] == 0
    assert all(H.ckks_server_poll(S, r)[0] == H.CKKS_OK for r in ids)
    S.close()


def test_budget_packs_batches_up_to_the_limit():
    S, ring = _server(budget=10 * MiB, batch=8, inflight=1, service=0.2)
    first = _submit(S, ring, ws=MiB)
    assert _wait_status(S, first, H.CKKS_RUNNING)
    for _ in range(6):
        _submit(S, ring, ws=3 * MiB)
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    # arena 10 MiB: the first batch holds 1 MiB; later batches hold 3 x 3 MiB
    assert st["max_batch"] == 3 and st["batches"] == 3
    assert st["arena_peak"] <= 10 * MiB
    S.close()


def test_cancel_and_timeout():
    S, ring = _server(inflight=1, batch=1, service=0.4, timeout=0.0)
    a = _submit(S, ring)
    assert _wait_status(S, a, H.CKKS_RUNNING)
    b = _submit(S, ring)
    assert H.ckks_server_cancel(S, b) == H.CKKS_OK
    assert H.ckks_server_poll(S, b)[0] == H.CKKS_E_CANCELLED
    assert H.ckks_server_cancel(S, a) == H.CKKS_E_INVALID_ARG  # already running
    H.ckks_server_wait_all(S)
    S.close()

    S, ring = _server(inflight=1, batch=1, service=0.5, timeout=0.1)
    a = _submit(S, ring)
    assert _wait_status(S, a, H.CKKS_RUNNING)
    b = _submit(S, ring)
    assert _wait_status(S, b, H.CKKS_E_TIMEOUT, limit=2.0)
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    assert st["completed"] == 1 and st["failed"] == 1
    S.close()


def test_rings_are_batched_separately_in_arrival_order():
    S = H.Server(64 * MiB, max_batch=8, max_inflight=1, simulated=True, simulated_service_s=0.1)
    r0 = H.ckks_server_add_ring(S, None, {})
    r1 = H.ckks_server_add_ring(S, None, {})
    head = _submit(S, r0)
    assert _wait_status(S, head, H.CKKS_RUNNING)
    ids = [_submit(S, r) for r in (r1, r0, r1, r0)]
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    # head alone; then ring 1's two requests (oldest first); then ring 0's two
    assert st["batches"] == 3 and st["max_batch"] == 2
    lat = {r: H.ckks_server_poll(S, r)[1] for r in ids}
    assert abs(lat[ids[0]] - lat[ids[2]]) < 0.05 and abs(lat[ids[1]] - lat[ids[3]]) < 0.05
    assert lat[ids[0]] < lat[ids[1]]
    S.close()


def test_latency_statistics_and_invalid_arguments():
    S, ring = _server(inflight=2, batch=2, service=0.02)
    for _ in range(10):
        _submit(S, ring)
    H.ckks_server_wait_all(S)
    st = H.ckks_server_stats(S)
    assert st["completed"] == 10 and 0 < st["p50_s"] <= st["p99_s"] and st["span_s"] > 0
    assert st["p50_s"] <= st["mean_s"] * 2
    with pytest.raises(H.CkksError) as e:
        H.ckks_server_submit(S, 7, level=1, sim_ws_bytes=1)
    assert e.value.code == H.CKKS_E_INVALID_ARG
    with pytest.raises(H.CkksError):
        H.ckks_server_poll(S, 12345)
    S.close()
    with pytest.raises(H.CkksError):
        H.Server(MiB, max_batch=1, max_inflight=0, simulated=True)
