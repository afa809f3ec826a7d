"""Full-size properties in the launch configurations the benchmark times.

The oracle cannot evaluate 32 ragged LTs at N = 2^16 (or a serving burst) in
a test, so these check a property that holds at any size: batching and
serving do not change results.  Inputs are uniform residues drawn on the
device, as in the benchmark (every value is a valid input of the exact
arithmetic; bit-exactness against the oracle on real keys and ciphertexts is
checked by the other GPU tests).  Sampled items of a 32-item ragged batch
(autotuned splits, shared keys) must equal their evaluation alone byte for
byte; so must 16 requests of the serving stream (three ring sizes, resident
split (4,16,4), resident plaintext pools) submitted as one burst."""
import numpy as np
import pytest

import bench as B
import paper_2605_17222_amd as H
import workload as W
from gpu_common import gpu_params, log

pytestmark = pytest.mark.gpu


def _alone(P, it, torch):
    ws_bytes = H.ckks_lt_workspace_size(P, it.level, it.split, it.pts, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device="cuda")
    o0, o1 = H.empty((it.level, it.out0.shape[1])), H.empty((it.level, it.out0.shape[1]))
    H.ckks_lt_eval(P, it.level, it.scale, it.c0, it.c1, it.split, it.pts, it.pt_scale, it.keys,
                   H.CKKS_LT_TH_BSGS, o0, o1, ws, ws_bytes)
    torch.cuda.synchronize()
    return H.to_host(o0), H.to_host(o1)


def test_ragged_batch_of_32_equals_alone():
    import torch
    prm = W.params_n16()
    P = gpu_params(prm)
    specs = B.ragged_specs(prm, 32, H)
    log("ragged specs", specs)
    residues = B.residue_maker(prm.n, torch, 77)
    pq = list(prm.p) + list(prm.q)
    keys = B.device_keys(prm, sorted(set().union(*[W.th_rotations(*sp) for _, _, sp in specs])), residues)
    delta = 2.0 ** prm.log_delta
    batch = []
    for level, nd, sp in specs:
        K = prm.alpha + level + 1
        qm = [prm.q[j] for j in range(level + 1)]
        pts = [residues(pq[:K]) for _ in range(nd)]
        batch.append(H.BatchItem(level, delta, residues(qm), residues(qm), sp, pts, delta, keys,
                                 H.empty((level, prm.n)), H.empty((level, prm.n))))
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    log("batch of 32, workspace", wsb)
    assert H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb) == H.CKKS_OK
    torch.cuda.synchronize()
    del ws
    for t in np.random.Generator(np.random.PCG64(78)).choice(32, size=8, replace=False):
        it = batch[int(t)]
        assert it.status == H.CKKS_OK
        log("item", int(t), specs[int(t)])
        a0, a1 = _alone(P, it, torch)
        assert np.array_equal(a0, H.to_host(it.out0)) and np.array_equal(a1, H.to_host(it.out1))


def test_serving_burst_of_16_equals_alone():
    import torch
    split = B.SERVING_SPLIT
    rings = []
    for log_n in (14, 15, 16):
        prm = W.params_n16(log_n=log_n)
        P = gpu_params(prm)
        residues = B.residue_maker(prm.n, torch, 2024 + log_n)
        pq = list(prm.p) + list(prm.q)
        kmax = prm.alpha + prm.max_level + 1
        keys = B.device_keys(prm, W.th_rotations(*split), residues)
        pool = [residues(pq[:kmax]) for _ in range(256)]
        cts = [(residues(list(prm.q)), residues(list(prm.q))) for _ in range(4)]
        rings.append((prm, P, keys, pool, cts))
    reqs = B.serving_requests(10.0, 200.0)[:16]
    log("requests", [(g, level, nd) for _, g, level, nd, _ in reqs])
    outs = []
    torch.cuda.synchronize()
    with H.Server(64 << 30, max_batch=8, max_inflight=2) as S:
        rid = [H.ckks_server_add_ring(S, r[1], r[2]) for r in rings]
        ids = []
        for _, g, level, nd, ci in reqs:
            prm, P, keys, pool, cts = rings[g]
            o0, o1 = H.empty((level, prm.n)), H.empty((level, prm.n))
            delta = 2.0 ** prm.log_delta
            ids.append(H.ckks_server_submit(S, rid[g], level, delta, cts[ci][0], cts[ci][1], split, pool[:nd], delta,
                                            o0, o1))
            outs.append((o0, o1))
        H.ckks_server_wait_all(S)
        st = H.ckks_server_stats(S)
        for i in ids:
            status, _ = H.ckks_server_poll(S, i)
            assert status == H.CKKS_OK, H.strerror(status)
    log("server stats", st)
    assert st["completed"] == 16
    for (_, g, level, nd, ci), (o0, o1) in zip(reqs, outs):
        prm, P, keys, pool, cts = rings[g]
        delta = 2.0 ** prm.log_delta
        it = H.BatchItem(level, delta, cts[ci][0], cts[ci][1], split, pool[:nd], delta, keys, o0, o1)
        a0, a1 = _alone(P, it, torch)
        assert np.array_equal(a0, H.to_host(o0)) and np.array_equal(a1, H.to_host(o1)), (g, level, nd)


def test_ragged_batch_of_128_in_one_graph_equals_alone():
    # The batched benchmark's step: all 128 ragged items in one
    # ckks_lt_eval_batch call, captured once into a HIP graph.  Every replay
    # (outputs cleared eagerly in between) must give each sampled item the
    # bytes of its evaluation alone.
    import torch
    prm = W.params_n16()
    P = gpu_params(prm)
    specs = B.ragged_specs(prm, 128, H)
    residues = B.residue_maker(prm.n, torch, 77)
    pq = list(prm.p) + list(prm.q)
    keys = B.device_keys(prm, sorted(set().union(*[W.th_rotations(*sp) for _, _, sp in specs])), residues)
    delta = 2.0 ** prm.log_delta
    batch = []
    for level, nd, sp in specs:
        K = prm.alpha + level + 1
        qm = [prm.q[j] for j in range(level + 1)]
        pts = [residues(pq[:K]) for _ in range(nd)]
        batch.append(H.BatchItem(level, delta, residues(qm), residues(qm), sp, pts, delta, keys,
                                 H.empty((level, prm.n)), H.empty((level, prm.n))))
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    log("batch of 128, workspace", wsb)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            code = H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb, torch.cuda.current_stream())
    assert code == H.CKKS_OK, H.strerror(code)
    torch.cuda.synchronize()
    sample = [int(t) for t in np.random.Generator(np.random.PCG64(79)).choice(128, size=6, replace=False)]
    ref = {}
    for rep in range(3):
        for it in batch:
            it.out0.zero_()
            it.out1.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        log("replay", rep)
        for t in sample:
            it = batch[t]
            assert it.status == H.CKKS_OK
            got = (H.to_host(it.out0), H.to_host(it.out1))
            if t not in ref:
                ref[t] = _alone(P, it, torch)
            assert np.array_equal(got[0], ref[t][0]) and np.array_equal(got[1], ref[t][1]), (rep, t, specs[t])
    del g, ws
    torch.cuda.empty_cache()
