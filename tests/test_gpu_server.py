"""The continuous-batching server on the device: requests with different
levels, splits and diagonal counts, on rings of different N, submitted while
others run.  Each result must equal the oracle's single-LT result bit for bit,
be the same bytes as the request evaluated alone (a server that runs one
request at a time), and decrypt to M v within the stated tolerance."""
import numpy as np
import pytest

import paper_2605_17222_amd as H
import workload as W
from gpu_common import batch_case, gpu_params, limbs_tensor, log

pytestmark = pytest.mark.gpu

MiB = 1 << 20


class Ring:
    def __init__(self, prm, specs, seed):
        self.prm = prm
        self.o, self.keys, self.items, self.delta = batch_case(prm, specs, seed)
        self.P = gpu_params(prm)
        self.dkeys = {r: limbs_tensor(k) for r, k in self.keys.items()}
        self.dev = []
        for it in self.items:
            c0, c1 = limbs_tensor(it["ct"][0]), limbs_tensor(it["ct"][1])
            pts = [None if f is None else limbs_tensor(f) for f in it["pts"]]
            self.dev.append((c0, c1, pts))


def _serve(rings, order, budget, max_batch, max_inflight, gap_s=0.0):
    """Submits (ring index, item index) in `order`; returns outputs by key."""
    import time

    import torch
    torch.cuda.synchronize()  # inputs complete before submission
    outs, ids = {}, {}
    with H.Server(budget, max_batch=max_batch, max_inflight=max_inflight) as S:
        rid = [H.ckks_server_add_ring(S, R.P, R.dkeys) for R in rings]
        for g, t in order:
            R = rings[g]
            it = R.items[t]
            c0, c1, pts = R.dev[t]
            o0, o1 = H.empty((it["level"], R.prm.n)), H.empty((it["level"], R.prm.n))
            torch.cuda.synchronize()
            ids[g, t] = H.ckks_server_submit(S, rid[g], it["level"], R.delta, c0, c1, it["split"], pts, R.delta,
                                             o0, o1)
            outs[g, t] = (o0, o1)
            if gap_s:
                time.sleep(gap_s)
        H.ckks_server_wait_all(S)
        st = H.ckks_server_stats(S)
        res = {}
        for key, rq in ids.items():
            status, lat = H.ckks_server_poll(S, rq)
            assert status == H.CKKS_OK, (key, H.strerror(status))
            lvl, scale = H.ckks_server_result(S, rq)
            o0, o1 = outs[key]
            res[key] = (np.stack([H.to_host(o0), H.to_host(o1)]), lvl, scale)
    return res, st


def _check(rings, res, tol):
    for (g, t), (got, lvl, scale) in res.items():
        R = rings[g]
        it = R.items[t]
        ref = R.o.lt_th(it["level"], it["ct"], it["split"], it["pts"], R.keys)
        assert np.array_equal(got, ref), (g, t)
        assert lvl == it["level"] - 1
        z = R.o.decrypt_slots(got, scale)
        assert np.abs(z - W.matvec(it["diags"], it["v"])).max() <= tol


def test_server_toy_mix_equals_alone_and_oracle():
    prm = W.params_toy()
    specs = [(2, 16, (2, 2, 4)), (1, 16, (2, 2, 4)), (2, 8, (2, 2, 2)), (1, 5, (1, 4, 2)), (2, 12, (4, 1, 4)),
             (2, 1, (2, 2, 1)), (2, 16, (4, 2, 2)), (1, 9, (2, 2, 4))]
    R = Ring(prm, specs, 21)
    order = [(0, t) for t in range(len(specs))]
    log("toy server mix")
    mix, st = _serve([R], order, 64 * MiB, max_batch=3, max_inflight=2)
    assert st["completed"] == len(specs) and st["batches"] >= 3
    _check([R], mix, 5e-3)
    log("toy server alone")
    alone, st1 = _serve([R], order[::-1], 64 * MiB, max_batch=1, max_inflight=1)
    assert st1["max_batch"] == 1
    for key in mix:
        assert np.array_equal(mix[key][0], alone[key][0])


def test_server_two_rings_n15_n16():
    # Resident key sets for two ring sizes; requests of both interleaved and
    # submitted while earlier ones run.
    log("building the N=2^15 and N=2^16 server rings")
    r15 = Ring(W.params_n16(log_n=15), [(12, 32, (2, 4, 4)), (24, 16, (2, 2, 4)), (9, 32, (2, 4, 4))], 31)
    r16 = Ring(W.params_n16(), [(24, 32, (2, 4, 4)), (8, 16, (2, 2, 4)), (17, 32, (2, 4, 4))], 32)
    order = [(1, 0), (0, 0), (1, 1), (0, 1), (1, 2), (0, 2)]
    log("n15/n16 server mix")
    mix, st = _serve([r15, r16], order, 4 << 30, max_batch=2, max_inflight=2, gap_s=0.002)
    assert st["completed"] == 6
    _check([r15, r16], mix, 1e-4)
    log("n15/n16 server alone")
    alone, _ = _serve([r15, r16], order, 4 << 30, max_batch=1, max_inflight=1)
    for key in mix:
        assert np.array_equal(mix[key][0], alone[key][0])


def test_server_serving_split_n14():
    # The serving benchmark's resident split (4, 16, 4) with up to 256
    # diagonals, N = 2^14, requests of different levels and diagonal counts.
    r14 = Ring(W.params_n16(log_n=14), [(24, 256, (4, 16, 4)), (8, 40, (4, 16, 4)), (15, 200, (4, 16, 4))], 41)
    order = [(0, 0), (0, 1), (0, 2)]
    log("n14 serving split")
    mix, st = _serve([r14], order, 8 << 30, max_batch=4, max_inflight=2)
    assert st["completed"] == 3
    _check([r14], mix, 1e-4)


def test_server_request_missing_key_fails_alone():
    # The ring lacks rotation 8, which only the (2, 2, 4) request needs.  The
    # requests behind the first queue while it runs, so the bad one is
    # batched with good ones: it alone fails, the others are bit-exact.
    import torch
    prm = W.params_toy()
    specs = [(2, 8, (1, 4, 2)), (2, 16, (2, 2, 4)), (2, 8, (1, 4, 2)), (2, 6, (1, 4, 2))]
    R = Ring(prm, specs, 51)
    short = {r: k for r, k in R.dkeys.items() if r != 8}
    assert len(short) == len(R.dkeys) - 1
    torch.cuda.synchronize()
    outs, ids = [], []
    with H.Server(64 * MiB, max_batch=4, max_inflight=1) as S:
        ring = H.ckks_server_add_ring(S, R.P, short)
        for t, it in enumerate(R.items):
            c0, c1, pts = R.dev[t]
            o0, o1 = H.empty((2, prm.n)), H.empty((2, prm.n))
            outs.append((o0, o1))
            ids.append(H.ckks_server_submit(S, ring, 2, R.delta, c0, c1, it["split"], pts, R.delta, o0, o1))
        H.ckks_server_wait_all(S)
        sts = [H.ckks_server_poll(S, i)[0] for i in ids]
    assert sts[1] == H.CKKS_E_UNSUPPORTED
    for t in (0, 2, 3):
        assert sts[t] == H.CKKS_OK, t
        it = R.items[t]
        ref = R.o.lt_th(2, it["ct"], it["split"], it["pts"], R.keys)
        assert np.array_equal(np.stack([H.to_host(outs[t][0]), H.to_host(outs[t][1])]), ref), t
