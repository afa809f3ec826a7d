"""A ragged batch captured into a HIP graph (the library only enqueues
kernels on the caller's stream: no allocation, copy or memset) and replayed
several times, with eager device work and synchronisation between replays:
every replay must reproduce the eager result bit for bit."""
import numpy as np
import pytest

import paper_2605_17222_amd as H
import workload as W
from gpu_common import batch_case, gpu_params, limbs_tensor, log

pytestmark = pytest.mark.gpu


def test_batch_graph_replays_match_eager():
    import torch
    prm = W.params_toy()
    specs = [(2, 16, (2, 2, 4)), (1, 12, (4, 1, 4)), (2, 5, (1, 4, 2))]
    o, keys, items, delta = batch_case(prm, specs, 13)
    P = gpu_params(prm)
    dkeys = {r: limbs_tensor(k) for r, k in keys.items()}
    batch, keep = [], []
    for it in items:
        c0, c1 = limbs_tensor(it["ct"][0]), limbs_tensor(it["ct"][1])
        pts = [None if f is None else limbs_tensor(f) for f in it["pts"]]
        keep += [c0, c1, pts]
        batch.append(H.BatchItem(it["level"], delta, c0, c1, it["split"], pts, delta, dkeys,
                                 H.empty((it["level"], prm.n)), H.empty((it["level"], prm.n))))
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def outputs():
        return [np.stack([H.to_host(b.out0), H.to_host(b.out1)]) for b in batch]

    log("eager batch")
    assert H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb) == H.CKKS_OK
    torch.cuda.synchronize()
    eager = outputs()
    for it, e in zip(items, eager):
        assert np.array_equal(e, o.lt_th(it["level"], it["ct"], it["split"], it["pts"], keys))

    log("capture")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            code = H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb, torch.cuda.current_stream())
    assert code == H.CKKS_OK
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        log("replay", rep)
        for b in batch:  # clobber the outputs with eager work first
            b.out0.fill_(7)
            b.out1.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = outputs()
        for e, x in zip(eager, got):
            assert np.array_equal(e, x), rep
