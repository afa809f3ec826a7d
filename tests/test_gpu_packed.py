"""Packed resident operands (ckks_pack): keys and TH-BSGS plaintexts whose
limbs of primes below 2^40 are stored as a 32-bit and an 8-bit plane.  The
packed bytes must follow the documented layout exactly, and every LT must be
bit-identical with packed and unpacked operands (and so equal the oracle)."""
import numpy as np
import pytest

import paper_2605_17222_amd as H
import workload as W
from gpu_common import LTCase, gpu_params, limbs_tensor, log

pytestmark = pytest.mark.gpu


def _layout(prm, polys):
    """The packed bytes of [count][kmax][N] words, built independently."""
    primes = list(prm.p) + list(prm.q)
    out = []
    for poly in polys.reshape(-1, len(primes), prm.n):
        for q, limb in zip(primes, poly):
            if q < 2 ** 40:
                # runs of 256: the run's 32-bit low words, then its high bytes
                lo = (limb & 0xFFFFFFFF).astype("<u4").view(np.uint8).reshape(-1, 1024)
                hi = (limb >> 32).astype(np.uint8).reshape(-1, 256)
                out.append(np.concatenate([lo, hi], axis=1).ravel())
            else:
                out.append(limb.astype("<u8").view(np.uint8))
    return np.concatenate(out)


@pytest.fixture(scope="module", params=["toy", "n16"])
def case(request):
    w = W.workload_toy() if request.param == "toy" else W.workload_n16()
    return LTCase(w, algos=("th", "bsgs"))


def _run(c, algo, packed_keys, packed_pts, level=None):
    import torch
    w = c.w
    prm = w.params
    P = gpu_params(prm)
    level = w.level if level is None else level
    d = c.device()
    keys = d["keys"]
    if packed_keys:
        keys = {r: H.ckks_pack(P, k) for r, k in keys.items()}
    pts = d["pts"]["th" if algo in ("th", "dh") else "bsgs"]
    if packed_pts:
        pts = [None if f is None else H.ckks_pack(P, f) for f in pts]
    code = {"th": H.CKKS_LT_TH_BSGS, "dh": H.CKKS_LT_DH_BSGS, "bsgs": H.CKKS_LT_BSGS}[algo]
    split = {"th": w.th_split, "dh": (w.th_split[0] * w.th_split[1], w.th_split[2]), "bsgs": w.bsgs_split}[algo]
    if algo == "dh":
        # DH (n1 n2, n3) covers the same diagonals as TH (n1, n2, n3) and
        # takes the TH plaintexts of the split (1, n1 n2, n3)
        split3 = (1,) + split
        pts_np = c.o.th_plaintexts(w.diags, *split3, c.delta)
        pts = [None if f is None else limbs_tensor(f) for f in pts_np]
        if packed_pts:
            pts = [None if f is None else H.ckks_pack(P, f) for f in pts]
        keys = {r: keys[r] if r in keys else None for r in W.th_rotations(*split3)}
        if any(v is None for v in keys.values()):
            missing = [r for r, v in keys.items() if v is None]
            extra = c.o.rotkeys(missing)
            for r in missing:
                t = limbs_tensor(extra[r])
                keys[r] = H.ckks_pack(P, t) if packed_keys else t
    wsb = H.ckks_lt_workspace_size(P, level, split, pts, code)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
    o0, o1 = H.empty((level, prm.n)), H.empty((level, prm.n))
    H.ckks_lt_eval(P, level, c.delta, d["ct"][0], d["ct"][1], split, pts, c.delta, keys, code, o0, o1, ws, wsb)
    torch.cuda.synchronize()
    return np.stack([H.to_host(o0), H.to_host(o1)])


def test_packed_layout(case):
    import torch
    prm = case.w.params
    P = gpu_params(prm)
    r = sorted(case.keys)[0]
    key = case.keys[r]
    packed = H.ckks_pack(P, limbs_tensor(key))
    torch.cuda.synchronize()
    got = packed.t.cpu().numpy()
    assert H.ckks_packed_poly_bytes(P) * key.size // ((prm.alpha + prm.max_level + 1) * prm.n) == got.size
    assert np.array_equal(got, _layout(prm, key))


@pytest.mark.parametrize("algo", ["th", "dh", "bsgs"])
def test_packed_equals_unpacked(case, algo):
    log("packed", case.w.params.log_n, algo)
    ref = _run(case, algo, False, False)
    if algo == "th":
        assert np.array_equal(ref, case.oracle_out("th"))
    assert np.array_equal(_run(case, algo, True, False), ref)
    if algo != "bsgs":
        assert np.array_equal(_run(case, algo, False, True), ref)
        assert np.array_equal(_run(case, algo, True, True), ref)


def test_packed_lower_level(case):
    # a lower level reads a prefix of every packed limb table
    level = max(1, case.w.level - 1)
    assert np.array_equal(_run(case, "th", True, True, level), _run(case, "th", False, False, level))


def test_packed_errors(case):
    import torch
    prm = case.w.params
    P = gpu_params(prm)
    d = case.device()
    # packed plaintexts are PQ-basis (TH-/DH-BSGS) only
    th_pts = [H.ckks_pack(P, f) for f in d["pts"]["th"] if f is not None][:2]
    with pytest.raises(H.CkksError) as e:
        H.ckks_lt_workspace_size(P, case.w.level, case.w.bsgs_split, th_pts, H.CKKS_LT_BSGS)
    assert e.value.code == H.CKKS_E_UNSUPPORTED
    with pytest.raises(ValueError):
        H.ckks_lt_workspace_size(P, case.w.level, case.w.th_split, th_pts + [d["pts"]["th"][2]], H.CKKS_LT_TH_BSGS)
    torch.cuda.synchronize()


def test_packed_batch_and_server(case):
    # packed keys and plaintexts through a batch (packed and unpacked items
    # mixed, so packed and unpacked keys meet in the same phase) and through
    # the server (a ring registered with packed keys): every result equals the
    # single unpacked evaluation
    import torch
    w = case.w
    prm = w.params
    P = gpu_params(prm)
    d = case.device()
    ref = _run(case, "th", False, False)
    keys_p = {r: H.ckks_pack(P, k) for r, k in d["keys"].items()}
    pts_p = [None if f is None else H.ckks_pack(P, f) for f in d["pts"]["th"]]
    c0, c1 = d["ct"]
    forms = [(pts_p, keys_p), (d["pts"]["th"], d["keys"]), (pts_p, keys_p), (d["pts"]["th"], keys_p)]
    items = [H.BatchItem(w.level, case.delta, c0, c1, w.th_split, pts, case.delta, keys,
                         H.empty((w.level, prm.n)), H.empty((w.level, prm.n))) for pts, keys in forms]
    wsb = H.ckks_lt_batch_workspace_size(P, items, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
    log("mixed packed/unpacked batch of 4, workspace", wsb)
    assert H.ckks_lt_eval_batch(P, items, H.CKKS_LT_TH_BSGS, ws, wsb) == H.CKKS_OK
    torch.cuda.synchronize()
    for it in items:
        assert it.status == H.CKKS_OK
        assert np.array_equal(np.stack([H.to_host(it.out0), H.to_host(it.out1)]), ref)
    del ws
    outs, ids = [], []
    with H.Server(8 << 30, max_batch=4, max_inflight=2) as S:
        ring = H.ckks_server_add_ring(S, P, keys_p)
        for _ in range(4):
            o0, o1 = H.empty((w.level, prm.n)), H.empty((w.level, prm.n))
            ids.append(H.ckks_server_submit(S, ring, w.level, case.delta, c0, c1, w.th_split, pts_p, case.delta,
                                            o0, o1))
            outs.append((o0, o1))
        H.ckks_server_wait_all(S)
        for i in ids:
            status, _ = H.ckks_server_poll(S, i)
            assert status == H.CKKS_OK, H.strerror(status)
    for o0, o1 in outs:
        assert np.array_equal(np.stack([H.to_host(o0), H.to_host(o1)]), ref)
