"""End-to-end GPU LT parity: GPU ciphertext limbs equal the oracle's bit for bit
on the same seeded keys, plaintexts and ciphertext; decryptions meet the
stated accuracy (<= 5e-3 at Delta = 2^30, <= 1e-4 at Delta = 2^40)."""
import numpy as np
import pytest

import paper_2605_17222_amd as H
import workload as W
from gpu_common import LTCase, gpu_params, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def toy():
    return LTCase(W.workload_toy(), algos=("th", "bsgs", "naive"))


@pytest.fixture(scope="module")
def n16():
    log("building the N=2^16 oracle case (keys, plaintexts)")
    return LTCase(W.workload_n16())


@pytest.mark.parametrize("algo", ["th", "bsgs", "naive"])
def test_lt_toy_bit_exact(toy, algo):
    log("toy", algo)
    got, lvl, scale = toy.gpu_out(algo)
    ref = toy.oracle_out(algo)
    assert lvl == toy.w.level - 1
    assert np.array_equal(got, ref)
    z = toy.decode(got, scale)
    assert np.abs(z - toy.ref).max() <= 5e-3


def test_lt_toy_repeatable(toy):
    a, _, _ = toy.gpu_out("th")
    b, _, _ = toy.gpu_out("th")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("algo", ["th", "bsgs"])
def test_lt_n16_bit_exact(n16, algo):
    log("n16", algo)
    got, lvl, scale = n16.gpu_out(algo)
    ref = n16.oracle_out(algo)
    assert np.array_equal(got, ref)
    z = n16.decode(got, scale)
    assert np.abs(z - n16.ref).max() <= 1e-4


def test_lt_errors(toy):
    import torch
    w = toy.w
    P = gpu_params(w.params)
    d = toy.device()
    pts = d["pts"]["th"]
    n = w.params.n
    ws_bytes = H.ckks_lt_workspace_size(P, w.level, w.th_split, pts, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    o0, o1 = H.empty((w.level, n)), H.empty((w.level, n))
    args = (P, w.level, toy.delta, d["ct"][0], d["ct"][1], w.th_split, pts, toy.delta)
    # missing key
    keys = dict(d["keys"])
    keys.pop(1)
    with pytest.raises(H.CkksError) as e:
        H.ckks_lt_eval(*args, keys, H.CKKS_LT_TH_BSGS, o0, o1, ws, ws_bytes)
    assert e.value.code == H.CKKS_E_UNSUPPORTED
    # workspace too small
    with pytest.raises(H.CkksError) as e:
        H.ckks_lt_eval(*args, d["keys"], H.CKKS_LT_TH_BSGS, o0, o1, ws, ws_bytes - 1)
    assert e.value.code == H.CKKS_E_WORKSPACE
    # output aliasing the input
    with pytest.raises(H.CkksError) as e:
        H.ckks_lt_eval(*args, d["keys"], H.CKKS_LT_TH_BSGS, d["ct"][0], o1, ws, ws_bytes)
    assert e.value.code == H.CKKS_E_INVALID_ARG
    # more diagonals than the split holds
    with pytest.raises(H.CkksError) as e:
        H.ckks_lt_eval(P, w.level, toy.delta, d["ct"][0], d["ct"][1], (2, 2, 2), pts, toy.delta, d["keys"],
                       H.CKKS_LT_TH_BSGS, o0, o1, ws, ws_bytes)
    assert e.value.code == H.CKKS_E_INVALID_ARG


@pytest.mark.parametrize("split", [(4, 4), (2, 8), (8, 2)])
def test_dh_bsgs_equals_algorithm1_oracle(toy, split):
    # CKKS_LT_DH_BSGS (n1, n2) against the oracle's own Algorithm 1, bit for bit.
    import torch
    w = toy.w
    o = toy.o
    pts = o.dh_plaintexts(w.diags, *split, toy.delta)
    keys = {r: k for r, k in toy.keys.items()}
    need = set(W.th_rotations(1, *split))
    for r in need - set(keys):
        keys[r] = o.rotkey(r)
    ref = o.lt_dh(w.level, toy.ct, split, pts, keys)
    P = gpu_params(w.params)
    d = toy.device()
    dpts = [None if f is None else H.to_device(f) for f in pts]
    dkeys = {r: H.to_device(k) for r, k in keys.items()}
    wsb = H.ckks_lt_workspace_size(P, w.level, split, dpts, H.CKKS_LT_DH_BSGS)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    o0, o1 = H.empty((w.level, w.params.n)), H.empty((w.level, w.params.n))
    H.ckks_lt_eval(P, w.level, toy.delta, d["ct"][0], d["ct"][1], split, dpts, toy.delta, dkeys,
                   H.CKKS_LT_DH_BSGS, o0, o1, ws, wsb)
    torch.cuda.synchronize()
    assert np.array_equal(np.stack([H.to_host(o0), H.to_host(o1)]), ref)
