"""Bit-exact parity of each GPU step against the CPU oracle (via the C-ABI)."""
import numpy as np
import pytest

import oracle as O
import paper_2605_17222_amd as H
import workload as W
from gpu_common import gpu_params, limbs_tensor, log, random_limbs

pytestmark = pytest.mark.gpu

PARAMS = {"n12": W.params_toy(), "n16": W.params_n16(), "n14": W.params_n16(14), "n15": W.params_n16(15)}


@pytest.fixture(scope="module")
def oracles():
    return {}


def _oracle(oracles, name):
    if name not in oracles:
        o = O.Oracle(PARAMS[name])
        o.keygen(7)
        oracles[name] = o
    return oracles[name]


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["n12", "n14", "n15", "n16"])
def test_ntt_forward_inverse(oracles, name):
    prm = PARAMS[name]
    o = _oracle(oracles, name)
    P = gpu_params(prm)
    K = len(o.pq)
    log("ntt", name, "limbs", K)
    x = random_limbs(1, o.pq, o.n)
    xd = limbs_tensor(x)
    yd = H.empty((K, o.n))
    H.ckks_op_ntt(P, True, 0, K, xd, yd)
    _sync()
    ref = o.ntt(x, range(K))
    got = H.to_host(yd)
    assert np.array_equal(got, ref)
    # inverse, out of place and in place
    zd = H.empty((K, o.n))
    H.ckks_op_ntt(P, False, 0, K, yd, zd)
    H.ckks_op_ntt(P, False, 0, K, yd, yd)
    _sync()
    assert np.array_equal(H.to_host(zd), x)
    assert np.array_equal(H.to_host(yd), x)
    # a sub-range of primes
    H.ckks_op_ntt(P, True, 3, K - 3, limbs_tensor(x[3:]), zd[: K - 3])
    _sync()
    assert np.array_equal(H.to_host(zd[: K - 3]), ref[3:])


def _ws(P, level):
    import torch
    b = H.ckks_op_workspace_size(P, level)
    return torch.empty(b, dtype=torch.uint8, device="cuda"), b


@pytest.mark.parametrize("name,level", [("n12", 2), ("n12", 0), ("n16", 24), ("n16", 10), ("n16", 17)])
def test_decompose(oracles, name, level):
    o = _oracle(oracles, name)
    P = gpu_params(PARAMS[name])
    log("decompose", name, level)
    x = random_limbs(2, [o.pq[i] for i in o.q_basis(level)], o.n)
    ref = o.decompose(level, x)
    dig = H.empty(ref.shape)
    ws, wb = _ws(P, level)
    H.ckks_op_decompose(P, level, limbs_tensor(x), dig, ws, wb)
    _sync()
    assert np.array_equal(H.to_host(dig), ref)


@pytest.mark.parametrize("name,level", [("n12", 2), ("n12", 1), ("n16", 24), ("n16", 9)])
def test_moddown_and_rescale(oracles, name, level):
    o = _oracle(oracles, name)
    P = gpu_params(PARAMS[name])
    log("moddown", name, level)
    x = random_limbs(3, [o.pq[i] for i in o.pq_basis(level)], o.n)
    ws, wb = _ws(P, level)
    out = H.empty((level + 1, o.n))
    H.ckks_op_moddown(P, level, False, limbs_tensor(x), out, ws, wb)
    out2 = H.empty((level, o.n))
    H.ckks_op_moddown(P, level, True, limbs_tensor(x), out2, ws, wb)
    xq = random_limbs(4, [o.pq[i] for i in o.q_basis(level)], o.n)
    out3 = H.empty((level, o.n))
    H.ckks_op_rescale(P, level, limbs_tensor(xq), out3, ws, wb)
    _sync()
    assert np.array_equal(H.to_host(out), o.moddown(level, x))
    assert np.array_equal(H.to_host(out2), o.moddown_rescale(level, x))
    assert np.array_equal(H.to_host(out3), o.rescale(level, xq))


@pytest.mark.parametrize("name,level,rot", [("n12", 2, 1), ("n12", 1, -3), ("n16", 24, 4), ("n16", 12, 48)])
def test_keyswitch_with_automorphism(oracles, name, level, rot):
    o = _oracle(oracles, name)
    P = gpu_params(PARAMS[name])
    log("keyswitch", name, level, rot)
    K = o.K(level)
    digits = np.stack([random_limbs(10 + b, [o.pq[i] for i in o.pq_basis(level)], o.n)
                       for b in range(o.beta(level))])
    key = o.rotkey(rot)
    add = random_limbs(5, [o.pq[i] for i in o.pq_basis(level)], o.n)
    x, y = o.ks_inner(level, digits, key)
    qs = [o.pq[i] for i in range(K)]
    xa = np.stack([(x[l].astype(object) + add[l].astype(object)) % qs[l] for l in range(K)]).astype(np.uint64)
    ref_a = o.automorph_ntt(xa, rot)
    ref_b = o.automorph_ntt(y, rot)
    oa, ob = H.empty((K, o.n)), H.empty((K, o.n))
    H.ckks_op_keyswitch(P, level, limbs_tensor(digits), limbs_tensor(key), rot, limbs_tensor(add), oa, ob)
    _sync()
    assert np.array_equal(H.to_host(oa), ref_a)
    assert np.array_equal(H.to_host(ob), ref_b)


@pytest.mark.parametrize("name,rot", [("n12", 5), ("n16", 1), ("n16", -7)])
def test_automorph(oracles, name, rot):
    o = _oracle(oracles, name)
    P = gpu_params(PARAMS[name])
    log("automorph", name, rot)
    x = random_limbs(6, o.pq, o.n)
    out = H.empty(x.shape)
    H.ckks_op_automorph(P, rot, len(o.pq), limbs_tensor(x), out)
    _sync()
    assert np.array_equal(H.to_host(out), o.automorph_ntt(x, rot))


def test_psi_matches_oracle_convention(oracles):
    # Parameters created with the oracle's psi give the same NTT as the default rule.
    o = _oracle(oracles, "n12")
    prm = PARAMS["n12"]
    P2 = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum, psi=[o.psi(i) for i in range(len(o.pq))])
    x = random_limbs(8, o.pq, o.n)
    y = H.empty(x.shape)
    H.ckks_op_ntt(P2, True, 0, len(o.pq), limbs_tensor(x), y)
    _sync()
    assert np.array_equal(H.to_host(y), o.ntt(x, range(len(o.pq))))
