"""Edge cases of the LT on the device, bit-exact against the oracle: no
diagonal at all, one diagonal, every diagonal of the matrix (n = S), the
lowest level, a ragged last giant block, an all-absent outer block, and ring
sizes between the toy and the N = 2^16 configurations."""
import numpy as np
import pytest

import oracle as O
import paper_2605_17222_amd as H
import workload as W
from gpu_common import gpu_params, limbs_tensor, log

pytestmark = pytest.mark.gpu

ALGO = {"th": H.CKKS_LT_TH_BSGS, "bsgs": H.CKKS_LT_BSGS, "naive": H.CKKS_LT_NAIVE}


class Ring:
    def __init__(self, prm, seed):
        self.prm = prm
        self.o = O.Oracle(prm)
        self.o.keygen(seed)
        self.delta = 2.0 ** prm.log_delta
        self.seed = seed
        self._keys = {}

    def keys(self, rots):
        need = [r for r in rots if r not in self._keys]
        self._keys.update(self.o.rotkeys(need) if need else {})
        return {r: self._keys[r] for r in rots}

    def case(self, level, offsets, algo, split, tol):
        prm, o = self.prm, self.o
        S = prm.slots
        diags = W.banded_diagonals(self.seed + len(offsets), S, offsets)
        v = W.input_vector(self.seed + level, S)
        ct = o.encrypt(level, v, self.delta, seed=self.seed + 7)
        if algo == "th":
            rots = W.th_rotations(*split)
            pts = o.th_plaintexts(diags, *split, self.delta) if diags else [None] * (split[0] * split[1] * split[2])
        elif algo == "bsgs":
            rots = W.bsgs_rotations(*split)
            pts = o.bsgs_plaintexts(diags, *split, self.delta) if diags else [None] * (split[0] * split[1])
        else:
            rots = sorted(d for d in diags if d)
            pts = o.naive_plaintexts(diags, self.delta) if diags else []
        keys = self.keys(rots)
        if algo == "th":
            ref = o.lt_th(level, ct, split, pts, keys)
        elif algo == "bsgs":
            ref = o.lt_bsgs(level, ct, split, pts, keys)
        else:
            ref = o.lt_naive(level, ct, pts, keys)
        got, lvl, scale = self.gpu(level, ct, split, pts, keys, algo)
        assert lvl == level - 1
        assert np.array_equal(got, ref)
        z = o.decrypt_slots(got, scale)
        assert np.abs(z - W.matvec(diags, v)).max() <= tol
        return got

    def gpu(self, level, ct, split, pts, keys, algo):
        import torch
        P = gpu_params(self.prm)
        dpts = [None if f is None else limbs_tensor(f) for f in pts]
        dkeys = {r: limbs_tensor(k) for r, k in keys.items()}
        c0, c1 = limbs_tensor(ct[0]), limbs_tensor(ct[1])
        wsb = H.ckks_lt_workspace_size(P, level, split, dpts, ALGO[algo])
        ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
        o0, o1 = H.empty((level, self.prm.n)), H.empty((level, self.prm.n))
        lvl, sc = H.ckks_lt_eval(P, level, self.delta, c0, c1, split, dpts, self.delta, dkeys, ALGO[algo], o0, o1,
                                 ws, wsb)
        torch.cuda.synchronize()
        return np.stack([H.to_host(o0), H.to_host(o1)]), lvl, sc


@pytest.fixture(scope="module")
def toy():
    return Ring(W.params_toy(), 401)


@pytest.mark.parametrize("algo,split", [("th", (2, 2, 4)), ("bsgs", (4, 4)), ("naive", (1, 1, 1))])
def test_no_diagonal_gives_zero(toy, algo, split):
    log("empty matrix", algo)
    got = toy.case(2, [], algo, split, 5e-3)
    assert not got.any()  # Decompose/ModDown of zero is zero: an all-zero ciphertext


@pytest.mark.parametrize("offset", [0, 1, 2047])
def test_single_diagonal(toy, offset):
    log("single diagonal", offset)
    toy.case(2, [offset], "th", (4, 8, 64), 5e-3)


def test_every_diagonal_of_the_matrix(toy):
    # n = S = 2048 diagonals: a dense 2048 x 2048 matrix, split (16, 8, 16)
    log("dense toy matrix")
    toy.case(2, list(range(2048)), "th", (16, 8, 16), 5e-3)


@pytest.mark.parametrize("algo,split", [("th", (4, 4, 4)), ("bsgs", (8, 8))])
def test_ragged_last_block_and_absent_block(toy, algo, split):
    # 61 diagonals: the last giant block is ragged; offsets 16..31 absent
    offs = [d for d in range(61) if not 16 <= d < 32]
    log("ragged", algo)
    toy.case(2, offs, algo, split, 5e-3)


def test_lowest_level_toy(toy):
    toy.case(1, list(range(16)), "th", (2, 2, 4), 5e-3)


@pytest.mark.parametrize("log_n,level,nd,split", [(13, 5, 32, (2, 4, 4)), (14, 9, 48, (4, 4, 4)),
                                                 (16, 1, 16, (2, 2, 4))])
def test_other_ring_sizes_and_levels(log_n, level, nd, split):
    log("ring", log_n, "level", level)
    r = Ring(W.params_n16(log_n=log_n), 500 + log_n)
    r.case(level, list(range(nd)), "th", split, 1e-4)
