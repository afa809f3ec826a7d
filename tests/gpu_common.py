"""Shared fixtures for the GPU parity tests (inputs come from the oracle)."""
from __future__ import annotations

import functools
import sys

import numpy as np

import oracle as O
import paper_2605_17222_amd as H
import workload as W


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def gpu_params(params: W.Params) -> H.Params:
    return H.ckks_params_create(params.log_n, params.q, params.p, params.dnum)


def limbs_tensor(a: np.ndarray):
    return H.to_device(np.ascontiguousarray(a, dtype=np.uint64))


def random_limbs(seed: int, moduli, n: int) -> np.ndarray:
    return W.uniform_residues(seed, moduli, n)


def batch_case(prm: W.Params, specs, seed: int):
    """Oracle keys, ciphertexts and TH plaintexts for several LTs sharing one
    key set.  specs: (level, n_diag, split) per item; banded diagonals
    0 .. n_diag-1.  Returns (oracle, keys, items, delta)."""
    o = O.Oracle(prm)
    o.keygen(seed)
    delta = 2.0 ** prm.log_delta
    S = prm.slots
    rots = set()
    for level, nd, split in specs:
        rots |= set(W.th_rotations(*split))
    keys = o.rotkeys(sorted(rots))
    items = []
    for t, (level, nd, split) in enumerate(specs):
        diags = W.banded_diagonals(seed * 100 + t, S, range(nd))
        v = W.input_vector(seed * 100 + t, S)
        ct = o.encrypt(level, v, delta, seed=seed * 100 + t)
        pts = o.th_plaintexts(diags, *split, delta)
        items.append(dict(level=level, split=split, diags=diags, v=v, ct=ct, pts=pts))
    return o, keys, items, delta


class LTCase:
    """Keys, plaintexts and a ciphertext for one workload, made by the oracle."""

    def __init__(self, w: W.LTWorkload, key_seed: int = 11, enc_seed: int = 5, algos=("th", "bsgs")):
        self.w = w
        p = w.params
        self.o = O.Oracle(p)
        self.o.keygen(key_seed)
        self.delta = 2.0 ** p.log_delta
        self.ct = self.o.encrypt(w.level, w.vector, self.delta, seed=enc_seed)
        rots = set()
        if "th" in algos:
            rots |= set(W.th_rotations(*w.th_split))
        if "bsgs" in algos:
            rots |= set(W.bsgs_rotations(*w.bsgs_split))
        if "naive" in algos:
            rots |= set(d for d in w.diags if d)
        self.keys = self.o.rotkeys(sorted(rots))
        self.pts = {}
        if "th" in algos:
            self.pts["th"] = self.o.th_plaintexts(w.diags, *w.th_split, self.delta)
        if "bsgs" in algos:
            self.pts["bsgs"] = self.o.bsgs_plaintexts(w.diags, *w.bsgs_split, self.delta)
        if "naive" in algos:
            self.pts["naive"] = self.o.naive_plaintexts(w.diags, self.delta)
        self.ref = W.matvec(w.diags, w.vector)
        self._dev = None

    def oracle_out(self, algo: str) -> np.ndarray:
        w = self.w
        if algo == "th":
            return self.o.lt_th(w.level, self.ct, w.th_split, self.pts["th"], self.keys)
        if algo == "bsgs":
            return self.o.lt_bsgs(w.level, self.ct, w.bsgs_split, self.pts["bsgs"], self.keys)
        return self.o.lt_naive(w.level, self.ct, self.pts["naive"], self.keys)

    def device(self):
        if self._dev is None:
            self._dev = {
                "ct": [limbs_tensor(self.ct[0]), limbs_tensor(self.ct[1])],
                "keys": {r: limbs_tensor(k) for r, k in self.keys.items()},
                "pts": {a: [None if f is None else limbs_tensor(f) for f in v] for a, v in self.pts.items()},
            }
        return self._dev

    def gpu_out(self, algo: str, level: int = None):
        import torch
        w = self.w
        P = gpu_params(w.params)
        level = w.level if level is None else level
        d = self.device()
        code = {"th": H.CKKS_LT_TH_BSGS, "bsgs": H.CKKS_LT_BSGS, "naive": H.CKKS_LT_NAIVE}[algo]
        split = {"th": w.th_split, "bsgs": w.bsgs_split, "naive": (1, 1, 1)}[algo]
        pts = d["pts"][algo]
        ws_bytes = H.ckks_lt_workspace_size(P, level, split, pts, code)
        ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device="cuda")
        n = w.params.n
        out0 = H.empty((level, n))
        out1 = H.empty((level, n))
        lvl, scale = H.ckks_lt_eval(P, level, self.delta, d["ct"][0], d["ct"][1], split, pts, self.delta,
                                    d["keys"], code, out0, out1, ws, ws_bytes)
        torch.cuda.synchronize()
        return np.stack([H.to_host(out0), H.to_host(out1)]), lvl, scale

    def decode(self, out: np.ndarray, scale: float) -> np.ndarray:
        return self.o.decrypt_slots(out, scale)
