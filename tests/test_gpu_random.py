"""Seeded random LT configurations at the toy size, bit-exact against the
oracle: algorithm (TH-BSGS, DH-BSGS, BSGS, diagonal method), split, level,
a sparse random subset of the diagonals, and a strided, centred progression
of offsets.  Each result must also decrypt to M v within 5e-3."""
import numpy as np
import pytest

import oracle as O
import paper_2605_17222_amd as H
import workload as W
from gpu_common import gpu_params, limbs_tensor, log

pytestmark = pytest.mark.gpu

CASES = 24


def _config(rng, S):
    algo = ["th", "dh", "bsgs", "naive"][int(rng.integers(0, 4))]
    stride = int(rng.choice([1, 1, 2, 3, 5, 16]))
    if algo == "th":
        split = tuple(int(x) for x in rng.choice([1, 2, 4], size=3))
    else:
        split = tuple(int(x) for x in rng.choice([1, 2, 4, 8], size=2))
    n = int(np.prod(split))
    if algo == "naive":
        n = int(rng.integers(1, 17))
    centre = int(rng.integers(0, n))
    # the progression must not repeat an offset modulo S
    assert n * stride <= S
    present = sorted(set(int(t) for t in rng.choice(n, size=int(rng.integers(1, n + 1)), replace=True)))
    return algo, split, n, stride, centre, present


def test_random_configurations_bit_exact():
    import torch
    prm = W.params_toy()
    S = prm.slots
    o = O.Oracle(prm)
    o.keygen(777)
    P = gpu_params(prm)
    delta = 2.0 ** prm.log_delta
    rng = np.random.Generator(np.random.PCG64(2026))
    keycache = {}
    for case in range(CASES):
        algo, split, n, stride, centre, present = _config(rng, S)
        level = int(rng.integers(1, prm.max_level + 1))
        offs = [stride * (t - centre) for t in present]
        diags = W.banded_diagonals(1000 + case, S, offs)
        v = W.input_vector(2000 + case, S)
        ct = o.encrypt(level, v, delta, seed=3000 + case)
        if algo in ("th", "dh"):
            th_split = split if algo == "th" else (1,) + split
            rots = W.th_rotations(*th_split, stride=stride, centre=centre, slots=S)
            pts = o.th_plaintexts(diags, *th_split, delta, stride=stride, centre=centre)
        elif algo == "bsgs":
            rots = W.bsgs_rotations(*split, stride=stride, centre=centre, slots=S)
            pts = o.bsgs_plaintexts(diags, *split, delta, stride=stride, centre=centre)
        else:
            rots = sorted(set((stride * (t - centre)) % S for t in range(n)) - {0})
            pts = o.naive_plaintexts(diags, delta, stride=stride, centre=centre, n=n)
        need = [r for r in rots if r not in keycache]
        if need:
            keycache.update(o.rotkeys(need))
        keys = {r: keycache[r] for r in rots}
        log("case", case, algo, split, "n", n, "stride", stride, "centre", centre, "level", level,
            "present", len(present))
        if algo == "th":
            ref = o.lt_th(level, ct, th_split, pts, keys, stride=stride, centre=centre)
        elif algo == "dh":  # the oracle's Algorithm 1
            ref = o.lt_dh(level, ct, split, pts, keys, stride=stride, centre=centre)
        elif algo == "bsgs":
            ref = o.lt_bsgs(level, ct, split, pts, keys, stride=stride, centre=centre)
        else:
            ref = o.lt_naive(level, ct, pts, keys, stride=stride, centre=centre)
        code = {"th": H.CKKS_LT_TH_BSGS, "dh": H.CKKS_LT_DH_BSGS, "bsgs": H.CKKS_LT_BSGS,
                "naive": H.CKKS_LT_NAIVE}[algo]
        dpts = [None if f is None else limbs_tensor(f) for f in pts]
        dkeys = {r: limbs_tensor(k) for r, k in keys.items()}
        c0, c1 = limbs_tensor(ct[0]), limbs_tensor(ct[1])
        gsplit = split if algo != "naive" else (1, 1, 1)
        wsb = H.ckks_lt_workspace_size(P, level, gsplit, dpts, code, stride=stride, centre=centre)
        ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
        o0, o1 = H.empty((level, prm.n)), H.empty((level, prm.n))
        lvl, sc = H.ckks_lt_eval(P, level, delta, c0, c1, gsplit, dpts, delta, dkeys, code, o0, o1, ws, wsb,
                                 stride=stride, centre=centre)
        torch.cuda.synchronize()
        got = np.stack([H.to_host(o0), H.to_host(o1)])
        assert lvl == level - 1
        assert np.array_equal(got, ref), case
        assert np.abs(o.decrypt_slots(got, sc) - W.matvec(diags, v)).max() <= 5e-3, case
