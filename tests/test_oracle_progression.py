"""Pins of the oracle's LT over a strided, centred progression of diagonals
(offset(t) = stride (t - centre)): the reading of Algorithm 2 used for sparse
factors such as those of a DFT, where offsets are negative and may wrap.
Decryptions must match FP64 M v, all three algorithms must agree, and the
operation counts must follow from which giant rotations vanish."""
import numpy as np
import pytest

import oracle as O
import workload as W


@pytest.fixture(scope="module")
def toy():
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(201)
    delta = 2.0 ** prm.log_delta
    v = W.input_vector(202, prm.slots)
    ct = o.encrypt(prm.max_level, v, delta, seed=203)
    return prm, o, v, ct, delta


def _run(o, prm, ct, diags, split, bsgs_split, stride, centre, delta, level=None):
    level = prm.max_level if level is None else level
    S = prm.slots
    rots = set(W.th_rotations(*split, stride=stride, centre=centre, slots=S))
    rots |= set(W.bsgs_rotations(*bsgs_split, stride=stride, centre=centre, slots=S))
    rots |= set((stride * (t - centre)) % S for t in range(split[0] * split[1] * split[2])) - {0}
    keys = o.rotkeys(sorted(rots))
    n = split[0] * split[1] * split[2]
    scale = delta * delta / prm.q[level]
    th = o.lt_th(level, ct, split, o.th_plaintexts(diags, *split, delta, stride=stride, centre=centre), keys,
                 stride=stride, centre=centre)
    bs = o.lt_bsgs(level, ct, bsgs_split,
                   o.bsgs_plaintexts(diags, *bsgs_split, delta, stride=stride, centre=centre), keys,
                   stride=stride, centre=centre)
    nv = o.lt_naive(level, ct, o.naive_plaintexts(diags, delta, stride=stride, centre=centre, n=n), keys,
                    stride=stride, centre=centre)
    return [o.decrypt_slots(x, scale) for x in (th, bs, nv)], th


@pytest.mark.parametrize("stride,centre", [(1, 8), (3, 8), (5, 3), (7, 0), (2, 15)])
def test_progression_lt_matches_matvec(toy, stride, centre):
    prm, o, v, ct, delta = toy
    S = prm.slots
    # every index but the first holds a diagonal: offsets stride*(t - centre)
    offs = [stride * (t - centre) for t in range(1, 16)]
    diags = W.banded_diagonals(stride * 100 + centre, S, offs)
    ref = W.matvec(diags, v)
    zs, _ = _run(o, prm, ct, diags, (2, 2, 4), (4, 4), stride, centre, delta)
    for z in zs:
        assert np.abs(z - ref).max() <= 5e-3
    # a wrong sign of the offsets would give M^T-like results instead
    wrong = W.matvec({(-d) % S: x for d, x in diags.items()}, v)
    assert np.abs(zs[0] - wrong).max() > 0.1


def test_giant_rotation_counts(toy):
    prm, o, v, ct, delta = toy
    S = prm.slots
    offs = [3 * (t - 8) for t in range(16)]
    diags = W.banded_diagonals(7, S, offs)
    o.reset_counters()
    _run(o, prm, ct, diags, (2, 2, 4), (4, 4), 3, 8, delta)
    # centre 8 = 2 n1 n2: block k = 2 is not rotated, like k = 0 in Algorithm 2
    o.reset_counters()
    o.lt_th(prm.max_level, ct, (2, 2, 4), o.th_plaintexts(diags, 2, 2, 4, delta, stride=3, centre=8),
            o.rotkeys(W.th_rotations(2, 2, 4, stride=3, centre=8, slots=S)), stride=3, centre=8)
    c = o.counters()
    assert c["decompose"] == 2 + 3 and c["moddown"] == 1 + 3 + 2 and c["keys"] == 1 + 1 + 3
    # centre 3 is no multiple of n1 n2: every block is rotated
    offs = [3 * (t - 3) for t in range(16)]
    diags = W.banded_diagonals(8, S, offs)
    keys = o.rotkeys(W.th_rotations(2, 2, 4, stride=3, centre=3, slots=S))
    # G_k = 3 (4k - 3) = -9, 3, 15, 27: G_1 coincides with the inner rotation 3
    assert len(keys) == 1 + 1 + 4 - 1
    o.reset_counters()
    out = o.lt_th(prm.max_level, ct, (2, 2, 4), o.th_plaintexts(diags, 2, 2, 4, delta, stride=3, centre=3), keys,
                  stride=3, centre=3)
    c = o.counters()
    assert c["decompose"] == 2 + 4 and c["moddown"] == 1 + 4 + 2 and c["keys"] == 5
    z = o.decrypt_slots(out, delta * delta / prm.q[prm.max_level])
    assert np.abs(z - W.matvec(diags, v)).max() <= 5e-3


def test_wrapped_offsets_are_merged(toy):
    # offsets j*256, |j| <= 7, wrap modulo 2048 slots onto 8 distinct ones
    prm, o, v, ct, delta = toy
    S = prm.slots
    diags = W.phase_diagonals(9, S, [j * 256 for j in range(-7, 8)])
    assert sorted(diags) == [256 * t for t in range(8)]
    # merged entries are sums of two unit phases (offset 0 keeps one)
    assert np.allclose(np.abs(diags[0]), 1.0) and np.abs(diags[256]).max() > 1.0
    zs, _ = _run(o, prm, ct, diags, (2, 2, 2), (2, 4), 256, 0, delta)
    ref = W.matvec(diags, v)
    for z in zs:
        assert np.abs(z - ref).max() <= 5e-3


def test_two_stage_chain_toy(toy):
    # stages with strides 1 and 16 (centred), one rescale each: level 2 -> 0
    prm, o, v, ct, delta = toy
    S = prm.slots
    stages = W.dft_chain(11, prm, stages=2)
    assert [st.stride for st in stages] == [1, 16] and all(st.centre == 8 for st in stages)
    rots = set()
    for st in stages:
        rots |= set(W.th_rotations(*st.split, stride=st.stride, centre=st.centre, slots=S))
    keys = o.rotkeys(sorted(rots))
    x, level, scale = ct, prm.max_level, delta
    for st in stages:
        pts = o.th_plaintexts(st.diags, *st.split, delta, stride=st.stride, centre=st.centre)
        x = o.lt_th(level, x, st.split, pts, keys, stride=st.stride, centre=st.centre)
        scale = scale * delta / prm.q[level]
        level -= 1
    z = o.decrypt_slots(x, scale)
    ref = W.chain_matvec(stages, v)
    assert np.abs(z - ref).max() <= 5e-3


def test_progression_must_not_repeat_offsets(toy):
    prm, o, v, ct, delta = toy
    with pytest.raises(AssertionError):
        o.th_plaintexts({0: np.ones(prm.slots)}, 2, 2, 4, delta, stride=prm.slots // 8, centre=0)
