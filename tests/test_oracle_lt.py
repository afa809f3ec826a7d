"""LT-level pins of the oracle: T3 (three algorithms agree), T4 (against FP64 M v),
the operation counts stated in Section III / Table I, and special cases."""
import numpy as np
import pytest

import oracle as O
import workload as W
from _helpers import small_params


@pytest.fixture(scope="module")
def toy():
    w = W.workload_toy()
    o = O.Oracle(w.params)
    o.keygen(101)
    delta = 2.0 ** w.params.log_delta
    ct = o.encrypt(w.level, w.vector, delta, seed=102)
    rots = set(W.th_rotations(*w.th_split)) | set(W.bsgs_rotations(*w.bsgs_split)) | set(range(1, 16))
    keys = o.rotkeys(sorted(rots))
    return w, o, ct, keys, delta


def _decode(o, out, w, delta):
    scale = delta * delta / w.params.q[w.level]
    return o.decrypt_slots(out, scale)


def test_t3_t4_toy(toy):
    w, o, ct, keys, delta = toy
    ref = W.matvec(w.diags, w.vector)
    th = o.lt_th(w.level, ct, w.th_split, o.th_plaintexts(w.diags, *w.th_split, delta), keys)
    bs = o.lt_bsgs(w.level, ct, w.bsgs_split, o.bsgs_plaintexts(w.diags, *w.bsgs_split, delta), keys)
    nv = o.lt_naive(w.level, ct, o.naive_plaintexts(w.diags, delta), keys)
    zs = [_decode(o, x, w, delta) for x in (th, bs, nv)]
    for z in zs:                                  # T4: <= 5e-3 at Delta = 2^30
        assert np.abs(z - ref).max() <= 5e-3
    for a in zs:                                  # T3: the three agree within tolerance
        for b in zs:
            assert np.abs(a - b).max() <= 5e-3
    # different algorithms give different (equally valid) ciphertexts
    assert not np.array_equal(th, bs)


@pytest.mark.parametrize("split", [(2, 2, 4), (4, 2, 2), (1, 4, 4), (2, 8, 1), (16, 1, 1), (1, 1, 16)])
def test_th_counts_match_text(toy, split):
    # Section III: n1'+n3'-1 Decompose, n1'+n3' ModDown (final one counted once per
    # polynomial) and n1'+n2'+n3'-3 switching keys.
    w, o, ct, keys, delta = toy
    n1, n2, n3 = split
    o.reset_counters()
    out = o.lt_th(w.level, ct, split, o.th_plaintexts(w.diags, n1, n2, n3, delta), keys)
    c = o.counters()
    if min(split) >= 2:
        assert c["decompose"] == n1 + n3 - 1
        assert c["moddown"] == n1 + n3
    # degenerate splits skip the Decompose/ModDown whose output nothing uses
    need_d0 = n1 > 1 or n2 > 1
    assert c["decompose"] == int(need_d0) + (n1 - 1) * (n2 > 1) + (n3 - 1)
    assert c["moddown"] == (n1 - 1) * (n2 > 1) + (n3 - 1) + 2
    assert c["keys"] == n1 + n2 + n3 - 3
    assert c["ks"] == n1 * n2 + n3 - 2
    ref = W.matvec(w.diags, w.vector)
    assert np.abs(_decode(o, out, w, delta) - ref).max() <= 5e-3


@pytest.mark.parametrize("split", [(4, 4), (2, 8), (8, 2)])
def test_bsgs_counts_match_table1(toy, split):
    # Table I, row BSGS: n1+n2-2 Decompose, 2(n1+n2-2) ModDown, n1+n2-2 keys.
    w, o, ct, keys, delta = toy
    n1, n2 = split
    o.reset_counters()
    out = o.lt_bsgs(w.level, ct, split, o.bsgs_plaintexts(w.diags, n1, n2, delta), keys)
    c = o.counters()
    assert c["decompose"] == n1 + n2 - 2
    assert c["moddown"] == 2 * (n1 + n2 - 2)
    assert c["keys"] == n1 + n2 - 2
    assert np.abs(_decode(o, out, w, delta) - W.matvec(w.diags, w.vector)).max() <= 5e-3


def test_th_skips_zero_diagonals(toy):
    # Absent diagonals are skipped exactly: a single diagonal at offset 5 needs
    # only the keys on its own path and no outer-layer work.
    w, o, ct, keys, delta = toy
    diags = {5: w.diags[5]}
    o.reset_counters()
    out = o.lt_th(w.level, ct, (2, 2, 4), o.th_plaintexts(diags, 2, 2, 4, delta), keys)
    c = o.counters()
    assert c["keys"] == 2                     # rotations 1 and 4
    assert c["decompose"] == 2 and c["moddown"] == 3
    ref = W.matvec(diags, w.vector)
    assert np.abs(_decode(o, out, w, delta) - ref).max() <= 5e-3


def test_th_identity_and_diagonal_scaling(toy):
    # The identity matrix (diagonal 0 all ones) reproduces the input slots.
    w, o, ct, keys, delta = toy
    S = w.params.slots
    diags = {0: np.ones(S, dtype=complex)}
    o.reset_counters()
    out = o.lt_th(w.level, ct, (2, 2, 4), o.th_plaintexts(diags, 2, 2, 4, delta), keys)
    assert np.abs(_decode(o, out, w, delta) - w.vector).max() <= 5e-3
    c = o.counters()
    assert c["decompose"] == 0 and c["keys"] == 0 and c["moddown"] == 2


def test_th_lower_level(toy):
    # Keys and plaintexts generated at the top level are truncated by prefix.
    w, o, ct, keys, delta = toy
    ct1 = o.encrypt(1, w.vector, delta, seed=7)
    out = o.lt_th(1, ct1, w.th_split, o.th_plaintexts(w.diags, *w.th_split, delta), keys)
    z = o.decrypt_slots(out, delta * delta / w.params.q[1])
    assert np.abs(z - W.matvec(w.diags, w.vector)).max() <= 5e-3


def test_th_multi_digit_groups():
    # Unequal digit groups (alpha = 2, five q limbs, beta = 3) and negative
    # effective rotations through the outer layer.
    prm = small_params(8, nq=5, np_=2, dnum=3, bits_q=40, bits_p=52, log_delta=30, h=16)
    prm = W.Params(log_n=8, q=(W.ntt_primes(50, 1, 512)[0],) + prm.q[1:], p=prm.p, dnum=3, log_delta=30, h=16)
    o = O.Oracle(prm)
    o.keygen(5)
    S = prm.slots
    diags = W.banded_diagonals(3, S, range(12))
    v = W.input_vector(3, S)
    delta = 2.0 ** 30
    ct = o.encrypt(4, v, delta, seed=9)
    keys = o.rotkeys(W.th_rotations(2, 2, 3) + W.bsgs_rotations(3, 4))
    th = o.lt_th(4, ct, (2, 2, 3), o.th_plaintexts(diags, 2, 2, 3, delta), keys)
    bs = o.lt_bsgs(4, ct, (3, 4), o.bsgs_plaintexts(diags, 3, 4, delta), keys)
    ref = W.matvec(diags, v)
    sc = delta * delta / prm.q[4]
    assert np.abs(o.decrypt_slots(th, sc) - ref).max() <= 5e-3
    assert np.abs(o.decrypt_slots(bs, sc) - ref).max() <= 5e-3


@pytest.mark.parametrize("split", [(4, 4), (8, 2), (2, 8)])
def test_dh_algorithm1_counts_and_t4(toy, split):
    # Algorithm 1 (DH-BSGS) as written in the oracle: Table I's DH row,
    # n2 Decompose, n2 + 1 ModDown, n1 + n2 - 2 keys; T4 against M v.
    w, o, ct, keys, delta = toy
    n1, n2 = split
    pts = o.dh_plaintexts(w.diags, n1, n2, delta)
    o.reset_counters()
    out = o.lt_dh(w.level, ct, split, pts, keys)
    c = o.counters()
    assert c["decompose"] == n2 and c["moddown"] == n2 + 1 and c["keys"] == n1 + n2 - 2
    assert np.abs(_decode(o, out, w, delta) - W.matvec(w.diags, w.vector)).max() <= 5e-3


@pytest.mark.parametrize("split,prog", [((4, 4), (1, 0)), ((8, 2), (1, 0)), ((2, 8), (1, 0)), ((4, 4), (3, 8)),
                                        ((2, 8), (5, 3))])
def test_dh_algorithm1_equals_algorithm2_with_unit_inner_layer(toy, split, prog):
    # Two separately written algorithms reach the same bytes: Algorithm 1
    # with (n1, n2) and Algorithm 2 with (n1', n2', n3') = (1, n1, n2) take
    # the same steps on the same operands (Section III), so any slip in
    # either one's indexing, rotation or accumulation shows here.
    w, o, ct, keys, delta = toy
    n1, n2 = split
    s, c = prog
    rots = set(W.th_rotations(1, n1, n2, stride=s, centre=c, slots=w.params.slots))
    ks = {r: keys[r] if r in keys else o.rotkey(r) for r in rots}
    diags = {d: w.diags[d] for d in w.diags}
    # a progression offset s (t - c): place the workload's diagonals there
    if prog != (1, 0):
        S = w.params.slots
        diags = {(s * (t - c)) % S: w.diags[t % 16] for t in range(n1 * n2) if t % 3 != 1}
    pts = o.dh_plaintexts(diags, n1, n2, delta, stride=s, centre=c)
    dh = o.lt_dh(w.level, ct, split, pts, ks, stride=s, centre=c)
    th = o.lt_th(w.level, ct, (1, n1, n2), o.th_plaintexts(diags, 1, n1, n2, delta, stride=s, centre=c), ks,
                 stride=s, centre=c)
    assert np.array_equal(dh, th)
    assert np.abs(_decode(o, dh, w, delta) - W.matvec(diags, w.vector)).max() <= 5e-3


def test_dh_algorithm1_sequential_last_line(toy):
    # The last line read literally (ModDown of c0 and c1, then eq. (1))
    # against the combined ModDown by P q_l: different floors, the same
    # message within the rounding error.
    w, o, ct, keys, delta = toy
    pts = o.dh_plaintexts(w.diags, 4, 4, delta)
    comb = o.lt_dh(w.level, ct, (4, 4), pts, keys)
    seq = o.lt_dh(w.level, ct, (4, 4), pts, keys, combined=False)
    assert not np.array_equal(comb, seq)
    za, zb = _decode(o, comb, w, delta), _decode(o, seq, w, delta)
    assert np.abs(za - zb).max() <= 5e-3
    assert np.abs(zb - W.matvec(w.diags, w.vector)).max() <= 5e-3


def test_paper_set_parameters_are_valid():
    # The paper's Set-A/B/C (Table V): N, L+1, alpha and beta as
    # printed, every prime 54 bits and 1 mod 2N; digits of alpha primes give
    # beta = ceil((L+1)/alpha) digits (Set-C: 32 primes, alpha 12, beta 3).
    table = {"A": (2 ** 13, 5, 5, 1), "B": (2 ** 15, 16, 8, 2), "C": (2 ** 16, 32, 12, 3)}
    for name, (n, lq, alpha, beta) in table.items():
        p = W.params_paper_set(name)
        assert (p.n, p.max_level + 1, p.alpha, p.beta(p.max_level), p.dnum) == (n, lq, alpha, beta, beta)
        primes = list(p.q) + list(p.p)
        assert len(set(primes)) == len(primes)
        for x in primes:
            assert x.bit_length() == 54 and x % (2 * n) == 1 and W.is_prime(x)


def test_paper_set_a_oracle_t3_t4():
    # T3/T4 at Set-A (N = 2^13, 54-bit primes, one digit): TH-BSGS and plain
    # BSGS on 32 banded diagonals decrypt to FP64 M v and to each other.
    prm = W.params_paper_set("A")
    o = O.Oracle(prm)
    o.keygen(181)
    S, delta = prm.slots, 2.0 ** prm.log_delta
    diags = W.banded_diagonals(182, S, range(32))
    v = W.input_vector(183, S)
    level = prm.max_level
    ct = o.encrypt(level, v, delta, seed=184)
    keys = o.rotkeys(sorted(set(W.th_rotations(2, 4, 4)) | set(W.bsgs_rotations(4, 8))))
    th = o.lt_th(level, ct, (2, 4, 4), o.th_plaintexts(diags, 2, 4, 4, delta), keys)
    bs = o.lt_bsgs(level, ct, (4, 8), o.bsgs_plaintexts(diags, 4, 8, delta), keys)
    scale = delta * delta / prm.q[level]
    ref = W.matvec(diags, v)
    zt, zb = o.decrypt_slots(th, scale), o.decrypt_slots(bs, scale)
    # The floors of eq. (1) and eq. (4) bias every coefficient of the result
    # by up to -(alpha + 1)/2 on average.  A constant c in every coefficient
    # evaluates at zeta^e to c (1 - zeta^(eN)) / (1 - zeta^e), of size about
    # |c| 2N / (pi e') with e' = min(e, 2N - e): the error lands on the slots
    # whose 5^t mod 2N is near 0 (slot 0 has e = 1), times |1 + s(zeta^e)|
    # (~ sqrt(h), taken 8 sqrt(h)) for the c1 part.  At output scale
    # 2^80 / q_l ~ 2^26, N = 2^13, alpha = 5 that is B / e' with
    # B = 3 * (2N / pi) * 8 sqrt(192) / 2^26 = 0.026; the rest is rounding
    # noise (1e-4 covers it).
    n = prm.n
    e5 = np.array([pow(5, t, 2 * n) for t in range(S)])
    bound = 0.026 / np.minimum(e5, 2 * n - e5) + 1e-4
    for z in (zt, zb):
        e = np.abs(z - ref)
        assert np.all(e <= bound)
        assert np.median(e) <= 3e-5
    assert np.all(np.abs(zt - zb) <= 2 * bound)


def test_paper_set_a_plaintext_scale_q_l_uniform_1e4():
    # Set-A with the plaintext scale taken from the set's own primes: Delta_pt
    # = q_l, the prime the LT's last line divides by, so the output scale is
    # the input's Delta = 2^40 again (not 2^80 / q_l ~ 2^26).  The floor bias
    # of eq. (1)/(4) then sits 2^14 times lower relative to the message and
    # T4 holds at 1e-4 in every slot, slot 0 included.
    prm = W.params_paper_set("A")
    o = O.Oracle(prm)
    o.keygen(181)
    S, delta = prm.slots, 2.0 ** prm.log_delta
    diags = W.banded_diagonals(182, S, range(32))
    v = W.input_vector(183, S)
    level = prm.max_level
    pt_scale = float(prm.q[level])
    ct = o.encrypt(level, v, delta, seed=184)
    keys = o.rotkeys(sorted(set(W.th_rotations(2, 4, 4)) | set(W.bsgs_rotations(4, 8))))
    th = o.lt_th(level, ct, (2, 4, 4), o.th_plaintexts(diags, 2, 4, 4, pt_scale), keys)
    bs = o.lt_bsgs(level, ct, (4, 8), o.bsgs_plaintexts(diags, 4, 8, pt_scale), keys)
    scale = delta * pt_scale / prm.q[level]
    ref = W.matvec(diags, v)
    for out in (th, bs):
        assert np.abs(o.decrypt_slots(out, scale) - ref).max() <= 1e-4
