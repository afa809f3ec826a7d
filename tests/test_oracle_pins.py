"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
a definition evaluated by brute force with Python integers, a closed form, an
invariant, or a value printed in the paper (tests/golden/paper_values.json).
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workload as W
from oracle import encoding as E
from _helpers import bitrev, centred, crt, crt_columns, negacyclic_schoolbook, small_params

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module")
def tiny():
    """N = 2^5, three 30-bit q, one 31-bit p, dnum 3 (alpha 1)."""
    o = O.Oracle(small_params(5))
    o.keygen(3)
    return o


@pytest.fixture(scope="module")
def tiny2():
    """N = 2^6, five q, two p (alpha 2, beta 3): groups of unequal size."""
    o = O.Oracle(small_params(6, nq=5, np_=2, dnum=3, bits_q=28, bits_p=30))
    o.keygen(4)
    return o


def test_bitrev_worked_example():
    # Section V: bitrev(1, 3) = '001' -> '100' = 4.
    ex = GOLDEN["bitrev_example"]
    assert bitrev(ex["x"], ex["bits"]) == ex["value"]


def test_primes_ntt_friendly():
    for prm in (W.params_toy(), W.params_n16()):
        two_n = 2 * prm.n
        allp = list(prm.q) + list(prm.p)
        assert len(set(allp)) == len(allp)
        for q in allp:
            assert q % two_n == 1 and W.is_prime(q) and q < 2 ** 61
    # trial division for the 30-bit primes of the toy chain
    for q in W.params_toy().q[1:]:
        assert all(q % d for d in range(2, int(q ** 0.5) + 1))
    prm = W.params_n16()
    assert [x.bit_length() for x in prm.q] == [60] + [40] * 24
    assert [x.bit_length() for x in prm.p] == [60] * 9


def test_ctx_rejects_bad_primes():
    prm = small_params(5)
    bad = W.Params(log_n=5, q=(prm.q[0], prm.q[1], prm.q[1]), p=prm.p, dnum=3, log_delta=20, h=8)
    with pytest.raises(RuntimeError):
        O.Oracle(bad)  # duplicate prime
    bad = W.Params(log_n=5, q=(prm.q[0], prm.q[1], prm.q[2] + 64), p=prm.p, dnum=3, log_delta=20, h=8)
    with pytest.raises(RuntimeError):
        O.Oracle(bad)  # 1 mod 2N but composite or not prime
    bad = W.Params(log_n=5, q=(prm.q[0], prm.q[1], 1000003), p=prm.p, dnum=3, log_delta=20, h=8)
    with pytest.raises(RuntimeError):
        O.Oracle(bad)  # prime but not 1 mod 2N


def test_psi_primitive(tiny):
    n = tiny.n
    for i, q in enumerate(tiny.pq):
        psi = tiny.psi(i)
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1


@pytest.mark.parametrize("log_n", [3, 5, 8])
def test_ntt_matches_definition(log_n):
    # Position p holds sum_k a_k psi^((2 br(p) + 1) k)  (bit-reversed storage, Section V).
    o = O.Oracle(small_params(log_n, nq=1, np_=1, dnum=1))
    n = o.n
    g = np.random.default_rng(log_n)
    for pqi, q in enumerate(o.pq):
        a = g.integers(0, q, n, dtype=np.uint64)
        got = o.ntt(a[None, :], [pqi])[0]
        psi = o.psi(pqi)
        for p in range(n):
            e = 2 * bitrev(p, log_n) + 1
            ref = sum(int(a[k]) * pow(psi, e * k, q) for k in range(n)) % q
            assert int(got[p]) == ref


@pytest.mark.parametrize("log_n", [3, 6, 8])
def test_ntt_product_is_negacyclic_convolution(log_n):
    # T1: INTT(NTT(a) .* NTT(b)) = a * b mod (x^N + 1).
    o = O.Oracle(small_params(log_n, nq=2, np_=1, dnum=2))
    g = np.random.default_rng(100 + log_n)
    for pqi, q in enumerate(o.pq):
        a = g.integers(0, q, o.n, dtype=np.uint64)
        b = g.integers(0, q, o.n, dtype=np.uint64)
        A = o.ntt(a[None], [pqi])[0]
        B = o.ntt(b[None], [pqi])[0]
        C = np.array([(int(x) * int(y)) % q for x, y in zip(A, B)], dtype=np.uint64)
        c = o.intt(C[None], [pqi])[0]
        assert [int(x) for x in c] == negacyclic_schoolbook(a, b, q)
        assert np.array_equal(o.intt(A[None], [pqi])[0], a)


def test_ntt_inverse_large():
    o = O.Oracle(W.params_toy())
    g = np.random.default_rng(7)
    x = W.uniform_residues(7, o.pq, o.n)
    y = o.intt(o.ntt(x, range(len(o.pq))), range(len(o.pq)))
    assert np.array_equal(x, y)


def test_galois_order():
    # g = 5 has order N/2 modulo 2N (Section II-A).
    for log_n in (5, 12, 16):
        n = 1 << log_n
        x, order = 5, 1
        while x != 1:
            x = x * 5 % (2 * n)
            order += 1
        assert order == n // 2


def test_automorph_coefficient_definition(tiny):
    # phi(a)(x) = a(x^g) mod x^N + 1 is a ring homomorphism, composes as g*h,
    # and in the NTT domain is the gather of eq. (7).
    n, q = tiny.n, tiny.pq[1]
    g = np.random.default_rng(5)
    a = g.integers(0, q, n, dtype=np.uint64)
    b = g.integers(0, q, n, dtype=np.uint64)
    for r in (1, 3, -2, 7):
        gr = tiny.galois(r)
        assert gr == pow(5, r % (n // 2), 2 * n)
        pa = tiny.automorph_coeff(a, 1, gr)
        pb = tiny.automorph_coeff(b, 1, gr)
        pab = tiny.automorph_coeff(np.array(negacyclic_schoolbook(a, b, q), dtype=np.uint64), 1, gr)
        assert [int(x) for x in pab] == negacyclic_schoolbook(pa, pb, q)
        # NTT-domain gather equals NTT of the coefficient automorphism
        A = tiny.ntt(a[None], [1])
        assert np.array_equal(tiny.automorph_ntt(A, r), tiny.ntt(pa[None], [1]))
    g1, g2 = tiny.galois(2), tiny.galois(5)
    assert np.array_equal(tiny.automorph_coeff(tiny.automorph_coeff(a, 1, g1), 1, g2),
                          tiny.automorph_coeff(a, 1, g1 * g2 % (2 * n)))


@pytest.mark.parametrize("log_n,dp", [(8, 64), (12, 64), (12, 128), (12, 256), (16, 256)])
def test_row_permutation_property(log_n, dp):
    # Eq. (8): in the layout "row i, block j holds A_br(i dp + j)", the automorphism
    # maps every row as a whole onto one row, with distinct columns.
    o = O.Oracle(small_params(log_n, nq=1, np_=1, dnum=1))
    n = o.n
    ident = np.arange(n, dtype=np.uint64)[None]
    rows = n // dp
    rs = range(n // 2) if log_n <= 8 else list(range(1, 40)) + [n // 4 - 1, n // 2 - 1, -1, -64]
    for r in rs:
        src = o.automorph_ntt(ident, r)[0].astype(np.int64)    # out[p] = in[src[p]]
        # storage position p = i*dp + j holds index br(p); eq. (8) is about rows of that storage
        src_rows = (src // dp).reshape(rows, dp)
        assert (src_rows == src_rows[:, :1]).all()
        assert len(set(src_rows[:, 0])) == rows
        cols = (src % dp).reshape(rows, dp)
        assert all(len(set(c)) == dp for c in cols[: min(rows, 8)])


def test_encode_decode_direct_embedding():
    n = 16
    g = np.random.default_rng(1)
    m = g.integers(-1000, 1000, n)
    zeta = np.exp(1j * np.pi / n)
    e = E.slot_exponents(n)
    direct = np.array([sum(m[k] * zeta ** (int(e[t]) * k) for k in range(n)) for t in range(n // 2)])
    assert np.allclose(E.decode(m, 1.0, n), direct, atol=1e-9)
    z = W.complex_uniform(g, n // 2)
    coef = E.encode(z, 2.0 ** 30, n)
    assert np.abs(E.decode(coef, 2.0 ** 30, n) - z).max() < n * 2.0 ** -30
    # encoding a real vector's conjugate-symmetric embedding gives integer coefficients
    assert coef.dtype == np.int64


def test_slot_rotation_by_automorphism():
    # T2 on plaintexts: decode(phi_5^r(encode z)) = rot(z, r).
    o = O.Oracle(small_params(6, nq=1, np_=1, dnum=1))
    n = o.n
    g = np.random.default_rng(2)
    z = W.complex_uniform(g, n // 2)
    coef = E.encode(z, 2.0 ** 25, n)
    q = o.pq[1]
    poly = np.array([c % q for c in coef.tolist()], dtype=np.uint64)
    for r in (1, 5, -3, n // 2 - 1):
        rp = o.automorph_coeff(poly, 1, o.galois(r))
        back = np.array([centred(int(x), q) for x in rp])
        assert np.abs(E.decode(back, 2.0 ** 25, n) - np.roll(z, -r)).max() < 1e-5


def test_bconv_crt(tiny2):
    # Eq. (3): BConv(x) = [x]_S + u S with 0 <= u < |S|, checked in every destination prime.
    o = tiny2
    g = np.random.default_rng(9)
    src, dst = [2, 3, 4], [0, 1, 5, 6]
    S = [o.pq[i] for i in src]
    x = np.stack([g.integers(0, m, o.n, dtype=np.uint64) for m in S])
    out = o.bconv(src, x, dst)
    Sp = int(np.prod([int(m) for m in S], dtype=object))
    for k in range(o.n):
        X = crt([int(x[j, k]) for j in range(3)], S)
        us = set()
        for m_i, di in enumerate(dst):
            d = o.pq[di]
            diff = (int(out[m_i, k]) - X) % d
            u = [u for u in range(len(S)) if (u * Sp) % d == diff]
            assert u, "BConv output is not X + u S"
            us.add(u[0])
        assert len(us) == 1


def _coef(o, x, basis):
    return o.intt(x, basis)


def test_decompose_digits(tiny2):
    o, level = tiny2, 4
    g = np.random.default_rng(11)
    Qb = o.q_basis(level)
    x = np.stack([g.integers(0, o.pq[i], o.n, dtype=np.uint64) for i in Qb])
    d = o.decompose(level, x)
    assert d.shape == (3, o.K(level), o.n)
    xc = _coef(o, x, Qb)
    for b in range(3):
        grp = [j for j in range(level + 1) if j // o.alpha == b]
        mods = [o.params.q[j] for j in grp]
        Qg = int(np.prod([int(m) for m in mods], dtype=object))
        dc = _coef(o, d[b], o.pq_basis(level))
        for j in grp:   # own limbs copied unchanged (NTT form)
            assert np.array_equal(d[b][o.alpha + j], x[j])
        for k in range(0, o.n, 7):
            X = crt([int(xc[j, k]) for j in grp], mods)
            vals = [(int(dc[l, k]) - X) % o.pq[l] for l in range(o.K(level))]
            ok = [u for u in range(len(grp)) if all((u * Qg) % o.pq[l] == vals[l] for l in range(o.K(level)))]
            assert ok


def test_moddown_of_p_multiple_is_exact(tiny2):
    o, level = tiny2, 4
    g = np.random.default_rng(12)
    Qb = o.q_basis(level)
    x = np.stack([g.integers(0, o.pq[i], o.n, dtype=np.uint64) for i in Qb])
    px = o.p_scale(level, x)
    assert np.array_equal(o.moddown(level, px), x)


def test_moddown_floor(tiny2):
    # Eq. (4): ModDown(c) = floor(c / P) - u, 0 <= u < alpha, for the integer c in [0, PQ).
    o, level = tiny2, 3
    g = np.random.default_rng(13)
    B = o.pq_basis(level)
    x = np.stack([g.integers(0, o.pq[i], o.n, dtype=np.uint64) for i in B])
    out = _coef(o, o.moddown(level, x), o.q_basis(level))
    xc = _coef(o, x, B)
    P = int(np.prod([int(p) for p in o.params.p], dtype=object))
    Q = int(np.prod([int(q) for q in o.params.q[: level + 1]], dtype=object))
    mods = [o.pq[i] for i in B]
    for k in range(o.n):
        c = crt([int(xc[l, k]) for l in range(len(B))], mods)
        got = crt([int(out[j, k]) for j in range(level + 1)], o.params.q[: level + 1])
        assert (c // P - got) % Q in range(o.alpha)


def test_rescale_floor(tiny2):
    # Eq. (1): rescale(c) = floor(c / q_l) exactly.
    o, level = tiny2, 4
    g = np.random.default_rng(14)
    Qb = o.q_basis(level)
    x = np.stack([g.integers(0, o.pq[i], o.n, dtype=np.uint64) for i in Qb])
    out = _coef(o, o.rescale(level, x), o.q_basis(level - 1))
    xc = _coef(o, x, Qb)
    qs = list(o.params.q[: level + 1])
    for k in range(o.n):
        c = crt([int(xc[j, k]) for j in range(level + 1)], qs)
        assert crt([int(out[j, k]) for j in range(level)], qs[:level]) == c // qs[level]


def test_moddown_rescale_floor(tiny2):
    # Combined ModDown + rescale: floor(c / (P q_l)) - u, 0 <= u <= alpha.
    o, level = tiny2, 4
    g = np.random.default_rng(15)
    B = o.pq_basis(level)
    x = np.stack([g.integers(0, o.pq[i], o.n, dtype=np.uint64) for i in B])
    out = _coef(o, o.moddown_rescale(level, x), o.q_basis(level - 1))
    xc = _coef(o, x, B)
    P = int(np.prod([int(p) for p in o.params.p], dtype=object)) * o.params.q[level]
    Qm = int(np.prod([int(q) for q in o.params.q[:level]], dtype=object))
    mods = [o.pq[i] for i in B]
    for k in range(o.n):
        c = crt([int(xc[l, k]) for l in range(len(B))], mods)
        got = crt([int(out[j, k]) for j in range(level)], o.params.q[:level])
        assert (c // P - got) % Qm in range(o.alpha + 1)


def test_encrypt_decrypt(tiny2):
    o = tiny2
    g = np.random.default_rng(16)
    m = g.integers(-(1 << 20), 1 << 20, o.n)
    for level in (0, 2, 4):
        ct = o.encrypt_coeffs(level, m, seed=level)
        assert np.abs(o.decrypt(ct) - m).max() <= 6 * 3.2


def test_switching_key_identity(tiny2):
    # swk~_{b,0} + swk~_{b,1} phi_{-r}(s) = phi_{-r}(e_b) + G_b s with |e_b| <= 6 sigma,
    # G_b = [P]_{q_j} on the q_j of group b, 0 elsewhere.
    o = tiny2
    L, K = o.L, o.K(o.L)
    s = o.secret()
    assert np.count_nonzero(s) == o.params.h and set(np.unique(s)) <= {-1, 0, 1}
    S = o.poly_from_signed(s, o.pq_basis(L))
    P = int(np.prod([int(p) for p in o.params.p], dtype=object))
    for r in (1, 3, -1):
        key = o.rotkey(r)
        Sr = o.automorph_ntt(S, -r)
        for b in range(o.beta(L)):
            res = np.empty((K, o.n), dtype=np.uint64)
            for l in range(K):
                q = o.pq[l]
                j = l - o.alpha
                G = P % q if (j >= 0 and j // o.alpha == b) else 0
                k0 = key[b, 0, l].astype(object)
                k1 = key[b, 1, l].astype(object)
                v = (k0 + k1 * Sr[l].astype(object) - G * S[l].astype(object)) % q
                res[l] = v.astype(np.uint64)
            e = o.intt(res, o.pq_basis(L))
            for l in range(K):
                cen = np.array([centred(int(v), o.pq[l]) for v in e[l]])
                assert np.abs(cen).max() <= 6 * 3.2
                if l:
                    assert np.array_equal(cen, prev)
                prev = cen


def test_rotation_decrypts_to_slot_rotation():
    # T2: every rotation (including negative r) decrypts to the cyclic slot rotation.
    w = W.workload_toy()
    o = O.Oracle(w.params)
    o.keygen(21)
    delta = 2.0 ** w.params.log_delta
    ct = o.encrypt(w.level, w.vector, delta, seed=3)
    for r in (1, 2, 5, 16, -1, -7, w.params.slots // 2):
        keys = {r % w.params.slots: o.rotkey(r)}
        out = o.rotate(w.level, ct, r, keys)
        assert np.abs(o.decrypt_slots(out, delta) - np.roll(w.vector, -r)).max() < 1e-3


def test_rotation_missing_key_raises():
    w = W.workload_toy()
    o = O.Oracle(w.params)
    o.keygen(1)
    ct = o.encrypt(w.level, w.vector, 2.0 ** 30, seed=3)
    with pytest.raises(RuntimeError):
        o.rotate(w.level, ct, 3, {1: o.rotkey(1)})
