"""Plaintext encoding on the device, and LTs whose diagonals the library
encodes on the fly, against the oracle.

FP64 rounding decides each integer coefficient of an encoding (Section II-A:
m = round(scale sigma^-1(z))).  The device's FFT and the oracle's FFT round
differently in the last bits, so a coefficient whose unrounded value lies
within that error of a half-integer may round either way.  The checks:
everywhere else the integers are equal, and there they differ by 1; the
NTT-form residues equal the oracle's NTT of the device's integers bit for bit;
an LT with on-the-fly diagonals equals, bit for bit, the oracle's LT given
the device's encodings of the same (pre-rotated) diagonals; and every result
decrypts to M v within the stated tolerance."""
import numpy as np
import pytest

import oracle as O
import paper_2605_17222_amd as H
import workload as W
from gpu_common import gpu_params, limbs_tensor, log
from oracle import encoding as E

pytestmark = pytest.mark.gpu


def _slots_tensor(z):
    import torch
    return torch.from_numpy(np.ascontiguousarray(z, dtype=np.complex128)).to("cuda")


def _encode(P, prm, zs, rots, scale, first, nl):
    import torch
    outs = [H.empty((nl, prm.n)) for _ in zs]
    coefs = [torch.empty(prm.n, dtype=torch.int64, device="cuda") for _ in zs]
    wsb = H.ckks_encode_workspace_size(P, len(zs))
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
    dz = [_slots_tensor(z) for z in zs]
    H.ckks_encode(P, dz, rots, scale, first, nl, outs, ws, wsb, coefs)
    torch.cuda.synchronize()
    return [H.to_host(o) for o in outs], [c.cpu().numpy() for c in coefs]


def _check_coefficients(coef, z, rot, scale, n):
    """Equal to the oracle's rounding except at near-ties (FFT error bound)."""
    v = E.encode_unrounded(E.rotate_slots(z, rot), scale, n)
    ref = np.sign(v) * np.floor(np.abs(v) + 0.5)
    d = coef - ref.astype(np.int64)
    assert np.abs(d).max() <= 1
    if np.any(d):
        # both FFTs are within ~log2(N) ulp of max|v| of the exact value
        tol = 64 * np.log2(n) * np.finfo(np.float64).eps * np.abs(v).max()
        frac = np.abs(v[d != 0]) % 1.0
        assert np.all(np.abs(frac - 0.5) < tol), (frac, tol)
    return int(np.count_nonzero(d))


def _encode_case(prm, count, seed, bases):
    o = O.Oracle(prm)
    P = gpu_params(prm)
    S, scale = prm.slots, 2.0 ** prm.log_delta
    g = np.random.default_rng(seed)
    zs = [W.complex_uniform(W.rng(seed, i), S) for i in range(count)]
    rots = [0, 1, -1, S - 3] + [int(x) for x in g.integers(-S, S, size=count)]
    rots = rots[:count]
    ties = 0
    for first, nl in bases:
        basis = list(range(first, first + nl))
        log("encode", prm.log_n, "count", count, "primes", first, "..", first + nl - 1)
        outs, coefs = _encode(P, prm, zs, rots, scale, first, nl)
        for z, r, out, coef in zip(zs, rots, outs, coefs):
            ties += _check_coefficients(coef, z, r, scale, prm.n)
            # poly_from_signed reduces the integers into each prime and applies the NTT
            assert np.array_equal(out, o.poly_from_signed(coef, basis))
            back = E.decode(coef, scale, prm.n)
            assert np.abs(back - E.rotate_slots(z, r)).max() < 1e-5
    assert ties <= max(2, count * prm.n // 1000)


def test_encode_toy_against_oracle():
    prm = W.params_toy()
    K = prm.alpha + prm.max_level + 1
    _encode_case(prm, 24, 51, [(0, K), (prm.alpha, prm.max_level + 1), (0, prm.alpha + 2)])


def test_encode_n16_against_oracle():
    prm = W.params_n16()
    K = prm.alpha + prm.max_level + 1
    _encode_case(prm, 3, 52, [(0, K)])


def _pre_rotations(algo, split, n, stride, centre, S):
    """The giant-step rotation folded into plaintext t (0 for the diagonal method)."""
    if algo == "naive":
        return [0] * n
    block = split[0] * split[1] if algo == "th" else split[0]
    return [-(stride * (block * (t // block) - centre)) % S for t in range(n)]


def _onfly_case(prm, o, keys, level, split, diags_by_t, v, seed, algo="th", stride=1, centre=0, tol=5e-3, n=None,
                pt_scale=None):
    """Runs the LT with slot diagonals encoded on the fly and with the device's
    own encodings as plaintexts; both must equal the oracle's LT given those
    encodings, and decrypt to M v.  algo: th, dh, bsgs or naive (n indices).
    pt_scale: the plaintexts' scale (default the ciphertext's Delta)."""
    import torch
    P = gpu_params(prm)
    S, delta = prm.slots, 2.0 ** prm.log_delta
    pts_scale = delta if pt_scale is None else pt_scale
    if algo in ("th", "dh"):
        osplit = tuple(split) if algo == "th" else (1,) + tuple(split)
        n = int(np.prod(osplit))
        first, nl = 0, prm.alpha + prm.max_level + 1
        rots = W.th_rotations(*osplit, stride=stride, centre=centre, slots=S)
        pre = _pre_rotations("th", osplit, n, stride, centre, S)
    elif algo == "bsgs":
        osplit = tuple(split)
        n = int(np.prod(osplit))
        first, nl = prm.alpha, prm.max_level + 1
        rots = W.bsgs_rotations(*osplit, stride=stride, centre=centre, slots=S)
        pre = _pre_rotations("bsgs", osplit, n, stride, centre, S)
    else:
        osplit = None
        first, nl = prm.alpha, prm.max_level + 1
        rots = sorted(set((stride * (t - centre)) % S for t in range(n) if diags_by_t.get(t) is not None) - {0})
        pre = _pre_rotations("naive", None, n, stride, centre, S)
    ts = [t for t in range(n) if diags_by_t.get(t) is not None]
    enc, _ = _encode(P, prm, [diags_by_t[t] for t in ts], [pre[t] for t in ts], pts_scale, first, nl)
    pts = [None] * n
    for t, f in zip(ts, enc):
        pts[t] = f
    ct = o.encrypt(level, v, delta, seed=seed)
    okeys = {r: keys[r] for r in rots}
    log("oracle LT", prm.log_n, algo, "level", level, "split", osplit, "diagonals", len(ts))
    if algo == "th":
        ref = o.lt_th(level, ct, osplit, pts, okeys, stride=stride, centre=centre)
    elif algo == "dh":  # the oracle's Algorithm 1
        ref = o.lt_dh(level, ct, split, pts, okeys, stride=stride, centre=centre)
    elif algo == "bsgs":
        ref = o.lt_bsgs(level, ct, osplit, pts, okeys, stride=stride, centre=centre)
    else:
        ref = o.lt_naive(level, ct, pts, okeys, stride=stride, centre=centre)
    code = {"th": H.CKKS_LT_TH_BSGS, "dh": H.CKKS_LT_DH_BSGS, "bsgs": H.CKKS_LT_BSGS, "naive": H.CKKS_LT_NAIVE}[algo]
    gsplit = split if algo != "naive" else (1, 1, 1)
    dkeys = {r: limbs_tensor(k) for r, k in okeys.items()}
    c0, c1 = limbs_tensor(ct[0]), limbs_tensor(ct[1])
    dslots = [None if diags_by_t.get(t) is None else _slots_tensor(diags_by_t[t]) for t in range(n)]
    dpts = [None if f is None else limbs_tensor(f) for f in pts]
    res = []
    for onfly, items in ((True, dslots), (False, dpts)):
        wsb = H.ckks_lt_workspace_size(P, level, gsplit, items, code, stride=stride, centre=centre, onfly=onfly)
        ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
        o0, o1 = H.empty((level, prm.n)), H.empty((level, prm.n))
        log("device LT onfly" if onfly else "device LT plaintexts", "workspace", wsb)
        lvl, sc = H.ckks_lt_eval(P, level, delta, c0, c1, gsplit, items, pts_scale, dkeys, code, o0, o1, ws, wsb,
                                 stride=stride, centre=centre, onfly=onfly)
        torch.cuda.synchronize()
        res.append((np.stack([H.to_host(o0), H.to_host(o1)]), sc))
        del ws
    assert np.array_equal(res[0][0], ref)
    assert np.array_equal(res[1][0], ref)
    offs = {(stride * (t - centre)) % S: diags_by_t[t] for t in ts}
    errs = np.abs(o.decrypt_slots(res[0][0], res[0][1]) - W.matvec(offs, v))
    err = errs.max()
    log("decrypted max error", err)
    assert np.all(errs <= tol)
    return res[0][0]


def test_onfly_dense_toy_th():
    # The dense n = N/2 LT of the paper's parameter sets, at the toy ring:
    # 2048 diagonals, split (16, 16, 8), every plaintext encoded on the fly.
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(61)
    split = (16, 16, 8)
    keys = o.rotkeys(W.th_rotations(*split))
    S = prm.slots
    diags = W.banded_diagonals(62, S, range(S))
    _onfly_case(prm, o, keys, prm.max_level, split, {t: diags[t] for t in range(S)}, W.input_vector(63, S), 64)


def test_onfly_sparse_progressions_th_dh():
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(71)
    S = prm.slots
    g = np.random.default_rng(72)
    cases = [("th", (2, 4, 4), 1, 0), ("th", (4, 2, 2), 3, 5), ("dh", (4, 8), 16, 7), ("th", (2, 2, 4), 5, 8)]
    rots = set()
    for algo, split, stride, centre in cases:
        th_split = split if algo == "th" else (1,) + split
        rots |= set(W.th_rotations(*th_split, stride=stride, centre=centre, slots=S))
    keys = o.rotkeys(sorted(rots))
    for c, (algo, split, stride, centre) in enumerate(cases):
        n = int(np.prod(split))
        present = sorted(set(int(t) for t in g.choice(n, size=n // 2 + 1)))
        offs = {t: (stride * (t - centre)) % S for t in present}
        dg = W.banded_diagonals(80 + c, S, sorted(offs.values()))
        by_t = {t: dg[offs[t]] for t in present}
        log("case", c, algo, split, "stride", stride, "centre", centre, "present", len(present))
        _onfly_case(prm, o, keys, 1 + c % prm.max_level, split, by_t, W.input_vector(90 + c, S), 100 + c,
                    algo=algo, stride=stride, centre=centre)


def test_onfly_n16_banded64():
    # The N = 2^16, level 24, 64-diagonal workload with its plaintexts
    # encoded on the fly.
    prm = W.params_n16()
    o = O.Oracle(prm)
    o.keygen(111)
    split = (4, 4, 4)
    keys = o.rotkeys(W.th_rotations(*split))
    S = prm.slots
    diags = W.banded_diagonals(112, S, range(64))
    _onfly_case(prm, o, keys, 24, split, {t: diags[t] for t in range(64)}, W.input_vector(113, S), 114, tol=1e-4)


def test_onfly_through_server_equals_direct():
    import torch
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(121)
    split = (2, 2, 4)
    keys = o.rotkeys(W.th_rotations(*split))
    S, delta = prm.slots, 2.0 ** prm.log_delta
    diags = W.banded_diagonals(122, S, range(16))
    v = W.input_vector(123, S)
    direct = _onfly_case(prm, o, keys, 2, split, {t: diags[t] for t in range(16)}, v, 124)
    P = gpu_params(prm)
    ct = o.encrypt(2, v, delta, seed=124)
    c0, c1 = limbs_tensor(ct[0]), limbs_tensor(ct[1])
    dslots = [_slots_tensor(diags[t]) for t in range(16)]
    o0, o1 = H.empty((2, prm.n)), H.empty((2, prm.n))
    torch.cuda.synchronize()
    with H.Server(1 << 28, max_batch=2, max_inflight=1) as srv:
        ring = H.ckks_server_add_ring(srv, P, {r: limbs_tensor(k) for r, k in keys.items()})
        rid = H.ckks_server_submit(srv, ring, 2, delta, c0, c1, split, dslots, delta, o0, o1, onfly=True)
        H.ckks_server_wait_all(srv)
        status, _ = H.ckks_server_poll(srv, rid)
        assert status == H.CKKS_OK, H.strerror(status)
    got = np.stack([H.to_host(o0), H.to_host(o1)])
    assert np.array_equal(got, direct)


def test_onfly_dense_paper_set_a():
    # The paper's Set-A (N = 2^13, L+1 = 5, alpha = 5, 54-bit primes) with its
    # dense n = N/2 = 4096 LT and split (16, 16, 16), at the top level.  The
    # plaintexts are encoded at the scale of the prime the LT divides by
    # (Delta_pt = q_l), so the output keeps the input's Delta = 2^40 and the
    # result is within 1e-4 of M v in every slot.
    prm = W.params_paper_set("A")
    split = W.PAPER_SETS["A"]["split"]
    o = O.Oracle(prm)
    o.keygen(131)
    keys = o.rotkeys(W.th_rotations(*split))
    S = prm.slots
    diags = W.banded_diagonals(132, S, range(S))
    _onfly_case(prm, o, keys, prm.max_level, split, {t: diags[t] for t in range(S)}, W.input_vector(133, S), 134,
                tol=1e-4, pt_scale=float(prm.q[prm.max_level]))


def test_encode_and_onfly_argument_errors():
    import torch
    prm = W.params_toy()
    P = gpu_params(prm)
    S, delta = prm.slots, 2.0 ** prm.log_delta
    K = prm.alpha + prm.max_level + 1
    z = _slots_tensor(W.complex_uniform(W.rng(5, 0), S))
    out = H.empty((K, prm.n))
    wsb = H.ckks_encode_workspace_size(P, 1)
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device="cuda")
    H.ckks_encode(P, [], [], delta, 0, K, [], ws, wsb)  # nothing to do
    for scale, first, nl in ((0.0, 0, K), (-1.0, 0, K), (float("inf"), 0, K), (delta, 0, K + 1), (delta, -1, 2),
                             (delta, 0, 0)):
        with pytest.raises(H.CkksError) as e:
            H.ckks_encode(P, [z], [0], scale, first, nl, [out], ws, wsb)
        assert e.value.code == H.CKKS_E_INVALID_ARG
    with pytest.raises(H.CkksError) as e:
        H.ckks_encode(P, [z], [0], delta, 0, K, [out], ws, 0)
    assert e.value.code == H.CKKS_E_WORKSPACE
    # pt and slots together are refused
    d, keep = H._diags((2, 2, 1), [z] * 4, delta, onfly=True)
    d.pt = d.slots
    import ctypes
    n = ctypes.c_size_t()
    assert H.lib().ckks_lt_workspace_size(P, 1, ctypes.byref(d), H.CKKS_LT_TH_BSGS, ctypes.byref(n)) == \
        H.CKKS_E_INVALID_ARG
    torch.cuda.synchronize()


def test_onfly_mixed_ragged_batch_and_graph():
    # One ragged batch: items with resident plaintexts and items whose
    # diagonals are encoded on the fly, at different levels and splits.  Each
    # item equals its evaluation alone (and the oracle given the device's
    # encodings); the batch captured in a HIP graph replays to the same bytes.
    import torch
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(141)
    S, delta = prm.slots, 2.0 ** prm.log_delta
    K = prm.alpha + prm.max_level + 1
    P = gpu_params(prm)
    specs = [(2, 16, (2, 2, 4), True), (1, 12, (4, 1, 4), False), (2, 30, (2, 4, 4), True), (1, 5, (1, 4, 2), False)]
    rots = set()
    for _, _, split, _ in specs:
        rots |= set(W.th_rotations(*split))
    keys = o.rotkeys(sorted(rots))
    dkeys = {r: limbs_tensor(k) for r, k in keys.items()}
    batch, refs, keep = [], [], []
    for i, (level, nd, split, onfly) in enumerate(specs):
        diags = W.banded_diagonals(150 + i, S, range(nd))
        v = W.input_vector(160 + i, S)
        ct = o.encrypt(level, v, delta, seed=170 + i)
        n = int(np.prod(split))
        pre = _pre_rotations("th", split, n, 1, 0, S)
        enc, _ = _encode(P, prm, [diags[t] for t in range(nd)], [pre[t] for t in range(nd)], delta, 0, K)
        pts = enc + [None] * (n - nd)
        refs.append(o.lt_th(level, ct, split, pts, keys))
        c0, c1 = limbs_tensor(ct[0]), limbs_tensor(ct[1])
        items = [_slots_tensor(diags[t]) for t in range(nd)] if onfly else [limbs_tensor(f) for f in enc]
        keep += [c0, c1, items]
        batch.append(H.BatchItem(level, delta, c0, c1, split, items, delta, dkeys, H.empty((level, prm.n)),
                                 H.empty((level, prm.n)), onfly=onfly))
    wsb = H.ckks_lt_batch_workspace_size(P, batch, H.CKKS_LT_TH_BSGS)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def outputs():
        return [np.stack([H.to_host(b.out0), H.to_host(b.out1)]) for b in batch]

    log("mixed batch, workspace", wsb)
    assert H.ckks_lt_eval_batch(P, batch, H.CKKS_LT_TH_BSGS, ws, wsb) == H.CKKS_OK
    torch.cuda.synchronize()
    eager = outputs()
    for i, (e, ref) in enumerate(zip(eager, refs)):
        assert batch[i].status == H.CKKS_OK
        assert np.array_equal(e, ref), i
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
        for b in batch:
            b.out0.fill_(7)
            b.out1.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, x in zip(eager, outputs()):
            assert np.array_equal(e, x), rep


def test_onfly_random_configurations():
    # Seeded random TH-/DH-BSGS configurations with slot diagonals: split,
    # level, a sparse random subset of the diagonals, stride and centre.
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(191)
    S = prm.slots
    rng = np.random.Generator(np.random.PCG64(192))
    cases = []
    for c in range(12):
        algo = "th" if c % 3 else "dh"
        split = tuple(int(x) for x in rng.choice([1, 2, 4], size=3 if algo == "th" else 2))
        n = int(np.prod(split))
        stride = int(rng.choice([1, 1, 3, 5, 16]))
        centre = int(rng.integers(0, n))
        level = int(rng.integers(1, prm.max_level + 1))
        present = sorted(set(int(t) for t in rng.choice(n, size=int(rng.integers(1, n + 1)))))
        cases.append((algo, split, stride, centre, level, present))
    rots = set()
    for algo, split, stride, centre, _, _ in cases:
        th_split = split if algo == "th" else (1,) + split
        rots |= set(W.th_rotations(*th_split, stride=stride, centre=centre, slots=S))
    keys = o.rotkeys(sorted(rots))
    for c, (algo, split, stride, centre, level, present) in enumerate(cases):
        offs = {t: (stride * (t - centre)) % S for t in present}
        dg = W.banded_diagonals(200 + c, S, sorted(offs.values()))
        log("case", c, algo, split, "stride", stride, "centre", centre, "level", level, "present", len(present))
        _onfly_case(prm, o, keys, level, split, {t: dg[offs[t]] for t in present}, W.input_vector(220 + c, S),
                    240 + c, algo=algo, stride=stride, centre=centre)


def test_onfly_bsgs_and_diagonal_method():
    # Plain BSGS (Q-basis plaintexts pre-rotated by -G_j) and the diagonal
    # method (no pre-rotation) with slot diagonals, banded and strided.
    prm = W.params_toy()
    o = O.Oracle(prm)
    o.keygen(251)
    S = prm.slots
    cases = [("bsgs", (4, 4), 1, 0, 16), ("bsgs", (8, 4), 3, 5, 20), ("naive", None, 1, 0, 12),
             ("naive", None, 5, 3, 9)]
    rots = set()
    for algo, split, stride, centre, nd in cases:
        if algo == "bsgs":
            rots |= set(W.bsgs_rotations(*split, stride=stride, centre=centre, slots=S))
        else:
            rots |= set((stride * (t - centre)) % S for t in range(nd)) - {0}
    keys = o.rotkeys(sorted(rots))
    for c, (algo, split, stride, centre, nd) in enumerate(cases):
        offs = {t: (stride * (t - centre)) % S for t in range(nd)}
        dg = W.banded_diagonals(260 + c, S, sorted(offs.values()))
        log("case", c, algo, split, "stride", stride, "centre", centre, "diagonals", nd)
        _onfly_case(prm, o, keys, 1 + c % prm.max_level, split, {t: dg[offs[t]] for t in range(nd)},
                    W.input_vector(270 + c, S), 280 + c, algo=algo, stride=stride, centre=centre, n=nd)


@pytest.mark.parametrize("which", ["set_a_n13", "n14", "n15"])
def test_encode_every_ring_size(which):
    # The FFT's two-pass split differs per ring size (A x B = N/2): N = 2^13,
    # 2^14 and 2^15 here, 2^12 and 2^16 above.
    prm = {"set_a_n13": lambda: W.params_paper_set("A"), "n14": lambda: W.params_n16(log_n=14),
           "n15": lambda: W.params_n16(log_n=15)}[which]()
    K = prm.alpha + prm.max_level + 1
    _encode_case(prm, 4, 53, [(0, K)])
