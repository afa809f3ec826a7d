"""CPU oracle for the RNS-CKKS homomorphic linear transformation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package.  The GPU library and its Python
binding never import, link or call it, and the two share no code.

The arithmetic lives in ckks_oracle.cpp (plain C++, 128-bit modular products,
textbook NTT, eq. (3) basis conversion, eq. (4) ModDown, eq. (1) rescale,
Algorithm 2 step by step); this module is a ctypes harness around it plus the
numpy canonical-embedding encoder in encoding.py.

Functions whose result has no independent pin say so in their docstring
("parity unpinned").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import encoding

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP over limbs)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
        L = ctypes.CDLL(_LIB)
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_ctx_create.restype = ctypes.c_void_p
        L.orc_ctx_create.argtypes = [ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_int, _u64p, ctypes.c_int]
        L.orc_ctx_destroy.argtypes = [ctypes.c_void_p]
        L.orc_psi.restype = ctypes.c_uint64
        L.orc_psi.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_galois.restype = ctypes.c_uint64
        L.orc_galois.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_counters.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_long)]
        L.orc_reset_counters.argtypes = [ctypes.c_void_p]
        for name in ["orc_ntt", "orc_intt", "orc_automorph_ntt", "orc_automorph_coeff", "orc_bconv",
                     "orc_decompose", "orc_moddown", "orc_moddown_rescale", "orc_rescale", "orc_ks_inner",
                     "orc_p_scale", "orc_poly_from_signed", "orc_keygen_secret", "orc_get_secret",
                     "orc_gen_rotkey", "orc_encrypt", "orc_decrypt", "orc_rotate", "orc_lt_th",
                     "orc_lt_bsgs", "orc_lt_naive", "orc_lt_dh"]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p if a.dtype == np.uint64 else _i64p)


def _check(rc: int):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_last_error().decode())


def _ptr_array(arrs: Sequence[Optional[np.ndarray]]):
    t = (ctypes.c_void_p * max(1, len(arrs)))()
    for i, a in enumerate(arrs):
        t[i] = None if a is None else a.ctypes.data
    return t


class Oracle:
    """One RNS-CKKS context (ring N, chain q_0..q_L, special primes p_0..p_{alpha-1})."""

    def __init__(self, params):
        self.params = params
        self.n = params.n
        self.alpha = params.alpha
        self.L = params.max_level
        q = np.array(params.q, dtype=np.uint64)
        p = np.array(params.p, dtype=np.uint64)
        self._ctx = lib().orc_ctx_create(params.log_n, len(q), _p(q), len(p), _p(p), params.dnum)
        if not self._ctx:
            raise RuntimeError("oracle: " + lib().orc_last_error().decode())
        self.pq = list(params.p) + list(params.q)   # P-first limb order

    def __del__(self):
        if getattr(self, "_ctx", None):
            lib().orc_ctx_destroy(ctypes.c_void_p(self._ctx))
            self._ctx = None

    @property
    def ctx(self):
        return ctypes.c_void_p(self._ctx)

    # ---- sizes --------------------------------------------------------------
    def K(self, level: int) -> int:
        return self.alpha + level + 1

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def q_basis(self, level: int) -> List[int]:
        return [self.alpha + j for j in range(level + 1)]

    def pq_basis(self, level: int) -> List[int]:
        return list(range(self.alpha + level + 1))

    def psi(self, pqi: int) -> int:
        return int(lib().orc_psi(self.ctx, pqi))

    def galois(self, r: int) -> int:
        return int(lib().orc_galois(self.ctx, r))

    # ---- primitives -----------------------------------------------------------
    def ntt(self, x: np.ndarray, basis: Sequence[int]) -> np.ndarray:
        out = np.ascontiguousarray(x, dtype=np.uint64).copy().reshape(len(basis), self.n)
        for l, b in enumerate(basis):
            _check(lib().orc_ntt(self.ctx, b, _p(out[l])))
        return out

    def intt(self, x: np.ndarray, basis: Sequence[int]) -> np.ndarray:
        out = np.ascontiguousarray(x, dtype=np.uint64).copy().reshape(len(basis), self.n)
        for l, b in enumerate(basis):
            _check(lib().orc_intt(self.ctx, b, _p(out[l])))
        return out

    def automorph_ntt(self, x: np.ndarray, r: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty_like(x)
        _check(lib().orc_automorph_ntt(self.ctx, r, _p(x), _p(out), x.size // self.n))
        return out

    def automorph_coeff(self, x: np.ndarray, pqi: int, g: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty_like(x)
        _check(lib().orc_automorph_coeff(self.ctx, pqi, ctypes.c_uint64(g), _p(x), _p(out)))
        return out

    def bconv(self, src: Sequence[int], x: np.ndarray, dst: Sequence[int]) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((len(dst), self.n), dtype=np.uint64)
        s = (ctypes.c_int * len(src))(*src)
        d = (ctypes.c_int * len(dst))(*dst)
        _check(lib().orc_bconv(self.ctx, len(src), s, _p(x), len(dst), d, _p(out)))
        return out

    def decompose(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((self.beta(level), self.K(level), self.n), dtype=np.uint64)
        _check(lib().orc_decompose(self.ctx, level, _p(x), _p(out)))
        return out

    def moddown(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        _check(lib().orc_moddown(self.ctx, level, _p(x), _p(out)))
        return out

    def moddown_rescale(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((level, self.n), dtype=np.uint64)
        _check(lib().orc_moddown_rescale(self.ctx, level, _p(x), _p(out)))
        return out

    def rescale(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((level, self.n), dtype=np.uint64)
        _check(lib().orc_rescale(self.ctx, level, _p(x), _p(out)))
        return out

    def ks_inner(self, level: int, digits: np.ndarray, key: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        digits = np.ascontiguousarray(digits, dtype=np.uint64)
        key = np.ascontiguousarray(key, dtype=np.uint64)
        x = np.empty((self.K(level), self.n), dtype=np.uint64)
        y = np.empty_like(x)
        _check(lib().orc_ks_inner(self.ctx, level, _p(digits), _p(key), _p(x), _p(y)))
        return x, y

    def p_scale(self, level: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty((self.K(level), self.n), dtype=np.uint64)
        _check(lib().orc_p_scale(self.ctx, level, _p(x), _p(out)))
        return out

    def poly_from_signed(self, coef: np.ndarray, basis: Sequence[int]) -> np.ndarray:
        coef = np.ascontiguousarray(coef, dtype=np.int64)
        out = np.empty((len(basis), self.n), dtype=np.uint64)
        b = (ctypes.c_int * len(basis))(*basis)
        _check(lib().orc_poly_from_signed(self.ctx, _p(coef), len(basis), b, _p(out)))
        return out

    # ---- keys, encryption ---------------------------------------------------
    def keygen(self, seed: int):
        _check(lib().orc_keygen_secret(self.ctx, ctypes.c_uint64(seed), self.params.h))
        self.seed = seed

    def secret(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _check(lib().orc_get_secret(self.ctx, _p(out)))
        return out

    def rotkey(self, r: int) -> np.ndarray:
        """swk~_r = phi_{-r}(swk_r), layout [beta_max][2][K_max][N], NTT form."""
        out = np.empty((self.beta(self.L), 2, self.K(self.L), self.n), dtype=np.uint64)
        _check(lib().orc_gen_rotkey(self.ctx, r, ctypes.c_uint64(self.seed), ctypes.c_double(self.params.sigma),
                                    _p(out)))
        return out

    def rotkeys(self, rots: Sequence[int]) -> Dict[int, np.ndarray]:
        S = self.n // 2
        return {int(r) % S: self.rotkey(int(r)) for r in rots}

    def encrypt_coeffs(self, level: int, m: np.ndarray, seed: int) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.int64)
        ct = np.empty((2, level + 1, self.n), dtype=np.uint64)
        _check(lib().orc_encrypt(self.ctx, level, _p(m), ctypes.c_uint64(seed), ctypes.c_double(self.params.sigma),
                                 _p(ct[0]), _p(ct[1])))
        return ct

    def encrypt(self, level: int, z: np.ndarray, scale: float, seed: int) -> np.ndarray:
        return self.encrypt_coeffs(level, encoding.encode(z, scale, self.n), seed)

    def decrypt(self, ct: np.ndarray) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        m = np.empty(self.n, dtype=np.int64)
        _check(lib().orc_decrypt(self.ctx, _p(np.ascontiguousarray(ct[0][0])), _p(np.ascontiguousarray(ct[1][0])),
                                 _p(m)))
        return m

    def decrypt_slots(self, ct: np.ndarray, scale: float) -> np.ndarray:
        return encoding.decode(self.decrypt(ct), scale, self.n)

    # ---- plaintext diagonals -------------------------------------------------
    def encode_plain(self, z: np.ndarray, scale: float, basis: Sequence[int]) -> np.ndarray:
        return self.poly_from_signed(encoding.encode(z, scale, self.n), basis)

    def plaintexts(self, diags: Dict[int, np.ndarray], idx_of: Dict[int, int], giant_of: Dict[int, int],
                   n_idx: int, scale: float, basis: Sequence[int]) -> List[Optional[np.ndarray]]:
        """f^_m = phi_{-G}(encode(diag)) for every plaintext index m.

        idx_of maps a cyclic diagonal offset to its index m; giant_of maps m to
        the giant-step rotation G folded into its plaintext."""
        out: List[Optional[np.ndarray]] = [None] * n_idx
        for d, z in diags.items():
            m = idx_of[d]
            f = self.encode_plain(z, scale, basis)
            G = giant_of.get(m, 0) % (self.n // 2)
            out[m] = self.automorph_ntt(f, -G) if G else f
        return out

    def _prog_index(self, diags, n: int, stride: int, centre: int) -> Dict[int, int]:
        """Index t of each cyclic offset d = stride (t - centre) mod S."""
        S = self.n // 2
        idx = {}
        for t in range(n):
            d = (stride * (t - centre)) % S
            assert d not in idx, "the progression repeats an offset"
            idx[d] = t
        missing = [d for d in diags if d % S not in idx]
        assert not missing, "diagonal offsets outside the progression: %r" % missing[:4]
        return {d: idx[d % S] for d in diags}

    def th_plaintexts(self, diags, n1: int, n2: int, n3: int, scale: float, stride: int = 1, centre: int = 0):
        """Algorithm 2 input: f^_{n1 n2 k + n1 j + i} = phi_{-G_k}(f), at PQ (K_max
        limbs), G_k = stride (n1 n2 k - centre); index t holds offset stride (t - centre)."""
        n = n1 * n2 * n3
        idx_of = self._prog_index(diags, n, stride, centre)
        giant_of = {m: stride * (n1 * n2 * (m // (n1 * n2)) - centre) for m in range(n)}
        return self.plaintexts(diags, idx_of, giant_of, n, scale, self.pq_basis(self.L))

    def bsgs_plaintexts(self, diags, n1: int, n2: int, scale: float, stride: int = 1, centre: int = 0):
        """Eq. (5) input: f^_{n1 j + i} = phi_{-G_j}(f), at Q (L+1 limbs), G_j = stride (n1 j - centre)."""
        n = n1 * n2
        idx_of = self._prog_index(diags, n, stride, centre)
        giant_of = {m: stride * (n1 * (m // n1) - centre) for m in range(n)}
        return self.plaintexts(diags, idx_of, giant_of, n, scale, self.q_basis(self.L))

    def naive_plaintexts(self, diags, scale: float, stride: int = 1, centre: int = 0, n: int = None):
        if n is None:
            n = max(diags) + 1
        idx_of = self._prog_index(diags, n, stride, centre)
        return self.plaintexts(diags, idx_of, {}, n, scale, self.q_basis(self.L))

    # ---- linear transformations -----------------------------------------------
    @staticmethod
    def _keys(keys: Dict[int, np.ndarray]):
        rots = sorted(keys)
        r = (ctypes.c_long * max(1, len(rots)))(*rots)
        ptrs = _ptr_array([np.ascontiguousarray(keys[k]) for k in rots])
        return len(rots), r, ptrs

    def _trunc(self, pts):
        return [None if f is None else np.ascontiguousarray(f) for f in pts]

    def lt_th(self, level: int, ct: np.ndarray, split: Tuple[int, int, int], pts, keys, stride: int = 1,
              centre: int = 0) -> np.ndarray:
        n1, n2, n3 = split
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty((2, level, self.n), dtype=np.uint64)
        pts = self._trunc(pts)
        nk, r, kp = self._keys(keys)
        _check(lib().orc_lt_th(self.ctx, level, _p(ct[0]), _p(ct[1]), n1, n2, n3, ctypes.c_long(stride),
                               ctypes.c_long(centre), len(pts), _ptr_array(pts),
                               nk, r, kp, _p(out[0]), _p(out[1])))
        return out

    def dh_plaintexts(self, diags, n1: int, n2: int, scale: float, stride: int = 1, centre: int = 0):
        """Algorithm 1 input: f^_{n1 j + i} = phi_{-G_j}(f), G_j = stride (n1 j - centre), at PQ.
        The same encodings as Algorithm 2's with an empty inner layer (n1' = 1)."""
        return self.th_plaintexts(diags, 1, n1, n2, scale, stride, centre)

    def lt_dh(self, level: int, ct: np.ndarray, split: Tuple[int, int], pts, keys, stride: int = 1,
              centre: int = 0, combined: bool = True) -> np.ndarray:
        """Double-hoisted BSGS (Algorithm 1), n1 baby and n2 giant steps."""
        n1, n2 = split
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty((2, level, self.n), dtype=np.uint64)
        pts = self._trunc(pts)
        nk, r, kp = self._keys(keys)
        _check(lib().orc_lt_dh(self.ctx, level, _p(ct[0]), _p(ct[1]), n1, n2, ctypes.c_long(stride),
                               ctypes.c_long(centre), 1 if combined else 0, len(pts), _ptr_array(pts),
                               nk, r, kp, _p(out[0]), _p(out[1])))
        return out

    def lt_bsgs(self, level: int, ct: np.ndarray, split: Tuple[int, int], pts, keys, stride: int = 1,
                centre: int = 0) -> np.ndarray:
        n1, n2 = split
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty((2, level, self.n), dtype=np.uint64)
        pts = self._trunc(pts)
        nk, r, kp = self._keys(keys)
        _check(lib().orc_lt_bsgs(self.ctx, level, _p(ct[0]), _p(ct[1]), n1, n2, ctypes.c_long(stride),
                                 ctypes.c_long(centre), len(pts), _ptr_array(pts),
                                 nk, r, kp, _p(out[0]), _p(out[1])))
        return out

    def lt_naive(self, level: int, ct: np.ndarray, pts, keys, stride: int = 1, centre: int = 0) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty((2, level, self.n), dtype=np.uint64)
        pts = self._trunc(pts)
        nk, r, kp = self._keys(keys)
        _check(lib().orc_lt_naive(self.ctx, level, _p(ct[0]), _p(ct[1]), ctypes.c_long(stride),
                                  ctypes.c_long(centre), len(pts), _ptr_array(pts),
                                  nk, r, kp, _p(out[0]), _p(out[1])))
        return out

    def rotate(self, level: int, ct: np.ndarray, r: int, keys) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty_like(ct)
        nk, rr, kp = self._keys(keys)
        _check(lib().orc_rotate(self.ctx, level, _p(ct[0]), _p(ct[1]), r, nk, rr, kp, _p(out[0]), _p(out[1])))
        return out

    def counters(self) -> Dict[str, int]:
        a = (ctypes.c_long * 6)()
        lib().orc_counters(self.ctx, a)
        return dict(zip(["decompose", "moddown", "ks", "ntt", "intt", "keys"], list(a)))

    def reset_counters(self):
        lib().orc_reset_counters(self.ctx)
