"""Independent big-integer helpers for pinning the oracle (Python ints only)."""
from __future__ import annotations

import functools
from typing import List, Sequence

import numpy as np

import workload as W


def bitrev(x: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def crt(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """The integer in [0, prod(moduli)) with the given residues."""
    M = functools.reduce(lambda a, b: a * b, moduli, 1)
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def crt_columns(limbs: np.ndarray, moduli: Sequence[int], cols: Sequence[int]) -> List[int]:
    return [crt([int(limbs[l, k]) for l in range(len(moduli))], moduli) for k in cols]


def small_params(log_n: int, nq: int = 3, np_: int = 1, dnum: int = 3, bits_q=30, bits_p=31,
                 log_delta: int = 20, h: int = 8) -> W.Params:
    """A tiny parameter set for brute-force pins (insecure)."""
    two_n = 2 << log_n
    q = W.ntt_primes(bits_q, nq, two_n)
    p = W.ntt_primes(bits_p, np_, two_n)
    return W.Params(log_n=log_n, q=tuple(q), p=tuple(p), dnum=dnum, log_delta=log_delta, h=h)


def negacyclic_schoolbook(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += ai * int(b[j])
            else:
                out[k - n] -= ai * int(b[j])
    return [x % q for x in out]


def centred(x: int, m: int) -> int:
    x %= m
    return x - m if x > m // 2 else x
