"""Seeded synthetic workloads for the triple-hoisted BSGS linear transformation.

This module is shared by the tests, the benchmark and the CPU oracle.  It holds
no CKKS arithmetic: it only chooses parameters (NTT-friendly primes, split
sizes, diagonal offsets) and draws the seeded random inputs that the
homomorphic computation consumes (matrix diagonals, input vectors, arbitrary
uniform residues for throughput runs).

Parameter recipe (the paper fixes none of this; see its Table V for the kind of
parameter sets it evaluates):
  * primes are NTT-friendly, q = 1 mod 2*N_max.  For each bit size w the
    candidates 2^w - k*2N_max + 1, k = 1, 2, ..., are tested in order and the
    primes found are assigned in order (q0 first, then the special primes p_i
    of the same size, then the remaining q_j).
  * diagonals follow the Halevi-Shoup convention diag_d[t] = M[t][(t+d) mod S].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# NTT-friendly primes (parameter selection, not part of the LT arithmetic)
# ----------------------------------------------------------------------------

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin, exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, count: int, two_n: int) -> List[int]:
    """The first `count` primes of the form 2^bits - k*two_n + 1, k = 1, 2, ..."""
    out = []
    k = 1
    while len(out) < count:
        c = (1 << bits) - k * two_n + 1
        if c < (1 << (bits - 1)):
            raise ValueError("ran out of %d-bit candidates" % bits)
        if is_prime(c):
            out.append(c)
        k += 1
    return out


@dataclasses.dataclass(frozen=True)
class Params:
    """An RNS-CKKS parameter set: Q = q_0..q_L, P = p_0..p_{alpha-1}."""
    log_n: int
    q: Tuple[int, ...]
    p: Tuple[int, ...]
    dnum: int
    log_delta: int
    h: int            # Hamming weight of the ternary secret
    sigma: float = 3.2

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def slots(self) -> int:
        return self.n // 2

    @property
    def max_level(self) -> int:
        return len(self.q) - 1

    @property
    def alpha(self) -> int:
        return len(self.p)

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def k(self, level: int) -> int:
        """Number of PQ limbs at this level."""
        return self.alpha + level + 1

    def with_log_n(self, log_n: int) -> "Params":
        return dataclasses.replace(self, log_n=log_n)


def params_toy() -> Params:
    """N = 2^12, Delta = 2^30; q0 of 50 bits, two 30-bit primes, one 50-bit
    special prime, dnum = 3; h = 64.  Toy and insecure."""
    two_n = 1 << 13
    p50 = ntt_primes(50, 2, two_n)
    p30 = ntt_primes(30, 2, two_n)
    return Params(log_n=12, q=(p50[0], p30[0], p30[1]), p=(p50[1],), dnum=3,
                  log_delta=30, h=64)


def params_n16(log_n: int = 16) -> Params:
    """N = 2^16 (or a smaller ring over the same chain), Delta = 2^40, level 24:
    q0 of 60 bits, 24 primes of 40 bits, alpha = 9 special primes of 60 bits,
    dnum = 3; h = 192.  All primes are 1 mod 2^17, so one chain serves
    N in {2^14, 2^15, 2^16}."""
    two_n = 1 << 17
    p60 = ntt_primes(60, 10, two_n)
    p40 = ntt_primes(40, 24, two_n)
    return Params(log_n=log_n, q=tuple([p60[0]] + p40), p=tuple(p60[1:]),
                  dnum=3, log_delta=40, h=192)


# The paper's evaluation sets (N, L+1, alpha, beta; w = 54-bit words) with the
# dense LT dimension n = N/2 (Table V) and the TH-BSGS split of Table VII.
PAPER_SETS = {
    "A": dict(log_n=13, n_q=5, alpha=5, dnum=1, split=(16, 16, 16)),
    "B": dict(log_n=15, n_q=16, alpha=8, dnum=2, split=(32, 16, 32)),
    "C": dict(log_n=16, n_q=32, alpha=12, dnum=3, split=(32, 32, 32)),
}


def params_paper_set(name: str) -> Params:
    """Set-A/B/C: every prime 54 bits and 1 mod 2N (N of the set), Delta =
    2^40, h = 192.  alpha special primes; the digits have alpha primes each
    (beta = ceil((L+1)/alpha) = dnum)."""
    s = PAPER_SETS[name]
    two_n = 1 << (s["log_n"] + 1)
    p54 = ntt_primes(54, s["n_q"] + s["alpha"], two_n)
    return Params(log_n=s["log_n"], q=tuple(p54[:s["n_q"]]), p=tuple(p54[s["n_q"]:]), dnum=s["dnum"],
                  log_delta=40, h=192)


# ----------------------------------------------------------------------------
# Splits (n1', n2', n3') and rotation sets
# ----------------------------------------------------------------------------

def th_rotations(n1: int, n2: int, n3: int, stride: int = 1, centre: int = 0, slots: int = None) -> List[int]:
    """Rotations whose keys TH-BSGS uses: s*i (inner), s*n1*j (middle) and the
    non-zero G_k = s*(n1*n2*k - centre) (outer), reduced mod slots if given."""
    r = [stride * i for i in range(1, n1)]
    r += [stride * n1 * j for j in range(1, n2)]
    r += [stride * (n1 * n2 * k - centre) for k in range(n3)]
    if slots:
        r = [x % slots for x in r]
    return sorted(set(x for x in r if x != 0))


def bsgs_rotations(n1: int, n2: int, stride: int = 1, centre: int = 0, slots: int = None) -> List[int]:
    r = [stride * i for i in range(1, n1)] + [stride * (n1 * j - centre) for j in range(n2)]
    if slots:
        r = [x % slots for x in r]
    return sorted(set(x for x in r if x != 0))


# ----------------------------------------------------------------------------
# Seeded inputs
# ----------------------------------------------------------------------------

def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def complex_uniform(g: np.random.Generator, size: int) -> np.ndarray:
    """Real and imaginary parts i.i.d. U[-1, 1]."""
    return g.uniform(-1.0, 1.0, size) + 1j * g.uniform(-1.0, 1.0, size)


def banded_diagonals(seed: int, slots: int, offsets: Sequence[int]) -> Dict[int, np.ndarray]:
    """Cyclic diagonals diag_d (d in offsets), entries complex U[-1,1]."""
    g = rng(seed, 1)
    return {int(d) % slots: complex_uniform(g, slots) for d in offsets}


def input_vector(seed: int, slots: int) -> np.ndarray:
    return complex_uniform(rng(seed, 2), slots)


def matvec(diags: Dict[int, np.ndarray], v: np.ndarray) -> np.ndarray:
    """FP64 M*v with M given by its cyclic diagonals: (Mv)[t] = sum_d diag_d[t] v[t+d]."""
    out = np.zeros_like(v)
    for d, dv in diags.items():
        out += dv * np.roll(v, -d)
    return out


def uniform_residues(seed: int, moduli: Sequence[int], n: int) -> np.ndarray:
    """[len(moduli)][n] uint64 residues, uniform in [0, q) per row."""
    g = rng(seed, 3)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, q, n, dtype=np.uint64)
    return out


@dataclasses.dataclass
class LTWorkload:
    """One LT evaluation: parameters, level, matrix diagonals, vector, splits."""
    name: str
    params: Params
    level: int
    diags: Dict[int, np.ndarray]
    vector: np.ndarray
    th_split: Tuple[int, int, int]
    bsgs_split: Tuple[int, int]
    seed: int

    @property
    def n_diag(self) -> int:
        return max(self.diags) + 1 if self.diags else 0


def workload_toy(seed: int = 0) -> LTWorkload:
    """2048x2048 matrix with 16 consecutive diagonals (offsets 0..15), TH (2,2,4),
    BSGS (4,4), one ciphertext at level 2."""
    prm = params_toy()
    return LTWorkload("toy_n12_d16", prm, prm.max_level,
                      banded_diagonals(seed, prm.slots, range(16)),
                      input_vector(seed, prm.slots), (2, 2, 4), (4, 4), seed)


def workload_n16(seed: int = 1, n_diag: int = 64, level: int = 24,
                 th_split=(4, 4, 4), bsgs_split=(8, 8), log_n: int = 16) -> LTWorkload:
    """N = 2^16 single LT: banded matrix with n_diag diagonals (offsets 0..n_diag-1)."""
    prm = params_n16(log_n)
    return LTWorkload("n%d_l%d_d%d" % (log_n, level, n_diag), prm, level,
                      banded_diagonals(seed, prm.slots, range(n_diag)),
                      input_vector(seed, prm.slots), tuple(th_split), tuple(bsgs_split), seed)


@dataclasses.dataclass
class ChainStage:
    """One sparse LT of a chain: cyclic diagonals and the TH split over the
    progression offset(t) = stride (t - centre), t < n1 n2 n3."""
    diags: Dict[int, np.ndarray]
    split: Tuple[int, int, int]
    stride: int
    centre: int


def phase_diagonals(seed: int, slots: int, offsets: Sequence[int]) -> Dict[int, np.ndarray]:
    """Diagonals with unit-modulus entries e^{i theta}, theta ~ U[0, 2 pi);
    offsets that coincide mod slots are merged by adding their entries."""
    g = rng(seed, 4)
    out: Dict[int, np.ndarray] = {}
    for d in offsets:
        z = np.exp(1j * g.uniform(0.0, 2.0 * np.pi, slots))
        k = int(d) % slots
        out[k] = out[k] + z if k in out else z
    return out


def dft_chain(seed: int, params: Params, radix: int = 16, half: int = 7, stages: int = 4) -> List[ChainStage]:
    """Factored DFT-like chain: stage s has diagonals at j radix^s, |j| <= half.

    Stages whose offsets do not wrap use the centred progression with stride
    radix^s, centre = 2 n1 n2 with split (2, 2, 4) (16 indices, the first one
    empty).  When the offsets wrap modulo the slot count they are merged; the
    distinct ones form the progression stride * t, t < count, run with the
    smallest near-cube split holding them."""
    S = params.slots
    out = []
    for s in range(stages):
        stride = radix ** s
        offs = [j * stride for j in range(-half, half + 1)]
        diags = phase_diagonals(seed * 100 + s, S, offs)
        if stride * (2 * half + 1) <= S:
            out.append(ChainStage(diags, (2, 2, 4), stride, 8))
        else:
            g = math.gcd(stride, S)
            period = S // g  # distinct multiples of stride mod S
            ks = sorted(diags)
            assert all(k % g == 0 for k in ks) and len(ks) <= period
            cnt = len(ks)
            split = (2, 2, 2) if cnt <= 8 else (2, 4, 4)
            out.append(ChainStage(diags, split, stride, 0))
    return out


def chain_matvec(stages: Sequence[ChainStage], v: np.ndarray) -> np.ndarray:
    for st in stages:
        v = matvec(st.diags, v)
    return v
