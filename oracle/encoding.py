"""CKKS canonical-embedding encode / decode for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Slot t of a polynomial m(X) in Z[X]/(X^N + 1) is m(zeta^(5^t)), zeta = e^(i pi/N),
0 <= t < N/2 (Section II-A: rotation by r uses g = 5, of order N/2 mod 2N, and
moves slot t + r to slot t).  The evaluations at all odd powers zeta^(2l+1) are
one length-N DFT of m_k zeta^k, so encode and decode use numpy's FFT as a step.
Rounding is to nearest with ties away from zero.
"""
from __future__ import annotations

import numpy as np


def slot_exponents(n: int) -> np.ndarray:
    """e_t = 5^t mod 2N for t < N/2."""
    s = n // 2
    e = np.empty(s, dtype=np.int64)
    x = 1
    for t in range(s):
        e[t] = x
        x = x * 5 % (2 * n)
    return e


def _round_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode(z: np.ndarray, scale: float, n: int) -> np.ndarray:
    """Integer coefficients (int64) of round(scale * sigma^-1(z))."""
    return _round_away(encode_unrounded(z, scale, n)).astype(np.int64)


def encode_unrounded(z: np.ndarray, scale: float, n: int) -> np.ndarray:
    """scale * sigma^-1(z) as float64, before the rounding of encode()."""
    s = n // 2
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (s,)
    e = slot_exponents(n)
    w = np.zeros(n, dtype=np.complex128)
    w[(e - 1) // 2] = z
    w[(2 * n - e - 1) // 2] = np.conj(z)
    k = np.arange(n)
    zeta_neg = np.exp(-1j * np.pi * k / n)
    # m_k = (1/N) sum_l w_l zeta^-(2l+1)k = zeta^-k/N * sum_l w_l e^{-2 pi i lk/N}
    m = (np.fft.fft(w) * zeta_neg / n).real
    return m * scale


def decode(m: np.ndarray, scale: float, n: int) -> np.ndarray:
    """Slots of m(X) / scale (m given by its integer coefficients)."""
    m = np.asarray(m, dtype=np.float64)
    k = np.arange(n)
    zeta = np.exp(1j * np.pi * k / n)
    # w_l = sum_k m_k zeta^(2l+1)k = sum_k (m_k zeta^k) e^{2 pi i lk/N}
    w = np.fft.ifft(m * zeta) * n
    e = slot_exponents(n)
    return w[(e - 1) // 2] / scale


def rotate_slots(z: np.ndarray, r: int) -> np.ndarray:
    """rot(z, r)[t] = z[(t + r) mod N/2] (toward slot 0)."""
    return np.roll(z, -r)
