"""RNS-CKKS parameter sets (primes q = 1 mod 2N) for the lookup workloads.

Prime rule: q_0 and the K special primes are the largest primes = 1 mod 2N
below 2^60 (q_0 first, then p_0 > p_1 > ...); q_1..q_L are the L largest such
primes below 2^40, descending.  Levels drop q_L first; q_0 is never dropped.
The paper fixes only "128-bit security" and n = 2^15 slots (Sec. II-A); the
N=2^16 set below has log2(QP) = 60 + 23*40 + 8*60 = 1460 bits.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve primes as bases: exact below 2^64."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for b in _MR_BASES:
        x = pow(b, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_below(bound: int, step: int, count: int) -> List[int]:
    out = []
    c = 1 + ((bound - 2) // step) * step
    while len(out) < count:
        if c < bound and is_prime(c):
            out.append(c)
        c -= step
    return out


@dataclass
class ParamSet:
    log_n: int
    L: int
    K: int
    alpha: int
    q: List[int]
    p: List[int]
    delta: float = 2.0 ** 40

    def n_digits(self, level: int) -> int:
        """Key-switching digits at this level: ceil((level + 1) / alpha)."""
        return -(-(level + 1) // self.alpha)

    @property
    def N(self) -> int:
        return 1 << self.log_n

    @property
    def n(self) -> int:
        return self.N // 2

    @property
    def dnum(self) -> int:
        return -(-(self.L + 1) // self.alpha)

    def digit_primes(self, j: int) -> List[int]:
        return list(range(j * self.alpha, min((j + 1) * self.alpha, self.L + 1)))

    def P_mod(self, m: int) -> int:
        r = 1
        for x in self.p:
            r = r * x % m
        return r


def make(log_n: int, L: int, K: int, alpha: int) -> ParamSet:
    twoN = 2 << log_n
    top = primes_below(1 << 60, twoN, 1 + K)
    return ParamSet(log_n, L, K, alpha, [top[0]] + primes_below(1 << 40, twoN, L), top[1:])


def toy() -> ParamSet:
    """N=2^12: q_0 (60-bit), three 40-bit primes, one special prime, one prime per digit."""
    return make(12, 3, 1, 1)


def n16() -> ParamSet:
    """N=2^16: q_0 + 23 40-bit primes, dnum=3 (alpha=8), K=8 special primes."""
    return make(16, 23, 8, 8)
