"""Server-side plan build and client-side selector build for packed lookups.

* Digit decomposition (Sec. IV-A): index i of a k-row table becomes l =
  ceil(log_p k) little-endian base-p digits i_j = floor(i / p^j) mod p, and the
  row is sum_j C_j[i_j] with l compressed p x d tables.
* Block-diagonal packing (Sec. IV-B): W_t = [C_{t,0}; ...; C_{t,l-1}]^T (or
  E_t^T for an uncompressed table), M = block_diag(W_t); the selector is the
  concatenation of every table's one-hot digits, so M s stacks the rows.
* Diagonal method with BSGS (Sec. II-A, III-B): hybrid diagonals
  u_k[j] = M[j mod m][(j+k) mod n] (m = next power of two >= rows, k < m),
  k = n1 g + b, pre-rotated v_{g,b} = rot(u_k, -n1 g), encoded at scale q_l,
  and a fold sums the m-periodic copies.
* Threshold rule (Sec. V-B): only tables with more rows than a threshold are
  compressed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import encoding


def n_digits(k: int, p: int) -> int:
    l, cap = 1, p
    while cap < k:
        l += 1
        cap *= p
    return l


def digits(i: int, p: int, l: int) -> List[int]:
    out = []
    for _ in range(l):
        out.append(i % p)
        i //= p
    return out


@dataclass
class Table:
    rows: int
    d: int
    base: Optional[int] = None                 # None: uncompressed
    parts: Optional[List[np.ndarray]] = None   # compressed C_j (p x d)
    full: Optional[np.ndarray] = None          # uncompressed E (rows x d)

    @property
    def width(self) -> int:
        return self.rows if self.base is None else self.base * len(self.parts)

    def weight_block(self) -> np.ndarray:
        if self.base is None:
            return self.full.T
        return np.vstack(self.parts).T

    def one_hot(self, i: int) -> np.ndarray:
        s = np.zeros(self.width)
        if self.base is None:
            s[i] = 1.0
        else:
            for j, dj in enumerate(digits(i, self.base, len(self.parts))):
                s[j * self.base + dj] = 1.0
        return s

    def row(self, i: int) -> np.ndarray:
        if self.base is None:
            return self.full[i]
        return sum(self.parts[j][dj] for j, dj in enumerate(digits(i, self.base, len(self.parts))))


def compress_rule(rows: int, threshold: int) -> bool:
    return rows > threshold


def packed_matrix(tables: Sequence[Table]) -> np.ndarray:
    blocks = [t.weight_block() for t in tables]
    M = np.zeros((sum(b.shape[0] for b in blocks), sum(b.shape[1] for b in blocks)))
    r = c = 0
    for b in blocks:
        M[r:r + b.shape[0], c:c + b.shape[1]] = b
        r += b.shape[0]
        c += b.shape[1]
    return M


def packed_selector(tables: Sequence[Table], idx: Sequence[int]) -> np.ndarray:
    return np.concatenate([t.one_hot(i) for t, i in zip(tables, idx)])


def next_pow2(x: int) -> int:
    return 1 << max(0, (int(x) - 1).bit_length())


def fold_stages(n: int, m: int, radix: int) -> List[Tuple[int, int]]:
    out, span = [], n
    while span > m:
        r = min(radix, span // m)
        out.append((span // r, r))
        span //= r
    return out


def bsgs_diagonals(M: np.ndarray, n: int, n1: int, sign: int = 1) -> Tuple[int, int, Dict[int, np.ndarray]]:
    """Non-zero hybrid diagonals u_k[j] = M[j mod m][(j + sign k) mod n],
    pre-rotated for BSGS (v = rot(u_k, -sign n1 g)), keyed by k = n1 g + b."""
    rows, cols = M.shape
    if cols > n:
        raise ValueError(f"matrix has {cols} columns, more than the {n} slots")
    m = next_pow2(rows)
    n2 = -(-m // n1)
    j = np.arange(n)
    R = np.zeros((m, n))
    R[:rows, :cols] = M
    out = {}
    for k in range(m):
        u = R[j % m, (j + sign * k) % n]
        if not u.any():
            continue
        g = k // n1
        out[k] = np.roll(u, sign * n1 * g)     # rot(u, -sign n1 g)
    return m, n2, out


def fold_span(rows: int, cols: int, n: int, sign: int) -> int:
    """With sign -1 the partial sums occupy [0, cols + m - 1) without wrapping,
    so the fold only has to cover the next power of two above that."""
    if sign == 1:
        return n
    return min(n, next_pow2(cols + next_pow2(rows) - 1))


@dataclass
class PlanSpec:
    level: int
    m: int
    n1: int
    n2: int
    radix: int
    diag: List[int]
    coeffs: np.ndarray            # int64 [n_diag][N]
    rows: int
    stages: List[Tuple[int, int]] = field(default_factory=list)
    sign: int = 1
    span: int = 0

    def rotation_steps(self) -> List[int]:
        st = set()
        for k in self.diag:
            g, b = divmod(k, self.n1)
            if b:
                st.add(self.sign * b)
            if g:
                st.add(self.sign * self.n1 * g)
        for s, r in self.stages:
            st.update(t * s for t in range(1, r))
        return sorted(st)


def make_plan(M: np.ndarray, N: int, level: int, scale: float, n1: int, radix: int = 2,
              sign: int = -1) -> PlanSpec:
    n = N // 2
    m, n2, vals = bsgs_diagonals(M, n, n1, sign)
    diag = sorted(vals)
    coeffs = np.stack([encoding.encode(vals[k], scale, N) for k in diag]) if diag else np.zeros((0, N), np.int64)
    span = fold_span(M.shape[0], M.shape[1], n, sign)
    return PlanSpec(level=level, m=m, n1=n1, n2=n2, radix=radix, diag=diag, coeffs=coeffs,
                    rows=M.shape[0], stages=fold_stages(span, m, radix), sign=sign, span=span)


def make_multi_plan(M: np.ndarray, N: int, level: int, scale: float, n1: int, radix: int = 2,
                    sign: int = -1) -> List[PlanSpec]:
    """A packed matrix wider than the N/2 slots of one ciphertext (Sec. III-C):
    one plan per block of N/2 columns, all folding over the widest block's
    span so their products can be summed before the fold."""
    n = N // 2
    blocks = [M[:, c:c + n] for c in range(0, M.shape[1], n)]
    span = max(fold_span(B.shape[0], B.shape[1], n, sign) for B in blocks)
    specs = []
    for B in blocks:
        sp = make_plan(B, N, level, scale, n1, radix, sign)
        sp.span = span
        sp.stages = fold_stages(span, sp.m, radix)
        specs.append(sp)
    return specs


def galois(step: int, N: int) -> int:
    return pow(5, step % (N // 2), 2 * N)
