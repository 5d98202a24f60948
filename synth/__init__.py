"""Seeded synthetic inputs shared by the CPU oracle and the GPU library's callers.

This module draws random numbers and nothing else: it holds none of the CKKS or
lookup arithmetic.  Everything the method randomises (the ternary secret, the
Gaussian errors, the uniform key/public-key polynomials, the encryption
randomness) is drawn here and handed to whichever side does the arithmetic, so
both sides consume identical randomness by construction.  Synthetic embedding
tables and query indices are drawn here too; the method's own client steps
(digit decomposition, one-hot packing, encoding) are done by each side itself.

Generator: numpy ``Generator(PCG64(seed))``.  Draw order for key material is
fixed by :class:`KeyDraws` (secret, public key, then one switching key per
Galois element in ascending order, then the relinearisation key if asked).
The uniform polynomials of switching keys are not drawn here: a switching key
gets a 64-bit seed, which the oracle and the library each expand with their
own implementation of the counter-based generator that both follow.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

SIGMA = 3.2          # error standard deviation (CKKS convention)
ERR_BOUND = 19       # errors are resampled until |e| <= 19 (about 6 sigma)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ternary(g: np.random.Generator, n: int) -> np.ndarray:
    """n coefficients uniform in {-1, 0, 1} (int64)."""
    return g.integers(-1, 2, size=n, dtype=np.int64)


def gaussian(g: np.random.Generator, n: int, sigma: float = SIGMA,
             bound: int = ERR_BOUND) -> np.ndarray:
    """Rounded normal samples, resampled until every |e| <= bound (int64)."""
    e = np.rint(g.normal(0.0, sigma, size=n)).astype(np.int64)
    bad = np.abs(e) > bound
    while bad.any():
        e[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(e) > bound
    return e


def uniform_residues(g: np.random.Generator, moduli: Sequence[int], n: int) -> np.ndarray:
    """One row per modulus, each entry uniform in [0, modulus) (uint64)."""
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for r, q in enumerate(moduli):
        out[r] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


@dataclass
class SwitchKeyDraws:
    """Randomness of one switching key: the 64-bit seed of its uniform
    polynomials (each side expands it with the same published counter-based
    generator, so a key need not store them) and one error per digit."""
    a_seed: int            # seed of the uniform part a_j of every digit j
    e: np.ndarray          # int64  [dnum][N]


@dataclass
class KeyDraws:
    s: np.ndarray                      # int64 [N], ternary secret
    pk_a: np.ndarray                   # uint64 [L+1][N]
    pk_e: np.ndarray                   # int64 [N]
    swk: Dict[int, SwitchKeyDraws] = field(default_factory=dict)  # galois -> draws
    relin: SwitchKeyDraws | None = None


def key_draws(seed: int, N: int, q_moduli: Sequence[int], p_moduli: Sequence[int],
              dnum: int, galois: Sequence[int], relin: bool = False) -> KeyDraws:
    """All key randomness for one parameter set, in the fixed draw order."""
    g = rng(seed)
    s = ternary(g, N)
    pk_a = uniform_residues(g, q_moduli, N)
    pk_e = gaussian(g, N)
    kd = KeyDraws(s=s, pk_a=pk_a, pk_e=pk_e)
    for gal in sorted(set(int(x) for x in galois)):
        seed = int(g.integers(0, 1 << 63))
        e = np.stack([gaussian(g, N) for _ in range(dnum)])
        kd.swk[gal] = SwitchKeyDraws(a_seed=seed, e=e)
    if relin:
        seed = int(g.integers(0, 1 << 63))
        e = np.stack([gaussian(g, N) for _ in range(dnum)])
        kd.relin = SwitchKeyDraws(a_seed=seed, e=e)
    return kd


@dataclass
class EncDraws:
    v: np.ndarray     # int64 [N] ternary
    e0: np.ndarray    # int64 [N]
    e1: np.ndarray    # int64 [N]


def enc_draws(g: np.random.Generator, N: int) -> EncDraws:
    v = ternary(g, N)
    e0 = gaussian(g, N)
    e1 = gaussian(g, N)
    return EncDraws(v=v, e0=e0, e1=e1)


# ---------------------------------------------------------------- workloads

def uniform_table(g: np.random.Generator, rows: int, d: int, lo: float, hi: float) -> np.ndarray:
    return g.uniform(lo, hi, size=(rows, d))


def loguniform_row_counts(g: np.random.Generator, n_tables: int, lo: float, hi: float) -> List[int]:
    """Row counts round(exp(U(ln lo, ln hi))) per table."""
    return [int(round(float(np.exp(g.uniform(np.log(lo), np.log(hi)))))) for _ in range(n_tables)]


def criteo_like_row_counts(n_tables: int = 26, lo: float = 4.0, hi: float = 1e7,
                           total_lo: float = 3.0e7, total_hi: float = 3.8e7):
    """Seeded 26-table row counts, log-uniform in [lo, hi]: seeds 0, 1, 2, ... are
    tried in order and the first draw whose total lies in [total_lo, total_hi]
    is kept.  Returns (seed, counts)."""
    seed = 0
    while True:
        counts = loguniform_row_counts(rng(seed), n_tables, lo, hi)
        if total_lo <= sum(counts) <= total_hi:
            return seed, counts
        seed += 1


def indices(g: np.random.Generator, row_counts: Sequence[int]) -> List[int]:
    """One uniform index per table; row counts of 2^62 or more (digit-encoded
    vocabularies such as 16^32) are drawn 62 bits at a time with rejection."""
    out = []
    for k in row_counts:
        k = int(k)
        if k < 1 << 62:
            out.append(int(g.integers(0, k)))
            continue
        nbits = (k - 1).bit_length()
        while True:
            v, got = 0, 0
            while got < nbits:
                take = min(62, nbits - got)
                v |= int(g.integers(0, 1 << take)) << got
                got += take
            if v < k:
                out.append(v)
                break
    return out


def poisson_arrivals(g: np.random.Generator, rate: float, n: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    return np.cumsum(g.exponential(1.0 / rate, size=n))


@dataclass
class SmallDLRMDraws:
    """Weights of the small DLRM: embedding tables (rows U{2..200} x d,
    values U[lo, hi]), dense layers (weights and biases N(0, sigma^2))."""
    table_rows: List[int]
    tables: List[np.ndarray]
    bottom: List[Tuple[np.ndarray, np.ndarray]]
    top: List[Tuple[np.ndarray, np.ndarray]]
    n_dense: int


def small_dlrm_draws(seed: int = 0, n_tables: int = 8, n_dense: int = 13, d: int = 16,
                     bottom: Sequence[int] = (64, 16), top: Sequence[int] = (32, 1),
                     rows_lo: int = 2, rows_hi: int = 200, lo: float = -0.05, hi: float = 0.05,
                     sigma: float = 0.1) -> SmallDLRMDraws:
    g = rng(seed)
    rows = [int(r) for r in g.integers(rows_lo, rows_hi + 1, size=n_tables)]
    tables = [uniform_table(g, r, d, lo, hi) for r in rows]
    layers_b, prev = [], n_dense
    for w in bottom:
        layers_b.append((g.normal(0.0, sigma, (w, prev)), g.normal(0.0, sigma, w)))
        prev = w
    layers_t, prev = [], n_tables * d + bottom[-1]
    for w in top:
        layers_t.append((g.normal(0.0, sigma, (w, prev)), g.normal(0.0, sigma, w)))
        prev = w
    return SmallDLRMDraws(table_rows=rows, tables=tables, bottom=layers_b, top=layers_t, n_dense=n_dense)


def dense_features(g: np.random.Generator, n_dense: int) -> np.ndarray:
    return g.uniform(0.0, 1.0, n_dense)
