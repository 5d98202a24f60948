"""Oracle-side construction of the synthetic lookup workloads used by the tests.

Everything random comes from ``synth``; every piece of CKKS or lookup
arithmetic (digits, packing, encoding, keys, encryption) is the oracle's.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

import synth
from oracle import oracle as O


@dataclass
class Workload:
    prm: O.Params
    tables: List[O.TableSpec]
    M: np.ndarray
    plan: O.Plan
    keys: O.Keys
    queries: List[List[int]]          # per query: one index per table
    cts: List[np.ndarray]             # per query: uint64 [2][level+1][N]
    expected: List[np.ndarray]        # per query: cleartext lookup (concatenated rows)
    level: int
    draws: object = None


def compressed_table(g, rows: int, d: int, base: int, lo: float, hi: float) -> O.TableSpec:
    l = O.num_digits(rows, base)
    C = [synth.uniform_table(g, base, d, lo, hi) for _ in range(l)]
    return O.TableSpec(rows=rows, d=d, base=base, C=C)


def uncompressed_table(g, rows: int, d: int, lo: float, hi: float) -> O.TableSpec:
    return O.TableSpec(rows=rows, d=d, E=synth.uniform_table(g, rows, d, lo, hi))


def build(prm: O.Params, tables: List[O.TableSpec], level: int, n1: int, radix: int,
          n_queries: int, seed: int = 0, key_seed: int = 0, sign: int = 1) -> Workload:
    M = O.pack_tables(tables)
    plan = O.make_plan(prm, M, level, n1, radix, sign)
    gals = [O.galois_for_step(k, prm) for k in plan.rotation_steps()]
    draws = synth.key_draws(key_seed, prm.N, prm.q, prm.p, prm.dnum, gals)
    keys = O.keygen(prm, draws)
    g = synth.rng(seed + 1000)
    queries, cts, expected = [], [], []
    for _ in range(n_queries):
        idx = synth.indices(g, [t.rows for t in tables])
        sel = O.pack_selector(tables, idx)
        m = O.encode(sel, prm.delta, prm)
        ct = O.encrypt(prm, keys, m, level, synth.enc_draws(g, prm.N))
        queries.append(idx)
        cts.append(ct)
        expected.append(np.concatenate([t.lookup(i) for t, i in zip(tables, idx)]))
    return Workload(prm=prm, tables=tables, M=M, plan=plan, keys=keys, queries=queries,
                    cts=cts, expected=expected, level=level, draws=draws)


def config1(n_queries: int = 2, compressed: bool = True, n1: int = 4, radix: int = 2, sign: int = 1) -> Workload:
    """Toy ring N=2^12: one 256-row x 16 table, values U[-1,1]; base-16
    digits (2 digits, 32 selector slots) or an uncompressed 256-slot control."""
    prm = O.config1_params()
    g = synth.rng(0)
    if compressed:
        t = compressed_table(g, 256, 16, 16, -1.0, 1.0)
    else:
        t = uncompressed_table(g, 256, 16, -1.0, 1.0)
    return build(prm, [t], level=prm.L, n1=n1, radix=radix, n_queries=n_queries, sign=sign)


def decrypt_slots(w: Workload, ct: np.ndarray, scale: float, count: int) -> np.ndarray:
    m = O.decrypt(w.prm, w.keys, ct)
    return O.decode(m, scale, w.prm)[:count].real


def small_dlrm(seed: int = 0, **kw) -> O.SmallDLRM:
    """The small DLRM of the batched end-to-end configuration: 8 uncompressed
    tables of 2-200 rows x 16, 13 dense features, bottom 13-64-16, top
    144-32-1 (weights from ``synth``)."""
    d = synth.small_dlrm_draws(seed, **kw)
    tables = [O.TableSpec(rows=r, d=t.shape[1], E=t) for r, t in zip(d.table_rows, d.tables)]
    return O.SmallDLRM(tables=tables, bottom=list(d.bottom), top=list(d.top), n_dense=d.n_dense)


def dlrm_params_toy() -> O.Params:
    """N=2^12 with a chain deep enough for the forward pass: L=8, digits of
    three primes (dnum=3), three special primes."""
    return O.make_params(N=4096, L=8, K=3, alpha=3)


def table1_shape(prm: O.Params, level: int, n_queries: int = 1, d: int = 768, p: int = 16, l: int = 32,
                 n1: int = 32, radix: int = 2, seed: int = 0) -> Workload:
    """The lookup shape of the paper's comparison with prior work (Table I):
    one table of p^l rows stored as l digit tables of p x d (512 selector
    slots for p=16, l=32), values U[-0.05, 0.05]."""
    g = synth.rng(seed)
    t = O.TableSpec(rows=p ** l, d=d, base=p, C=[synth.uniform_table(g, p, d, -0.05, 0.05) for _ in range(l)])
    return build(prm, [t], level=level, n1=n1, radix=radix, n_queries=n_queries, seed=seed, sign=-1)


@dataclass
class MultiWorkload:
    prm: O.Params
    tables: List[O.TableSpec]
    M: np.ndarray
    plans: List[O.Plan]
    keys: O.Keys
    cts: List[List[np.ndarray]]       # per query: one ciphertext per column block
    expected: List[np.ndarray]
    level: int


def build_multi(prm: O.Params, tables: List[O.TableSpec], level: int, n1: int, radix: int, n_queries: int,
                seed: int = 0, sign: int = -1) -> MultiWorkload:
    """Packed selectors wider than one ciphertext: one ciphertext per block
    of n slots (Sec. III-C)."""
    M = O.pack_tables(tables)
    plans = O.make_multi_plan(prm, M, level, n1, radix, sign)
    steps = sorted({k for p in plans for k in p.rotation_steps()})
    gals = [O.galois_for_step(k, prm) for k in steps]
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals))
    g = synth.rng(seed + 2000)
    cts, expected = [], []
    for _ in range(n_queries):
        idx = synth.indices(g, [t.rows for t in tables])
        sel = O.pack_selector(tables, idx)
        cts.append([O.encrypt(prm, keys, O.encode(part, prm.delta, prm), level, synth.enc_draws(g, prm.N))
                    for part in O.split_selector(sel, prm.n)])
        expected.append(np.concatenate([t.lookup(i) for t, i in zip(tables, idx)]))
    return MultiWorkload(prm=prm, tables=tables, M=M, plans=plans, keys=keys, cts=cts, expected=expected,
                         level=level)
