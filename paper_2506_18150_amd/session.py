"""One encrypted-lookup deployment on one GPU: context, resident keys, plan,
client-side query encryption and result decryption.

Randomness is supplied by the caller (key draws and per-query encryption
draws); everything else is this package's own arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import encoding, planner
from .binding import Context, Plan
from .client import Client
from .params import ParamSet


def plan_device_bytes(prm: ParamSet, level: int, spec, mfma_min_slots: int = 33) -> int:
    """Device bytes a plan made from spec holds (helrm_plan_create): every
    stored diagonal's residues over PQ_level at 13 bytes a word (the 8-byte
    word plus the 5-byte plane the 40-bit primes keep), and, for a plan with
    several giant steps whose baby-step count reaches the matrix-core MAC's
    floor (knob mfma_min_slots), its matrix-core operands: 4 KiB per limb,
    coefficient and giant tile of 8.  Folded keys are not included
    (helrm_plan_fold_keys reports those)."""
    pqn = level + 1 + prm.K
    total = len(spec.diag) * pqn * prm.N * (8 + 5)
    babies = len({k % spec.n1 for k in spec.diag})
    if spec.n2 >= 2 and babies >= mfma_min_slots:
        total += -(-spec.n2 // 8) * pqn * prm.N * 4096
    return total


def fold_plans(prm: ParamSet, level: int, plans: Sequence[Plan], specs) -> Tuple[int, int]:
    """Fold the keys into every plan with several giant steps (the batched
    matrix-core product; at most 3 key-switching digits).  Stops at the first
    plan that no longer fits in device memory: the rest stay unfolded and
    take the other kernels.  Returns (bytes, plans folded)."""
    from .binding import HELRM_ENOMEM, HelrmError
    if prm.n_digits(level) > 3:
        return 0, 0
    total = count = 0
    for p, sp in zip(plans, specs):
        if sp.n2 < 2:
            continue
        try:
            total += p.helrm_plan_fold_keys()
            count += 1
        except HelrmError as e:
            if e.code != HELRM_ENOMEM:
                raise
            break
    return total, count


class LookupSession:
    def __init__(self, prm: ParamSet, tables: Sequence[planner.Table], level: int, n1: int, radix: int,
                 key_draws_fn, ctx: Optional[Context] = None, sign: int = -1, fold: bool = False):
        """key_draws_fn(galois_list) -> key draws (secret, public-key and
        switching-key randomness) for those Galois elements.  fold: fold the
        keys into the plans of several giant steps (batched lookups on the
        matrix cores; helrm_plan_fold_keys)."""
        self.prm = prm
        self.tables = list(tables)
        self.level = level
        self.ctx = ctx or Context(prm.log_n, prm.q, prm.p, prm.alpha)
        self.M = planner.packed_matrix(self.tables)
        # a selector wider than one ciphertext travels as n_in ciphertexts,
        # one plan per column block (Sec. III-C)
        self.specs = planner.make_multi_plan(self.M, prm.N, level, float(prm.q[level]), n1, radix, sign)
        self.n_in = len(self.specs)
        self.plans: List[Plan] = [self.ctx.helrm_plan_create(level, sp.m, sp.n1, sp.n2, sp.radix, sp.diag,
                                                             sp.coeffs, sp.sign, sp.span) for sp in self.specs]
        self.spec, self.plan = self.specs[0], self.plans[0]
        steps = sorted({k for p in self.plans for k in p.rotation_steps()})
        assert steps == sorted({k for sp in self.specs for k in sp.rotation_steps()})
        self.galois = [planner.galois(s, prm.N) for s in steps]
        self.client = Client(self.ctx, prm)
        self.client.keygen(key_draws_fn(self.galois), self.galois)
        self.folded_bytes, self.folded_plans = fold_plans(prm, level, self.plans, self.specs) if fold else (0, 0)

    @property
    def out_slots(self) -> int:
        return self.M.shape[0]

    def encrypt(self, idx_batch: Sequence[Sequence[int]], enc_draws: Sequence) -> torch.Tensor:
        """Client: digits -> one-hots -> packed selector -> encode at Delta ->
        encrypt, for each query (one draw per selector ciphertext when the
        selector spans several).  Returns [B][2][level+1][N], or
        [B][n_in][2][level+1][N] for n_in > 1."""
        cts = []
        n = self.prm.N // 2
        for idx, ed in zip(idx_batch, enc_draws):
            sel = planner.packed_selector(self.tables, idx)
            eds = ed if isinstance(ed, (list, tuple)) else [ed]
            parts = []
            for c, e in zip(range(0, len(sel), n), eds):
                m = encoding.encode(sel[c:c + n], self.prm.delta, self.prm.N)
                parts.append(self.client.encrypt(m, self.level, e))
            assert len(parts) == self.n_in, "one encryption draw per selector ciphertext"
            cts.append(parts[0] if self.n_in == 1 else torch.stack(parts))
        return torch.stack(cts).contiguous()

    def new_output(self, batch: int) -> torch.Tensor:
        return torch.zeros(batch, 2, self.level, self.prm.N, dtype=torch.int64, device="cuda")

    def lookup(self, sel: torch.Tensor, out: torch.Tensor, stream=None):
        if self.n_in == 1:
            self.ctx.helrm_lookup_packed(self.plan, sel, sel.shape[0], out, stream)
        else:
            self.ctx.helrm_lookup_multi(self.plans, sel, sel.shape[0], out, stream)

    def decrypt_rows(self, out: torch.Tensor) -> np.ndarray:
        m = self.client.decrypt(out)
        lead = m.shape[:-1]
        flat = m.reshape(-1, self.prm.N)
        rows = np.stack([encoding.decode(v, self.prm.delta, self.prm.N)[: self.out_slots].real for v in flat])
        return rows.reshape(*lead, self.out_slots)

    def cleartext(self, idx: Sequence[int]) -> np.ndarray:
        return np.concatenate([t.row(i) for t, i in zip(self.tables, idx)])


class GroupedDeployment:
    """Tables split into fixed groups of consecutive tables, one packed plan
    per group, all sharing one context and one resident key set (the union of
    the groups' rotation keys).  A request touching some tables sends one
    selector ciphertext per touched group; untouched tables of a touched group
    get an all-zero one-hot block (their rows come out as zeros)."""

    def __init__(self, prm: ParamSet, tables: Sequence[planner.Table], group_size: int, level: int, n1: int,
                 radix: int, key_draws_fn, sign: int = -1, fold: bool = False):
        """fold: fold the keys into the plans of several giant steps, for
        batches of 8 and more on the matrix cores (helrm_plan_fold_keys);
        plans that no longer fit in device memory stay unfolded."""
        self.prm, self.level = prm, level
        self.tables = list(tables)
        self.groups = [list(range(i, min(i + group_size, len(tables)))) for i in range(0, len(tables), group_size)]
        self.ctx = Context(prm.log_n, prm.q, prm.p, prm.alpha)
        self.specs, self.plans = [], []
        steps = set()
        for grp in self.groups:
            M = planner.packed_matrix([self.tables[t] for t in grp])
            m = planner.next_pow2(M.shape[0])
            spec = planner.make_plan(M, prm.N, level, float(prm.q[level]), min(n1, m), radix, sign)
            self.specs.append(spec)
            self.plans.append(self.ctx.helrm_plan_create(level, spec.m, spec.n1, spec.n2, spec.radix, spec.diag,
                                                         spec.coeffs, spec.sign, spec.span))
            steps.update(spec.rotation_steps())
        self.galois = sorted({planner.galois(s, prm.N) for s in steps})
        self.client = Client(self.ctx, prm)
        self.client.keygen(key_draws_fn(self.galois), self.galois)
        kl = prm.L + 1 + prm.K
        # per key: Montgomery-form words plus the 40-bit planes of the b halves
        self.key_bytes = len(self.galois) * prm.dnum * kl * prm.N * (16 + 5)
        self.plan_bytes = sum(plan_device_bytes(prm, level, sp) for sp in self.specs)
        self.folded_bytes, self.folded_plans = fold_plans(prm, level, self.plans, self.specs) if fold else (0, 0)

    def group_of(self, table: int) -> int:
        for g, grp in enumerate(self.groups):
            if table in grp:
                return g
        raise ValueError(table)

    def selector(self, g: int, touched: dict) -> np.ndarray:
        """Packed one-hots of group g; touched maps table -> index."""
        parts = []
        for t in self.groups[g]:
            tb = self.tables[t]
            parts.append(tb.one_hot(touched[t]) if t in touched else np.zeros(tb.width))
        return np.concatenate(parts)

    def encrypt_group(self, g: int, touched: dict, ed) -> torch.Tensor:
        m = encoding.encode(self.selector(g, touched), self.prm.delta, self.prm.N)
        return self.client.encrypt(m, self.level, ed)

    def decrypt_group(self, g: int, out: torch.Tensor) -> np.ndarray:
        m = self.client.decrypt(out.reshape(2, self.level, self.prm.N))
        rows = 16 * len(self.groups[g])
        return encoding.decode(m, self.prm.delta, self.prm.N)[:rows].real

    def cleartext_group(self, g: int, touched: dict) -> np.ndarray:
        out = []
        for t in self.groups[g]:
            tb = self.tables[t]
            out.append(tb.row(touched[t]) if t in touched else np.zeros(tb.d))
        return np.concatenate(out)
