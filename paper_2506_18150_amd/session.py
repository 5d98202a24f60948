"""One encrypted-lookup deployment on one GPU: context, resident keys, plan,
client-side query encryption and result decryption.

Randomness is supplied by the caller (key draws and per-query encryption
draws); everything else is this package's own arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import encoding, planner
from .binding import Context, Plan
from .client import Client
from .params import ParamSet


class LookupSession:
    def __init__(self, prm: ParamSet, tables: Sequence[planner.Table], level: int, n1: int, radix: int,
                 key_draws_fn, ctx: Optional[Context] = None, sign: int = -1):
        """key_draws_fn(galois_list) -> key draws (secret, public-key and
        switching-key randomness) for those Galois elements."""
        self.prm = prm
        self.tables = list(tables)
        self.level = level
        self.ctx = ctx or Context(prm.log_n, prm.q, prm.p, prm.alpha)
        self.M = planner.packed_matrix(self.tables)
        self.spec = planner.make_plan(self.M, prm.N, level, float(prm.q[level]), n1, radix, sign)
        self.plan: Plan = self.ctx.helrm_plan_create(level, self.spec.m, self.spec.n1, self.spec.n2,
                                                     self.spec.radix, self.spec.diag, self.spec.coeffs,
                                                     self.spec.sign, self.spec.span)
        steps = self.plan.rotation_steps()
        assert steps == self.spec.rotation_steps()
        self.galois = [planner.galois(s, prm.N) for s in steps]
        self.client = Client(self.ctx, prm)
        self.client.keygen(key_draws_fn(self.galois), self.galois)

    @property
    def out_slots(self) -> int:
        return self.M.shape[0]

    def encrypt(self, idx_batch: Sequence[Sequence[int]], enc_draws: Sequence) -> torch.Tensor:
        """Client: digits -> one-hots -> packed selector -> encode at Delta ->
        encrypt, for each query.  Returns [B][2][level+1][N]."""
        cts = []
        for idx, ed in zip(idx_batch, enc_draws):
            sel = planner.packed_selector(self.tables, idx)
            m = encoding.encode(sel, self.prm.delta, self.prm.N)
            cts.append(self.client.encrypt(m, self.level, ed))
        return torch.stack(cts).contiguous()

    def new_output(self, batch: int) -> torch.Tensor:
        return torch.zeros(batch, 2, self.level, self.prm.N, dtype=torch.int64, device="cuda")

    def lookup(self, sel: torch.Tensor, out: torch.Tensor, stream=None):
        self.ctx.helrm_lookup_packed(self.plan, sel, sel.shape[0], out, stream)

    def decrypt_rows(self, out: torch.Tensor) -> np.ndarray:
        m = self.client.decrypt(out)
        lead = m.shape[:-1]
        flat = m.reshape(-1, self.prm.N)
        rows = np.stack([encoding.decode(v, self.prm.delta, self.prm.N)[: self.out_slots].real for v in flat])
        return rows.reshape(*lead, self.out_slots)

    def cleartext(self, idx: Sequence[int]) -> np.ndarray:
        return np.concatenate([t.row(i) for t, i in zip(self.tables, idx)])
