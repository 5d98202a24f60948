"""Encrypted small DLRM on the GPU: dense features and embedding lookups into
bottom and top MLPs with the square activation (Sec. II-B; the small model of
Sec. V-C), every step a libhelrm call.

Layout of the slot vectors (one ciphertext per request):
  * input: dense features in slots [0, n_dense), then the one-hots of every
    table (Sec. IV-B packing);
  * the embedding product writes rows [0, E) (E = tables x d) and the last
    bottom layer rows [E, E+H); both matrices have E+H rows, so both results
    are zero on every slot of [0, next_pow2(E+H)) they do not write and their
    sum is the concatenation [embeddings; bottom output];
  * every other layer reads slots [0, cols) and writes [0, rows); what the
    diagonal method leaves above next_pow2(rows) is ignored by the next layer,
    whose matrix is zero there.

Levels and scales: a matvec at level l consumes one level; its plaintext
diagonals are encoded at S_out q_l / S_in so its output is at S_out (Delta,
except the embedding product, which is put at the scale of the bottom output);
a square (ciphertext product, relinearisation, rescale) maps S to S^2 / q_l.
With two bottom and two top layers the pass takes 7 levels; the embedding
product runs on the input ciphertext and is brought to the concatenation
level by dropping primes.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import encoding, planner
from .binding import HELRM_OP_ADD, Context, Plan
from .client import Client
from .params import ParamSet


@dataclass
class DLRMWeights:
    tables: List[np.ndarray]                          # uncompressed tables, rows x d
    bottom: List[Tuple[np.ndarray, np.ndarray]]       # (W, b) per layer
    top: List[Tuple[np.ndarray, np.ndarray]]
    n_dense: int

    @property
    def emb_dim(self) -> int:
        return sum(t.shape[1] for t in self.tables)

    def input_slots(self, dense: np.ndarray, idx: Sequence[int]) -> np.ndarray:
        oh = []
        for t, i in zip(self.tables, idx):
            e = np.zeros(t.shape[0])
            e[i] = 1.0
            oh.append(e)
        return np.concatenate([np.asarray(dense, dtype=float)] + oh)

    def cleartext(self, dense: np.ndarray, idx: Sequence[int]) -> np.ndarray:
        h = np.asarray(dense, dtype=float)
        for W, b in self.bottom:
            h = (W @ h + b) ** 2
        z = np.concatenate([t[i] for t, i in zip(self.tables, idx)] + [h])
        for k, (W, b) in enumerate(self.top):
            z = W @ z + b
            if k + 1 < len(self.top):
                z = z ** 2
        return z


def layer_matrices(w: DLRMWeights):
    """(emb, bottom matrices, bottom bias vectors, top matrices, top bias
    vectors) over slot vectors, in the layout described above."""
    E = w.emb_dim
    H = w.bottom[-1][0].shape[0]
    width = w.n_dense + sum(t.shape[0] for t in w.tables)
    emb = np.zeros((E + H, width))
    r, c = 0, w.n_dense
    for t in w.tables:
        emb[r:r + t.shape[1], c:c + t.shape[0]] = t.T
        r += t.shape[1]
        c += t.shape[0]
    bottom, bb = [], []
    for k, (W, b) in enumerate(w.bottom):
        if k + 1 < len(w.bottom):
            bottom.append(np.asarray(W, dtype=float))
            bb.append(np.asarray(b, dtype=float))
        else:
            M = np.zeros((E + H, W.shape[1]))
            M[E:] = W
            bv = np.zeros(E + H)
            bv[E:] = b
            bottom.append(M)
            bb.append(bv)
    top = [np.asarray(W, dtype=float) for W, _ in w.top]
    bt = [np.asarray(b, dtype=float) for _, b in w.top]
    return emb, bottom, bb, top, bt


@dataclass
class Schedule:
    """Device plans and bias plaintexts of one forward pass."""
    level0: int
    emb: Plan
    bottom: List[Plan]
    bias_bottom: List[torch.Tensor]     # [level+1][N] residues at the layer's output level
    top: List[Plan]
    bias_top: List[torch.Tensor]
    concat_level: int
    out_level: int

    def plans(self) -> List[Plan]:
        return [self.emb] + self.bottom + self.top


def forward(ctx: Context, sch: Schedule, sel: torch.Tensor, batch: int, stream=None) -> torch.Tensor:
    """Encrypted forward pass of `batch` input ciphertexts [B][2][level0+1][N];
    returns the logit ciphertexts [B][2][out_level+1][N] (slot 0, scale Delta)."""
    N = ctx.N

    def new(level):
        return torch.empty(batch, 2, level + 1, N, dtype=torch.int64, device=sel.device)

    def matvec(plan, x):
        y = new(plan.level - 1)
        ctx.helrm_lookup_packed(plan, x, batch, y, stream)
        return y

    def square(x, level):
        sq = new(level)
        ctx.helrm_mul_relin(x, x, level, sq, batch, stream)
        y = new(level - 1)
        ctx.helrm_rescale(sq, level, y, batch, stream)
        return y

    x = sel
    for plan, b in zip(sch.bottom, sch.bias_bottom):
        lv = plan.level - 1
        y = matvec(plan, x)
        ctx.helrm_add_plain(y, b, lv, y, batch, stream)
        x = square(y, lv)
    e = matvec(sch.emb, sel)
    ed = new(sch.concat_level)
    ctx.helrm_mod_drop(e, sch.emb.level - 1, ed, sch.concat_level, batch, stream)
    z = new(sch.concat_level)
    cq = list(range(sch.concat_level + 1))
    ctx.helrm_poly_op(HELRM_OP_ADD, ed, x, z, cq + cq, batch, stream)
    for k, (plan, b) in enumerate(zip(sch.top, sch.bias_top)):
        lv = plan.level - 1
        z = matvec(plan, z)
        ctx.helrm_add_plain(z, b, lv, z, batch, stream)
        if k + 1 < len(sch.top):
            z = square(z, lv)
    return z


class DLRMSession:
    """One deployment: context, resident rotation and relinearisation keys,
    the layer plans and bias plaintexts, and the client side (encrypt the
    packed input, decrypt the logit)."""

    def __init__(self, prm: ParamSet, w: DLRMWeights, level0: int, key_draws_fn, n1: int = 16, radix: int = 8,
                 sign: int = -1, ctx: Optional[Context] = None):
        """key_draws_fn(galois_list) -> key draws including the
        relinearisation randomness."""
        self.prm, self.w, self.level0 = prm, w, level0
        self.ctx = ctx or Context(prm.log_n, prm.q, prm.p, prm.alpha)
        self.client = Client(self.ctx, prm)
        emb, bottom, bb, top, bt = layer_matrices(w)
        delta = float(prm.delta)

        def plan(M, level, s_in, s_out):
            m = planner.next_pow2(M.shape[0])
            spec = planner.make_plan(M, prm.N, level, s_out * prm.q[level] / s_in, min(n1, m), radix, sign)
            return self.ctx.helrm_plan_create(level, spec.m, spec.n1, spec.n2, spec.radix, spec.diag, spec.coeffs,
                                              spec.sign, spec.span)

        lv, S = level0, delta
        bottom_p, bb_t = [], []
        for M, bv in zip(bottom, bb):
            bottom_p.append(plan(M, lv, S, delta))
            lv -= 1
            S = delta
            bb_t.append(self._plain(bv, S, lv))
            S = S * S / prm.q[lv]
            lv -= 1
        concat_level, concat_scale = lv, S
        emb_p = plan(emb, level0, delta, concat_scale)
        top_p, bt_t = [], []
        for k, (M, bv) in enumerate(zip(top, bt)):
            top_p.append(plan(M, lv, S, delta))
            lv -= 1
            S = delta
            bt_t.append(self._plain(bv, S, lv))
            if k + 1 < len(top):
                S = S * S / prm.q[lv]
                lv -= 1
        self.schedule = Schedule(level0=level0, emb=emb_p, bottom=bottom_p, bias_bottom=bb_t, top=top_p,
                                 bias_top=bt_t, concat_level=concat_level, out_level=lv)
        steps = sorted({s for p in self.schedule.plans() for s in p.rotation_steps()})
        self.galois = [planner.galois(s, prm.N) for s in steps]
        self.client.keygen(key_draws_fn(self.galois), self.galois)

    def _plain(self, z: np.ndarray, scale: float, level: int) -> torch.Tensor:
        coeffs = encoding.encode(z, scale, self.prm.N)
        out = torch.zeros(level + 1, self.prm.N, dtype=torch.int64, device="cuda")
        src = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.int64)).cuda()
        primes = list(range(level + 1))
        self.ctx.helrm_from_signed(src, out, primes, 1)
        self.ctx.helrm_ntt(out, primes, 1)
        return out

    def encrypt(self, dense_batch: Sequence[np.ndarray], idx_batch: Sequence[Sequence[int]],
                enc_draws: Sequence) -> torch.Tensor:
        cts = []
        for dense, idx, ed in zip(dense_batch, idx_batch, enc_draws):
            m = encoding.encode(self.w.input_slots(dense, idx), self.prm.delta, self.prm.N)
            cts.append(self.client.encrypt(m, self.level0, ed))
        return torch.stack(cts).contiguous()

    def forward(self, sel: torch.Tensor, stream=None) -> torch.Tensor:
        return forward(self.ctx, self.schedule, sel, sel.shape[0], stream)

    def decrypt_logits(self, out: torch.Tensor) -> np.ndarray:
        m = self.client.decrypt(out)
        flat = m.reshape(-1, self.prm.N)
        return np.array([encoding.decode(v, self.prm.delta, self.prm.N)[0].real for v in flat])
