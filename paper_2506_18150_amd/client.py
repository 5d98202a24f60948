"""Client side of the protocol on the GPU: key generation, encryption and
decryption built from the library's element-wise, NTT and automorphism calls
(Appendix A "Encryption", "Key-switching").

Randomness (ternary secret, Gaussian errors, uniform polynomials) is an input:
it comes from the caller's seeded draws, so this module only does the
arithmetic:
  pk = (-a s + e, a) over Q_L;
  switching key s' -> s, digit j: b_j = -a_j s + e_j + [P]_{q_i} s' on the
  primes q_i of digit j, a_j over all Q and special primes, expanded on the
  GPU from the key's seed (helrm_key_uniform);
  rotation by k: s' = sigma_{5^k}(s); relinearisation: s' = s^2;
  encryption at level l: (v pk_b + e0 + m, v pk_a + e1) over q_0..q_l;
  decryption: c0 + c1 s on q_0, centred.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence

import numpy as np
import torch

from .binding import (HELRM_OP_ADD, HELRM_OP_MUL, HELRM_OP_SUB, Context, device_u64, host_u64)
from .params import ParamSet


class Client:
    def __init__(self, ctx: Context, prm: ParamSet, device: str = "cuda"):
        self.ctx, self.prm, self.dev = ctx, prm, device
        self.N = prm.N
        self.kl = prm.L + 1 + prm.K
        self.s_all: Optional[torch.Tensor] = None
        self.pk: Optional[torch.Tensor] = None

    def _zeros(self, *shape) -> torch.Tensor:
        return torch.zeros(*shape, dtype=torch.int64, device=self.dev)

    def _signed_ntt(self, v: np.ndarray, primes: Sequence[int]) -> torch.Tensor:
        src = torch.from_numpy(np.ascontiguousarray(v, dtype=np.int64)).to(self.dev)
        out = self._zeros(len(primes), self.N)
        self.ctx.helrm_from_signed(src, out, primes, 1)
        self.ctx.helrm_ntt(out, primes, 1)
        return out

    def keygen(self, draws, galois: Iterable[int]) -> None:
        """Secret and public key from the draws, then one switching key per
        Galois element (loaded into the context)."""
        allp = list(range(self.kl))
        self.s_all = self._signed_ntt(draws.s, allp)
        Qp = list(range(self.prm.L + 1))
        a = device_u64(draws.pk_a, self.dev)
        e = self._signed_ntt(draws.pk_e, Qp)
        t = self._zeros(len(Qp), self.N)
        self.ctx.helrm_poly_op(HELRM_OP_MUL, a, self.s_all[: len(Qp)].contiguous(), t, Qp, 1)
        b = self._zeros(len(Qp), self.N)
        self.ctx.helrm_poly_op(HELRM_OP_SUB, e, t, b, Qp, 1)
        self.pk = torch.stack([b, a]).contiguous()
        for g in sorted(set(int(x) for x in galois)):
            sg = self._zeros(self.kl, self.N)
            self.ctx.helrm_automorph(self.s_all, sg, g, self.kl, 1)
            key = self.switch_key(sg, draws.swk[g])
            self.ctx.helrm_load_eval_keys([g], key, [draws.swk[g].a_seed])
            del key
        if getattr(draws, "relin", None) is not None:
            # relinearisation key (s^2 -> s), loaded as Galois element 0
            s2 = self._zeros(self.kl, self.N)
            self.ctx.helrm_poly_op(HELRM_OP_MUL, self.s_all, self.s_all, s2, allp, 1)
            key = self.switch_key(s2, draws.relin)
            self.ctx.helrm_load_eval_keys([0], key, [draws.relin.a_seed])
            del key
        torch.cuda.synchronize()

    def switch_key(self, s_from: torch.Tensor, d) -> torch.Tensor:
        """Switching key from s_from (evaluation form over every prime) to
        the secret: [dnum][2][L+1+K][N] as helrm_load_eval_keys takes it."""
        allp = list(range(self.kl))
        key = self._zeros(self.prm.dnum, 2, self.kl, self.N)
        for j in range(self.prm.dnum):
            a = self._zeros(self.kl, self.N)
            self.ctx.helrm_key_uniform(d.a_seed, j, a)
            e = self._signed_ntt(d.e[j], allp)
            t = self._zeros(self.kl, self.N)
            self.ctx.helrm_poly_op(HELRM_OP_MUL, a, self.s_all, t, allp, 1)
            b = self._zeros(self.kl, self.N)
            self.ctx.helrm_poly_op(HELRM_OP_SUB, e, t, b, allp, 1)
            dp = self.prm.digit_primes(j)
            lo, hi = dp[0], dp[-1] + 1
            g = self._zeros(len(dp), self.N)
            self.ctx.helrm_mul_scalar(s_from[lo:hi].contiguous(), [self.prm.P_mod(self.prm.q[i]) for i in dp],
                                      g, dp, 1)
            seg = b[lo:hi].contiguous()
            self.ctx.helrm_poly_op(HELRM_OP_ADD, seg, g, seg, dp, 1)
            b[lo:hi] = seg
            key[j, 0] = b
            key[j, 1] = a
        return key

    def encrypt(self, m_coeffs: np.ndarray, level: int, ed) -> torch.Tensor:
        """Encrypt integer coefficients at the given level -> [2][level+1][N]."""
        Qp = list(range(level + 1))
        v = self._signed_ntt(ed.v, Qp)
        e0 = self._signed_ntt(ed.e0, Qp)
        e1 = self._signed_ntt(ed.e1, Qp)
        m = self._signed_ntt(m_coeffs, Qp)
        pkb = self.pk[0, : level + 1].contiguous()
        pka = self.pk[1, : level + 1].contiguous()
        c = self._zeros(2, level + 1, self.N)
        t = self._zeros(level + 1, self.N)
        self.ctx.helrm_poly_op(HELRM_OP_MUL, v, pkb, t, Qp, 1)
        self.ctx.helrm_poly_op(HELRM_OP_ADD, t, e0, t, Qp, 1)
        c0 = self._zeros(level + 1, self.N)
        self.ctx.helrm_poly_op(HELRM_OP_ADD, t, m, c0, Qp, 1)
        t2 = self._zeros(level + 1, self.N)
        self.ctx.helrm_poly_op(HELRM_OP_MUL, v, pka, t2, Qp, 1)
        c1 = self._zeros(level + 1, self.N)
        self.ctx.helrm_poly_op(HELRM_OP_ADD, t2, e1, c1, Qp, 1)
        c[0] = c0
        c[1] = c1
        return c

    def decrypt(self, ct: torch.Tensor) -> np.ndarray:
        """ct [..., 2, limbs, N] -> int64 coefficients [..., N] (q_0 limb, centred)."""
        lead = ct.shape[:-3]
        flat = ct.reshape(-1, *ct.shape[-3:])
        out = []
        s0 = self.s_all[:1].contiguous()
        q0 = self.prm.q[0]
        for k in range(flat.shape[0]):
            c0 = flat[k, 0, :1].contiguous()
            c1 = flat[k, 1, :1].contiguous()
            t = self._zeros(1, self.N)
            self.ctx.helrm_poly_op(HELRM_OP_MUL, c1, s0, t, [0], 1)
            self.ctx.helrm_poly_op(HELRM_OP_ADD, t, c0, t, [0], 1)
            self.ctx.helrm_intt(t, [0], 1)
            v = host_u64(t)[0].astype(np.int64)      # q_0 < 2^60 fits
            out.append(np.where(v > q0 // 2, v - q0, v))
        return np.stack(out).reshape(*lead, self.N)
