"""Helpers for the GPU parity tests: move oracle-built inputs (keys, plans,
ciphertexts) into the HIP library and bring results back.  No expected value is
ever produced here; the oracle computes those."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O


def say(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def context_for(prm: O.Params):
    from paper_2506_18150_amd import binding as B
    return B.Context(prm.logN, prm.q, prm.p, prm.alpha)


def load_keys(ctx, keys: O.Keys):
    import torch
    from paper_2506_18150_amd import binding as B
    for g, k in sorted(keys.swk.items()):
        ctx.helrm_load_eval_keys([g], B.device_u64(k), [keys.seeds[g]])
    torch.cuda.synchronize()


def gpu_plan(ctx, plan: O.Plan):
    diag = sorted(g * plan.n1 + b for (g, b) in plan.coeffs)
    coeffs = np.stack([plan.coeffs[divmod(k, plan.n1)] for k in diag])
    return ctx.helrm_plan_create(plan.level, plan.m, plan.n1, plan.n2, plan.radix, diag, coeffs,
                                 plan.sign, plan.span)


def to_dev(a: np.ndarray):
    from paper_2506_18150_amd import binding as B
    return B.device_u64(np.ascontiguousarray(a, dtype=np.uint64))


def to_host(t) -> np.ndarray:
    import torch
    from paper_2506_18150_amd import binding as B
    torch.cuda.synchronize()
    return B.host_u64(t)


def empty(*shape):
    import torch
    return torch.zeros(*shape, dtype=torch.int64, device="cuda")


def assert_bit_exact(got: np.ndarray, want: np.ndarray, what: str):
    got = np.asarray(got, dtype=np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, f"{what}: shape {got.shape} != {want.shape}"
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{what}: {len(bad)} residues differ, first at {tuple(bad[0])}: " \
                          f"{int(got[tuple(bad[0])])} != {int(want[tuple(bad[0])])}"
