"""The batching workload at its full size (26 tables of log-uniform row
counts packed into one 416 x 13,962 selector matrix, m = 512 diagonals,
N = 2^16, selector at level 23, n1 = 64, fold radix 8, rotation sign -1, a
batch of 8 queries: the configuration the batching benchmark times).  The
oracle cannot replay 512 diagonals at level 23 in test time, so the checks
are properties that hold at any size (Sec. III-B, Sec. IV-A/IV-B):
  * every decrypted row of every query is within 1e-4 of the cleartext row
    of its table (sum of the digit tables' rows, or the uncompressed row);
  * every batch element is bit-identical to the same query looked up alone
    (batch 8 runs the workgroup-shared baby-step kernel, batch 1 the
    per-thread one with regenerated key halves)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _tables():
    """The same draws twice: oracle table specs (expected rows) and the
    product's table descriptions (plan)."""
    from paper_2506_18150_amd import planner
    _, counts = synth.criteo_like_row_counts()
    specs, tables = [], []
    g = synth.rng(0)
    for k in counts:
        if k <= 256:
            E = synth.uniform_table(g, k, 16, -0.05, 0.05)
            specs.append(O.TableSpec(rows=k, d=16, E=E))
            tables.append(planner.Table(rows=k, d=16, full=E))
        else:
            C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(O.num_digits(k, 256))]
            specs.append(O.TableSpec(rows=k, d=16, base=256, C=C))
            tables.append(planner.Table(rows=k, d=16, base=256, parts=C))
    return specs, tables


def test_batching_workload_full_size():
    import torch
    from paper_2506_18150_amd import params
    from paper_2506_18150_amd.session import LookupSession

    prm = params.n16()
    specs, tables = _tables()
    assert len(tables) == 26
    say("full-size batching workload: 26 tables, level 23, n1=64, radix 8, batch 8")
    sess = LookupSession(prm, tables, 23, 64, 8, lambda gals: synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum,
                                                                               gals), sign=-1)
    assert sess.n_in == 1 and sess.spec.m == 512 and sess.out_slots == 416
    B = 8
    g = synth.rng(5)
    idx = [synth.indices(g, [t.rows for t in tables]) for _ in range(B)]
    sel = sess.encrypt(idx, [synth.enc_draws(g, prm.N) for _ in range(B)])
    out = sess.new_output(B)
    sess.ctx.helrm_set_tuning("baby_share", 4)
    sess.lookup(sel, out)
    torch.cuda.synchronize()
    rows = sess.decrypt_rows(out)
    for b in range(B):
        want = np.concatenate([t.lookup(i) for t, i in zip(specs, idx[b])])
        assert np.max(np.abs(rows[b] - want)) < 1e-4, f"query {b}"
    say("batch elements against single lookups")
    one = sess.new_output(1)
    for b in (0, 3, 7):
        sess.lookup(sel[b:b + 1].contiguous(), one)
        torch.cuda.synchronize()
        assert torch.equal(one[0], out[b]), f"query {b}: batch of 8 differs from batch of 1"
