"""GPU parity of the matrix-core plaintext MAC (the batched baby-step stage on
the int8 matrix cores): lookups whose batch takes it are bit-exact against the
oracle on every residue, and equal to the same batch with the VALU kernels
(knob baby_mfma = 0).  Covered: ragged ciphertext tiles (batches 9 and 17),
both digit counts (primes below 2^40: five balanced base-256 digits; 60-bit
primes: eight), one to four key-switching digits, several giant tiles (Table I
shape: 32 giant outputs), the accumulating launches of multi-ciphertext
selectors, and the batching workload's table group at level 23.  Double-hoisted
BSGS product: Sec. III-B; packing: Sec. IV-B."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _mfma_ctx(prm):
    """A context whose matrix-core MAC also takes plans with few baby steps
    (by default those stay on the VALU kernels)."""
    ctx = context_for(prm)
    ctx.helrm_set_tuning("mfma_min_slots", 1)
    return ctx


def _lookup(ctx, plan, cts, level, N, mfma):
    ctx.helrm_set_tuning("baby_mfma", 8 if mfma else 0)
    try:
        B = len(cts)
        out = empty(B, 2, level, N)
        ctx.helrm_lookup_packed(plan, to_dev(np.stack(cts)), B, out)
        return to_host(out).reshape(B, 2, level, N)
    finally:
        ctx.helrm_set_tuning("baby_mfma", 8)


def _both_and_oracle(ctx, w, plan, check, what):
    """The batch with the matrix-core MAC and with the VALU kernels: equal;
    elements `check` also against the oracle and the cleartext rows."""
    say(f"{what}: matrix-core MAC, batch {len(w.cts)}")
    got = _lookup(ctx, plan, w.cts, w.level, w.prm.N, True)
    say(f"{what}: VALU MAC")
    ref = _lookup(ctx, plan, w.cts, w.level, w.prm.N, False)
    assert_bit_exact(got, ref, f"{what}: matrix cores vs VALU")
    pts = O.plan_residues(w.prm, w.plan)
    for k in check:
        assert_bit_exact(got[k], O.lookup(w.prm, w.keys, w.plan, w.cts[k], pts), f"{what}: query {k}")
        rows = W.decrypt_slots(w, got[k], w.prm.delta, len(w.expected[k]))
        assert np.max(np.abs(rows - w.expected[k])) < 1e-4


@pytest.mark.parametrize("level", [3, 1])
def test_mfma_toy_ring_ragged(level):
    """Toy ring N=2^12 (three 40-bit primes, a 60-bit q_0 and special prime;
    one prime per digit: four digits at level 3, two at level 1): the 256-row
    table with n1 = 4 (four giant outputs), batch 9 (a tile of 8 and one)."""
    prm = O.config1_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 256, 16, 16, -1.0, 1.0)
    w = W.build(prm, [t], level=level, n1=4, radix=2, n_queries=9)
    ctx = _mfma_ctx(prm)
    load_keys(ctx, w.keys)
    _both_and_oracle(ctx, w, gpu_plan(ctx, w.plan), [0, 7, 8], f"toy level {level}")
    ctx.close()


def test_mfma_table1_shape_giant_tiles():
    """d = 768 from 32 base-16 digit tables on the toy ring at level 1: m =
    1024 diagonals, n1 = 32, 32 giant outputs in four tiles of 8, batch 8."""
    prm = O.config1_params()
    w = W.table1_shape(prm, 1, n_queries=8)
    assert w.plan.n2 == 32
    ctx = _mfma_ctx(prm)
    load_keys(ctx, w.keys)
    _both_and_oracle(ctx, w, gpu_plan(ctx, w.plan), [0, 5], "Table I shape")
    ctx.close()


def test_mfma_multi_ciphertext_accumulates():
    """Two selector ciphertexts per query on the toy ring (the second block's
    products are added to the first's giant accumulators), batch 8."""
    prm = O.config1_params()
    ctx = _mfma_ctx(prm)
    g = synth.rng(9)
    tables = [W.uncompressed_table(g, 1000, 16, -1, 1) for _ in range(3)]
    w = W.build_multi(prm, tables, level=2, n1=16, radix=4, n_queries=8)
    load_keys(ctx, w.keys)
    plans = [gpu_plan(ctx, p) for p in w.plans]
    sel = to_dev(np.stack([np.stack(c) for c in w.cts]))
    outs = []
    for mfma in (True, False):
        ctx.helrm_set_tuning("baby_mfma", 8 if mfma else 0)
        say(f"multi-ciphertext batch 8 mfma={mfma}")
        out = empty(8, 2, 2, prm.N)
        ctx.helrm_lookup_multi(plans, sel, 8, out)
        outs.append(to_host(out).reshape(8, 2, 2, prm.N))
    ctx.helrm_set_tuning("baby_mfma", 8)
    assert_bit_exact(outs[0], outs[1], "multi: matrix cores vs VALU")
    for k in (0, 7):
        assert_bit_exact(outs[0][k], O.lookup_multi(prm, w.keys, w.plans, w.cts[k]), f"multi query {k}")
    ctx.close()


def test_mfma_n16_multitable_batch17():
    """N=2^16, four tables (64 outputs, m = 64, n1 = 16: four giant outputs),
    selector at level 1 (one digit), batch 17 (tiles 8, 8, 1)."""
    prm = O.config2_params()
    g = synth.rng(0)
    tables = [W.compressed_table(g, 65536, 16, 256, -0.05, 0.05),
              W.uncompressed_table(g, 100, 16, -0.05, 0.05),
              W.compressed_table(g, 300000, 16, 256, -0.05, 0.05),
              W.compressed_table(g, 1000, 16, 256, -0.05, 0.05)]
    w = W.build(prm, tables, level=1, n1=16, radix=8, n_queries=17, sign=-1)
    ctx = _mfma_ctx(prm)
    load_keys(ctx, w.keys)
    _both_and_oracle(ctx, w, gpu_plan(ctx, w.plan), [0, 16], "N=2^16 level 1 batch 17")
    ctx.close()


@pytest.mark.timeout(900)
def test_mfma_n16_level23_group():
    """The request loop's first table group of the batching workload at level
    23 (three key-switching digits, 24 + 8 primes), n1 = 16, radix 8, sign -1,
    batch 8."""
    prm = O.config2_params()
    _, counts = synth.criteo_like_row_counts()
    g = synth.rng(0)
    specs = []
    for k in counts[:4]:
        if k <= 256:
            specs.append(O.TableSpec(rows=k, d=16, E=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(O.num_digits(k, 256))]
            specs.append(O.TableSpec(rows=k, d=16, base=256, C=C))
    w = W.build(prm, specs, level=23, n1=16, radix=8, n_queries=8, sign=-1)
    assert w.plan.n2 == 4 and prm.n_digits(23) == 3
    ctx = _mfma_ctx(prm)
    load_keys(ctx, w.keys)
    _both_and_oracle(ctx, w, gpu_plan(ctx, w.plan), [0, 7], "level 23 group")
    ctx.close()
