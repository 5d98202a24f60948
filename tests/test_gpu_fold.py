"""GPU parity of the key-folded matrix-core product (helrm_plan_fold_keys and
the batched lookups that use it): bit-exact against the oracle on every
residue and equal to the same batch on the VALU kernels, for one to three
key-switching digits, ragged 16-ciphertext tiles, several giant tiles, the
accumulating launches of multi-ciphertext selectors, and the batching
workload's table group at level 23.  Loading keys again makes the folded
words stale, and the lookup falls back (still bit-exact).  Double-hoisted BSGS
product: Sec. III-B; packing: Sec. IV-B; key switching: Appendix A."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev, to_host

pytestmark = pytest.mark.gpu

VALU = dict(baby_fold=0, baby_mfma=0)
FOLD = dict(baby_fold=8, baby_mfma=0)


def _run(ctx, plan, cts, level, N, knobs):
    for k, v in knobs.items():
        ctx.helrm_set_tuning(k, v)
    try:
        B = len(cts)
        out = empty(B, 2, level, N)
        ctx.helrm_lookup_packed(plan, to_dev(np.stack(cts)), B, out)
        return to_host(out).reshape(B, 2, level, N)
    finally:
        ctx.helrm_set_tuning("baby_fold", 8)
        ctx.helrm_set_tuning("baby_mfma", 8)


def _check(ctx, w, plan, check, what):
    say(f"{what}: folded product, batch {len(w.cts)}")
    got = _run(ctx, plan, w.cts, w.level, w.prm.N, FOLD)
    say(f"{what}: VALU kernels")
    ref = _run(ctx, plan, w.cts, w.level, w.prm.N, VALU)
    assert_bit_exact(got, ref, f"{what}: folded vs VALU")
    pts = O.plan_residues(w.prm, w.plan)
    for k in check:
        assert_bit_exact(got[k], O.lookup(w.prm, w.keys, w.plan, w.cts[k], pts), f"{what}: query {k}")
        rows = W.decrypt_slots(w, got[k], w.prm.delta, len(w.expected[k]))
        assert np.max(np.abs(rows - w.expected[k])) < 1e-4
    return got


@pytest.mark.parametrize("level", [2, 1])
def test_fold_toy_ring(level):
    """Toy ring N=2^12 (one prime per digit: three digits at level 2, two at
    level 1), the 256-row table with n1 = 4 (four giant outputs), batch 17
    (tiles of 16 and 1)."""
    prm = O.config1_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 256, 16, 16, -1.0, 1.0)
    w = W.build(prm, [t], level=level, n1=4, radix=2, n_queries=17)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    assert plan.helrm_plan_fold_keys() > 0
    _check(ctx, w, plan, [0, 16], f"toy level {level}")
    ctx.close()


def test_fold_table1_shape_giant_tiles():
    """d = 768 from 32 base-16 digit tables on the toy ring at level 1: 32
    giant outputs in four tiles, 32 baby steps (two depth chunks), batch 8."""
    prm = O.config1_params()
    w = W.table1_shape(prm, 1, n_queries=8)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    plan.helrm_plan_fold_keys()
    _check(ctx, w, plan, [0, 7], "Table I shape")
    ctx.close()


def test_fold_multi_ciphertext_and_stale_keys():
    """Two selector ciphertexts per query on the toy ring at level 2, batch 8
    (the second block accumulates); then the keys are loaded again, the folded
    words are stale and the same call (now on the other kernels) gives the
    same residues."""
    prm = O.config1_params()
    ctx = context_for(prm)
    g = synth.rng(9)
    tables = [W.uncompressed_table(g, 1000, 16, -1, 1) for _ in range(3)]
    w = W.build_multi(prm, tables, level=2, n1=16, radix=4, n_queries=8)
    load_keys(ctx, w.keys)
    plans = [gpu_plan(ctx, p) for p in w.plans]
    for p in plans:
        p.helrm_plan_fold_keys()
    sel = to_dev(np.stack([np.stack(c) for c in w.cts]))
    outs = []
    for what in ("folded", "valu", "stale"):
        if what == "stale":
            load_keys(ctx, w.keys)
        knobs = VALU if what == "valu" else FOLD
        for k, v in knobs.items():
            ctx.helrm_set_tuning(k, v)
        say(f"multi-ciphertext batch 8 {what}")
        out = empty(8, 2, 2, prm.N)
        ctx.helrm_lookup_multi(plans, sel, 8, out)
        outs.append(to_host(out).reshape(8, 2, 2, prm.N))
    assert_bit_exact(outs[0], outs[1], "multi: folded vs VALU")
    assert_bit_exact(outs[2], outs[1], "multi: stale fold falls back")
    for k in (0, 7):
        assert_bit_exact(outs[0][k], O.lookup_multi(prm, w.keys, w.plans, w.cts[k]), f"multi query {k}")
    ctx.close()


@pytest.mark.timeout(900)
def test_fold_n16_level23_group():
    """The request loop's first table group of the batching workload at level
    23 (three digits, 24 + 8 primes), n1 = 16, radix 8, sign -1, batch 17."""
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
    w = W.build(prm, specs, level=23, n1=16, radix=8, n_queries=17, sign=-1)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    plan.helrm_plan_fold_keys()
    _check(ctx, w, plan, [0, 16], "level 23 group")
    ctx.close()


@pytest.mark.timeout(900)
def test_fold_one_digit_n16_level1():
    """One key-switching digit: the Table I shape (d = 768 from 32 base-16
    digit tables, m = 1024 diagonals, n1 = 32, 32 giant outputs in four
    tiles) at N=2^16 with the selector at level 1 (two Q primes, one digit,
    the level of the token-embedding runs), batch 17 (row tiles of 16 and 1;
    the wide primes share each operand load between the two)."""
    prm = O.config2_params()
    assert prm.n_digits(1) == 1
    w = W.table1_shape(prm, 1, n_queries=17)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    assert plan.helrm_plan_fold_keys() > 0
    _check(ctx, w, plan, [0, 16], "N=2^16 level 1")
    ctx.close()


def test_block_chain_order_off():
    """The matrix-core kernels with the workgroups in plain block order (knob
    block_chain = 0) give the same residues as in chain order: the folded
    product and the matrix-core MAC, toy ring at level 2, batch 17."""
    prm = O.config1_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 256, 16, 16, -1.0, 1.0)
    w = W.build(prm, [t], level=2, n1=4, radix=2, n_queries=17)
    ctx = context_for(prm)
    # four baby steps: below the matrix-core MAC's default floor, so lower it
    # before the plan is made (the plan keeps matrix-core operands only then)
    ctx.helrm_set_tuning("mfma_min_slots", 1)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    plan.helrm_plan_fold_keys()
    MFMA = dict(baby_fold=0, baby_mfma=8)
    outs = {}
    try:
        for chain in (1, 0):
            ctx.helrm_set_tuning("block_chain", chain)
            for what, knobs in (("fold", FOLD), ("mfma", MFMA)):
                say(f"block_chain {chain}: {what}")
                outs[(chain, what)] = _run(ctx, plan, w.cts, w.level, prm.N, knobs)
    finally:
        ctx.helrm_set_tuning("block_chain", 1)
    for k, v in outs.items():
        assert_bit_exact(v, outs[(1, "fold")], f"block_chain {k}")
    pts = O.plan_residues(prm, w.plan)
    assert_bit_exact(outs[(0, "fold")][0], O.lookup(prm, w.keys, w.plan, w.cts[0], pts), "query 0")
    ctx.close()



@pytest.mark.parametrize("shape", ["toy", "table1"])
def test_fold_two_tiles_per_operand_load(shape):
    """Two row tiles of 16 ciphertexts per load of the folded operands (knob
    fold_mp on both digit counts) give the residues of one tile per load: toy
    ring at level 2, batch 40 (tiles 16, 16, 8: the second group holds a
    partial and an absent tile), and the Table I shape at level 1, batch 33
    (two depth chunks); the last query against the oracle."""
    prm = O.config1_params()
    if shape == "toy":
        g = synth.rng(0)
        t = W.compressed_table(g, 256, 16, 16, -1.0, 1.0)
        w = W.build(prm, [t], level=2, n1=4, radix=2, n_queries=40)
    else:
        w = W.table1_shape(prm, 1, n_queries=33)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    plan.helrm_plan_fold_keys()
    outs = {}
    try:
        for mp in (0, 3):
            ctx.helrm_set_tuning("fold_mp", mp)
            say(f"{shape}: fold_mp {mp}, batch {len(w.cts)}")
            outs[mp] = _run(ctx, plan, w.cts, w.level, prm.N, FOLD)
    finally:
        ctx.helrm_set_tuning("fold_mp", 2)
    assert_bit_exact(outs[3], outs[0], "fold_mp 3 vs 0")
    last = len(w.cts) - 1
    pts = O.plan_residues(prm, w.plan)
    assert_bit_exact(outs[3][last], O.lookup(prm, w.keys, w.plan, w.cts[last], pts), f"query {last}")
    ctx.close()
