"""GPU parity of batches over uneven packings (helrm_lookup_batch and its
captured graph): every element goes through its own plan (its own subset of
tables, Sec. IV-B block-diagonal packing), and every residue of every result
equals the oracle's lookup with that plan, bit-exact.  The plans differ in
diagonals, fold span and number of fold stages; the batch order interleaves
them, so the library's regrouping and scatter are exercised."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import assert_bit_exact, context_for, empty, gpu_plan, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _mixed(prm, table_sets, level, n1, radix, sign, order, seed=0):
    """Oracle side: one plan per table set, keys for the union of their
    rotations, and one encrypted query per batch element (element b uses
    table set order[b])."""
    plans = [O.make_plan(prm, O.pack_tables(ts), level, n1, radix, sign) for ts in table_sets]
    steps = sorted({k for p in plans for k in p.rotation_steps()})
    keys = O.keygen(prm, synth.key_draws(seed, prm.N, prm.q, prm.p, prm.dnum,
                                         [O.galois_for_step(k, prm) for k in steps]))
    g = synth.rng(seed + 3000)
    cts, expected = [], []
    for k in order:
        ts = table_sets[k]
        idx = synth.indices(g, [t.rows for t in ts])
        cts.append(O.encrypt(prm, keys, O.encode(O.pack_selector(ts, idx), prm.delta, prm), level,
                             synth.enc_draws(g, prm.N)))
        expected.append(np.concatenate([t.lookup(i) for t, i in zip(ts, idx)]))
    return plans, keys, cts, expected


def _load(ctx, keys):
    import torch
    from paper_2506_18150_amd import binding as B
    for gal, k in sorted(keys.swk.items()):
        ctx.helrm_load_eval_keys([gal], B.device_u64(k), [keys.seeds[gal]])
    torch.cuda.synchronize()


def _check(prm, keys, plans, order, cts, got, expected, what):
    pts = [O.plan_residues(prm, p) for p in plans]
    for b, k in enumerate(order):
        want = O.lookup(prm, keys, plans[k], cts[b], pts[k])
        assert_bit_exact(got[b], want, f"{what}: element {b} (plan {k})")
        m = O.decrypt(prm, keys, got[b])
        rows = O.decode(m, prm.delta, prm)[:len(expected[b])].real
        assert np.max(np.abs(rows - expected[b])) < 1e-4


def _toy_sets():
    g = synth.rng(0)
    t_a = W.uncompressed_table(g, 40, 16, -1, 1)
    t_b = W.compressed_table(g, 256, 16, 16, -1, 1)
    t_c = W.uncompressed_table(g, 100, 16, -1, 1)
    t_d = W.uncompressed_table(g, 7, 16, -1, 1)
    t_e = W.compressed_table(g, 4096, 16, 16, -1, 1)
    # 32 outputs each (m = 32): fold spans 128, 256 and 128 slots
    return [[t_a, t_b], [t_c, t_e], [t_d, t_a]]


@pytest.mark.parametrize("fuse", [1, 0])
def test_mixed_batch_toy_ring(fuse):
    """Toy ring N=2^12 at level 3, n1 = 8 (four giant outputs), radix 2, sign
    -1; three plans of two tables each with different widths and fold spans,
    batch of 6 in interleaved order; fused boundaries and the plain order."""
    prm = O.config1_params()
    sets = _toy_sets()
    order = [1, 0, 2, 1, 0, 0]
    plans, keys, cts, expected = _mixed(prm, sets, prm.L, 8, 2, -1, order)
    assert len({len(p.stages) for p in plans}) > 1, [p.stages for p in plans]
    ctx = context_for(prm)
    _load(ctx, keys)
    gp = [gpu_plan(ctx, p) for p in plans]
    try:
        ctx.helrm_set_tuning("fuse_ks", fuse)
        say(f"mixed batch toy ring fuse_ks={fuse} order={order}")
        out = empty(len(order), 2, prm.L, prm.N)
        ctx.helrm_lookup_batch([gp[k] for k in order], to_dev(np.stack(cts)), out)
        got = to_host(out).reshape(len(order), 2, prm.L, prm.N)
    finally:
        ctx.helrm_set_tuning("fuse_ks", 1)
    _check(prm, keys, plans, order, cts, got, expected, f"fuse_ks={fuse}")
    # each element also equals helrm_lookup_packed with its own plan, alone
    for b in (0, 2):
        one = empty(1, 2, prm.L, prm.N)
        ctx.helrm_lookup_packed(gp[order[b]], to_dev(cts[b][None]), 1, one)
        assert_bit_exact(to_host(one).reshape(2, prm.L, prm.N), got[b], f"element {b} alone")
    ctx.close()


def test_mixed_batch_graph_n16():
    """N=2^16 at level 4: request-loop table groups (the first 14 of the 26
    tables of the batching workload: three groups of 4, four giant outputs, and
    one group of 2, two giant outputs; n1 = 16, radix 8, sign -1) as one mixed
    batch of 8 ciphertexts, run eagerly and replayed twice from a captured
    graph (with other work in between)."""
    import torch
    prm = O.config2_params()
    _, counts = synth.criteo_like_row_counts()
    g = synth.rng(0)
    specs = []
    for k in counts[:14]:
        if k <= 256:
            specs.append(O.TableSpec(rows=k, d=16, E=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(O.num_digits(k, 256))]
            specs.append(O.TableSpec(rows=k, d=16, base=256, C=C))
    sets = [specs[0:4], specs[4:8], specs[8:12], specs[12:14]]
    order = [2, 0, 3, 1, 0, 2, 2, 1]
    plans, keys, cts, expected = _mixed(prm, sets, 4, 16, 8, -1, order)
    assert [p.n2 for p in plans] == [4, 4, 4, 2]
    ctx = context_for(prm)
    _load(ctx, keys)
    gp = [gpu_plan(ctx, p) for p in plans]
    B = len(order)
    sel = to_dev(np.stack(cts))
    say(f"mixed batch N=2^16 level 4 eager, order={order}")
    out = empty(B, 2, 4, prm.N)
    ctx.helrm_lookup_batch([gp[k] for k in order], sel, out)
    eager = to_host(out).reshape(B, 2, 4, prm.N)
    _check(prm, keys, plans, order, cts, eager, expected, "eager")
    say("mixed batch N=2^16 level 4 graph")
    gout = empty(B, 2, 4, prm.N)
    graph = ctx.helrm_batch_graph_create_mixed([gp[k] for k in order], sel, gout)
    for rep in range(2):
        gout.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert_bit_exact(to_host(gout).reshape(B, 2, 4, prm.N), eager, f"graph replay {rep}")
        # other work on the device between replays
        ctx.helrm_lookup_packed(gp[0], sel[1:2].contiguous(), 1, empty(1, 2, 4, prm.N))
        torch.cuda.synchronize()
    graph.close()
    ctx.close()


def test_mixed_batch_rejects_incompatible_plans():
    """Plans with different n1 cannot share a batch: HELRM_EINVAL on the host."""
    from paper_2506_18150_amd import binding as B
    prm = O.config1_params()
    sets = _toy_sets()
    p8 = O.make_plan(prm, O.pack_tables(sets[0]), prm.L, 8, 2, -1)
    p4 = O.make_plan(prm, O.pack_tables(sets[1]), prm.L, 4, 2, -1)
    ctx = context_for(prm)
    a, b = gpu_plan(ctx, p8), gpu_plan(ctx, p4)
    sel = empty(2, 2, prm.L + 1, prm.N)
    with pytest.raises(B.HelrmError) as e:
        ctx.helrm_lookup_batch([a, b], sel, empty(2, 2, prm.L, prm.N))
    assert e.value.code == -1
    ctx.close()
