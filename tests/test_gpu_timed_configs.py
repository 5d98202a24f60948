"""GPU parity of the configurations the benchmark and the request loop time,
and of the C-ABI calls at full size (N=2^16, level 23), against the oracle,
bit-exact on every residue.

* The headline workload (one 65,536-row table as two base-256 digit tables,
  selector at level 23) with the schedule and kernel knobs the benchmark takes
  from the autotuner's records, at batch 1 and batch 8.
* The batching workload at full size (26 tables packed into a 416 x 13,962
  matrix, m = 512 diagonals, n1 = 64, fold radix 8, rotation sign -1, three
  key-switching digits at level 23) with the batch-64 and batch-8 knobs,
  batch 64 replayed from the captured graph of the C ABI.
* A table group of the request loop (4 tables, m = 64, n1 = 16) at every
  workgroup width the loop's batches of 1..16 select.
* helrm_keyswitch_hoisted and helrm_mul_relin at level 23, and the GPU
  client's key generation and encryption against the oracle's from the same
  draws.
Double-hoisted BSGS product: Sec. III-B; packing: Sec. IV-B; key switching,
rotation, multiplication, encryption: Appendix A."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import (assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev,
                               to_host)

pytestmark = pytest.mark.gpu

KNOBS = ("ks_tile", "baby_tile", "baby_share", "ntt_col_w", "ntt_blk_w", "baby_mfma", "baby_fold")
DEFAULT_KNOBS = dict(ks_tile=4, baby_tile=4, baby_share=8, ntt_col_w=16, ntt_blk_w=4, baby_mfma=8, baby_fold=8)


def tuned(rows, cols, batch, level=23):
    """The autotuner's record the benchmark uses for this workload shape."""
    from paper_2506_18150_amd import autotune, params
    prm = params.n16()
    sc = autotune.tuned_schedule(prm.N, prm.L, level, rows, cols, batch)
    assert sc is not None, f"no tuning record for {rows}x{cols} batch {batch}"
    return sc


def set_knobs(ctx, sc):
    for k in KNOBS:
        ctx.helrm_set_tuning(k, getattr(sc, k))


def reset_knobs(ctx):
    for k, v in DEFAULT_KNOBS.items():
        ctx.helrm_set_tuning(k, v)


@pytest.fixture(scope="module")
def p2():
    return O.config2_params()


@pytest.fixture(scope="module")
def ctx2(p2):
    return context_for(p2)


def _w2(sc, n_queries):
    prm = O.config2_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 65536, 16, 256, -0.05, 0.05)
    return W.build(prm, [t], level=23, n1=sc.n1, radix=sc.radix, n_queries=n_queries, sign=sc.sign)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("batch", [1, 8])
def test_headline_workload_tuned_schedule(batch, ctx2):
    """One 65,536-row table at level 23 with the benchmark's tuned schedule
    (n1, radix, direction) and kernel knobs (key-switch and baby-step tiles,
    NTT workgroup shapes) for this batch size: every ciphertext of the batch
    bit-exact against the oracle."""
    sc = tuned(16, 512, batch)
    w = _w2(sc, batch)
    load_keys(ctx2, w.keys)
    plan = gpu_plan(ctx2, w.plan)
    set_knobs(ctx2, sc)
    try:
        say(f"headline workload tuned batch={batch} knobs={[getattr(sc, k) for k in KNOBS]}")
        out = empty(batch, 2, 23, w.prm.N)
        ctx2.helrm_lookup_packed(plan, to_dev(np.stack(w.cts)), batch, out)
        got = to_host(out).reshape(batch, 2, 23, w.prm.N)
    finally:
        reset_knobs(ctx2)
    pts = O.plan_residues(w.prm, w.plan)
    for k in range(batch):
        assert_bit_exact(got[k], O.lookup(w.prm, w.keys, w.plan, w.cts[k], pts), f"query {k}")
        assert np.max(np.abs(W.decrypt_slots(w, got[k], w.prm.delta, 16) - w.expected[k])) < 1e-4


def _w3_specs():
    """The 26 tables of the batching workload, as the benchmark draws them."""
    _, counts = synth.criteo_like_row_counts()
    specs = []
    g = synth.rng(0)
    for k in counts:
        if k <= 256:
            specs.append(O.TableSpec(rows=k, d=16, E=synth.uniform_table(g, k, 16, -0.05, 0.05)))
        else:
            C = [synth.uniform_table(g, 256, 16, -0.05, 0.05) for _ in range(O.num_digits(k, 256))]
            specs.append(O.TableSpec(rows=k, d=16, base=256, C=C))
    return specs


@pytest.mark.timeout(1200)
def test_batching_workload_full_size_bit_exact():
    """26 tables in one selector ciphertext per query (m = 512, n1 = 64, n2 =
    8, radix 8, sign -1, level 23: three digits), the plan's keys folded as
    the benchmark does, batch 64 through the captured graph with the batch-64
    knobs, the first 8 eagerly with the batch-8 knobs, query 63 alone with the
    batch-1 knobs, and the first 3 and 12 with the default knobs (the request
    loop's batches on this plan): queries 0 and 63 bit-exact against the
    oracle, every other run equal to the batch-64 one on its queries."""
    import torch
    prm = O.config2_params()
    specs = _w3_specs()
    B = 64
    say("batching workload: oracle keys, plan and 64 encryptions")
    w = W.build(prm, specs, level=23, n1=64, radix=8, n_queries=B, sign=-1)
    assert w.plan.m == 512 and w.plan.n2 == 8 and prm.n_digits(23) == 3
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    plan.helrm_plan_fold_keys()   # as the benchmark's session does for batches
    sel = to_dev(np.stack(w.cts))
    sc64 = tuned(416, 13962, 64)
    assert (sc64.n1, sc64.radix, sc64.sign) == (64, 8, -1)
    set_knobs(ctx, sc64)
    out = empty(B, 2, 23, prm.N)
    say(f"batching workload: graph capture + replay, batch {B}")
    g = ctx.helrm_batch_graph_create([plan], sel, B, out)
    g.replay()
    torch.cuda.synchronize()
    got = to_host(out).reshape(B, 2, 23, prm.N)
    g.close()
    del g
    torch.cuda.synchronize()
    sc8 = tuned(416, 13962, 8)
    set_knobs(ctx, sc8)
    say("batching workload: eager batch 8")
    out8 = empty(8, 2, 23, prm.N)
    ctx.helrm_lookup_packed(plan, sel[:8].contiguous(), 8, out8)
    got8 = to_host(out8).reshape(8, 2, 23, prm.N)
    sc1 = tuned(416, 13962, 1)
    set_knobs(ctx, sc1)
    say("batching workload: query 63 alone with the batch-1 knobs")
    out1 = empty(1, 2, 23, prm.N)
    ctx.helrm_lookup_packed(plan, sel[B - 1:].contiguous(), 1, out1)
    got1 = to_host(out1).reshape(1, 2, 23, prm.N)
    reset_knobs(ctx)
    # the request loop's batches on this plan with the library's default
    # knobs: 3 (workgroup-shared VALU kernel) and 12 (folded product, one
    # partial row tile)
    loop = {}
    for b in (3, 12):
        say(f"batching workload: eager batch {b}, default knobs")
        ob = empty(b, 2, 23, prm.N)
        ctx.helrm_lookup_packed(plan, sel[:b].contiguous(), b, ob)
        loop[b] = to_host(ob).reshape(b, 2, 23, prm.N)
        del ob
    del sel, out, out8, out1
    assert_bit_exact(got8[0], got[0], "query 0: batch 8 eager vs batch 64 graph")
    assert_bit_exact(got1[0], got[B - 1], "query 63: batch 1 vs batch 64 graph")
    for b, res in loop.items():
        for k in range(b):
            assert_bit_exact(res[k], got[k], f"query {k}: batch {b} vs batch 64 graph")
    say("batching workload: oracle lookups of queries 0 and 63")
    pts = O.plan_residues(prm, w.plan)
    for k in (0, B - 1):
        assert_bit_exact(got[k], O.lookup(prm, w.keys, w.plan, w.cts[k], pts), f"query {k}")
        rows = W.decrypt_slots(w, got[k], prm.delta, 416)
        assert np.max(np.abs(rows - w.expected[k])) < 1e-4
    ctx.close()


@pytest.mark.timeout(900)
def test_serving_group_plan_every_width():
    """A table group of the request loop (the first 4 of the 26 tables, level
    23, n1 = 16, radix 8, sign -1: m = 64, four giant outputs) at batches 1, 2,
    3 and 11 with the loop's default knobs: the per-thread kernel (batch 1) and
    the workgroup-shared kernel at widths 2, 4 and 8 (11 = a tile of 8 and a
    ragged tile of 3); every ciphertext bit-exact against the oracle."""
    prm = O.config2_params()
    specs = _w3_specs()[:4]
    w = W.build(prm, specs, level=23, n1=16, radix=8, n_queries=11, sign=-1)
    assert w.plan.m == 64 and w.plan.n2 == 4
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    pts = O.plan_residues(prm, w.plan)
    want = [O.lookup(prm, w.keys, w.plan, w.cts[k], pts) for k in range(11)]
    for b in (1, 2, 3, 11):
        say(f"serving group plan batch={b}")
        out = empty(b, 2, 23, prm.N)
        ctx.helrm_lookup_packed(plan, to_dev(np.stack(w.cts[:b])), b, out)
        got = to_host(out).reshape(b, 2, 23, prm.N)
        for k in range(b):
            assert_bit_exact(got[k], want[k], f"batch {b} query {k}")
    ctx.close()


@pytest.mark.timeout(600)
def test_keyswitch_hoisted_full_size(p2, ctx2):
    """helrm_keyswitch_hoisted at N=2^16, level 23 (three digits), batch 2,
    steps {1, 0, -3, 512}: the PQ outputs equal the oracle's key inner
    products and the Q outputs their ModDown."""
    from paper_2506_18150_amd import binding as B
    prm, level = p2, 23
    steps = [1, 0, -3, 512]
    gals = sorted({O.galois_for_step(s, prm) for s in steps if s})
    keys = O.keygen(prm, synth.key_draws(3, prm.N, prm.q, prm.p, prm.dnum, gals))
    load_keys(ctx2, keys)
    g = synth.rng(80)
    cts = np.stack([O.encrypt(prm, keys, O.encode(g.uniform(-1, 1, prm.n), prm.delta, prm), level,
                              synth.enc_draws(g, prm.N)) for _ in range(2)])
    pqn = level + 1 + prm.K
    say(f"keyswitch_hoisted N={prm.N} level={level} steps={steps} batch=2")
    outpq = empty(2, len(steps), 2, pqn, prm.N)
    ctx2.helrm_keyswitch_hoisted(to_dev(cts), level, steps, outpq, B.HELRM_BASIS_PQ, 2)
    outq = empty(2, len(steps), 2, level + 1, prm.N)
    ctx2.helrm_keyswitch_hoisted(to_dev(cts), level, steps, outq, B.HELRM_BASIS_Q, 2)
    gpq = to_host(outpq).reshape(2, len(steps), 2, pqn, prm.N)
    gq = to_host(outq).reshape(2, len(steps), 2, level + 1, prm.N)
    for b in range(2):
        d = O.modup(prm, cts[b][1], level)
        for i, s in enumerate(steps):
            if s == 0:
                assert_bit_exact(gpq[b, i], O.lift_P(prm, cts[b], level), "step 0 (PQ)")
                assert_bit_exact(gq[b, i], cts[b], "step 0 (Q)")
                continue
            gal = O.galois_for_step(s, prm)
            want = O.key_inner_product(prm, d, cts[b][0], level, keys.swk[gal], gal)
            assert_bit_exact(gpq[b, i], want, f"batch {b} step {s} (PQ)")
            assert_bit_exact(gq[b, i], O.moddown(prm, want, level), f"batch {b} step {s} (Q)")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("level", [23, 8])
def test_mul_relin_full_size(level, p2, ctx2):
    """helrm_mul_relin at N=2^16 (level 23: three digits; level 8: two),
    batch 2, product and square, against the oracle."""
    import torch
    from paper_2506_18150_amd import binding as B
    prm = p2
    keys = O.keygen(prm, synth.key_draws(4, prm.N, prm.q, prm.p, prm.dnum, [], relin=True))
    ctx2.helrm_load_eval_keys([0], B.device_u64(keys.relin), [keys.seeds[0]])
    torch.cuda.synchronize()
    g = synth.rng(90 + level)
    mk = lambda: O.encrypt(prm, keys, O.encode(g.uniform(-1, 1, prm.n), prm.delta, prm), level,
                           synth.enc_draws(g, prm.N))
    a = np.stack([mk(), mk()])
    b = np.stack([mk(), mk()])
    say(f"mul_relin N={prm.N} level={level} batch=2")
    out = empty(2, 2, level + 1, prm.N)
    ctx2.helrm_mul_relin(to_dev(a), to_dev(b), level, out, 2)
    sq = empty(2, 2, level + 1, prm.N)
    da = to_dev(a)
    ctx2.helrm_mul_relin(da, da, level, sq, 2)
    got, gsq = to_host(out), to_host(sq)
    for k in range(2):
        assert_bit_exact(got[k], O.mul_relin(prm, keys, a[k], b[k], level), f"mul_relin {k}")
        assert_bit_exact(gsq[k], O.mul_relin(prm, keys, a[k], a[k], level), f"square {k}")


@pytest.mark.timeout(600)
def test_client_keys_and_encryption_match_oracle():
    """The product's GPU client (used by the benchmark and the request loop)
    builds the same secret, public key, rotation and relinearisation keys and
    ciphertexts as the oracle from the same draws, residue for residue."""
    import torch
    from paper_2506_18150_amd import params
    from paper_2506_18150_amd.binding import Context
    from paper_2506_18150_amd.client import Client
    prm = O.config2_params()
    ps = params.n16()
    assert list(ps.q) == list(prm.q) and list(ps.p) == list(prm.p)
    gals = [O.galois_for_step(k, prm) for k in (1, -16, 1024)]
    draws = synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals, relin=True)
    keys = O.keygen(prm, draws)
    ctx = Context(ps.log_n, ps.q, ps.p, ps.alpha)
    cl = Client(ctx, ps)
    say("client keygen N=2^16")
    cl.keygen(draws, sorted(gals))
    assert_bit_exact(to_host(cl.s_all), keys.s, "secret")
    assert_bit_exact(to_host(cl.pk[0]), keys.pk[0], "public key b")
    assert_bit_exact(to_host(cl.pk[1]), keys.pk[1], "public key a")
    for gal in sorted(gals):
        sg = torch.zeros(prm.L + 1 + prm.K, prm.N, dtype=torch.int64, device="cuda")
        ctx.helrm_automorph(cl.s_all, sg, gal, prm.L + 1 + prm.K, 1)
        assert_bit_exact(to_host(cl.switch_key(sg, draws.swk[gal])).reshape(keys.swk[gal].shape),
                         keys.swk[gal], f"switching key {gal}")
    s2 = torch.zeros_like(cl.s_all)
    from paper_2506_18150_amd.binding import HELRM_OP_MUL
    allp = list(range(prm.L + 1 + prm.K))
    ctx.helrm_poly_op(HELRM_OP_MUL, cl.s_all, cl.s_all, s2, allp, 1)
    assert_bit_exact(to_host(cl.switch_key(s2, draws.relin)).reshape(keys.relin.shape), keys.relin,
                     "relinearisation key")
    g = synth.rng(95)
    for level in (23, 4):
        m = O.encode(g.uniform(-1, 1, prm.n), prm.delta, prm)
        ed = synth.enc_draws(g, prm.N)
        say(f"client encrypt level={level}")
        assert_bit_exact(to_host(cl.encrypt(m, level, ed)), O.encrypt(prm, keys, m, level, ed),
                         f"encryption at level {level}")
    ctx.close()
