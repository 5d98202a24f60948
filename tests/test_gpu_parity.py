"""GPU parity: every libhelrm call against the CPU oracle, bit-exact on every
residue, on the same seeded inputs (oracle-made keys, plans and ciphertexts)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import (assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev,
                               to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def p1():
    return O.config1_params()


@pytest.fixture(scope="module")
def p2():
    return O.config2_params()


@pytest.fixture(scope="module")
def ctx1(p1):
    return context_for(p1)


@pytest.fixture(scope="module")
def ctx2(p2):
    return context_for(p2)


def rand_limbs(rng, moduli, N, batch=1):
    return np.stack([np.stack([rng.integers(0, q, size=N, dtype=np.uint64) for q in moduli])
                     for _ in range(batch)])


def test_roots_match(p1, p2, ctx1, ctx2):
    say("roots")
    for prm, ctx in ((p1, ctx1), (p2, ctx2)):
        for i, q in enumerate(prm.q + prm.p):
            assert ctx.helrm_get_psi(i) == prm.psi[q]


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_ntt_parity(which, p1, p2, ctx1, ctx2):
    prm, ctx = (p1, ctx1) if which == "cfg1" else (p2, ctx2)
    allm = prm.q + prm.p
    rng = np.random.default_rng(10)
    # batch of 3, every prime once, plus a ragged list that repeats primes
    for pidx, batch in ((list(range(len(allm))), 3), ([0, 2, 2, len(allm) - 1, 1], 2)):
        say(f"ntt {which} primes={pidx} batch={batch}")
        mods = [allm[i] for i in pidx]
        x = rand_limbs(rng, mods, prm.N, batch)
        d = to_dev(x)
        ctx.helrm_ntt(d, pidx, batch)
        got = to_host(d).reshape(x.shape)
        for b in range(batch):
            assert_bit_exact(got[b], O.ntt(x[b], mods, prm), f"ntt batch {b}")
        ctx.helrm_intt(d, pidx, batch)
        assert_bit_exact(to_host(d).reshape(x.shape), x, "intt(ntt(x))")
        ctx.helrm_intt(d, pidx, batch)
        got = to_host(d).reshape(x.shape)
        for b in range(batch):
            assert_bit_exact(got[b], O.intt(x[b], mods, prm), f"intt batch {b}")


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
@pytest.mark.parametrize("wc,wb", [(8, 4), (8, 8), (16, 8)])
def test_ntt_parity_other_shapes(which, wc, wb, p1, p2, ctx1, ctx2):
    """The other workgroup shapes of both NTT passes (the default, 16 columns
    and 4 blocks, is covered above), forward and inverse, bit-exact."""
    prm, ctx = (p1, ctx1) if which == "cfg1" else (p2, ctx2)
    allm = prm.q + prm.p
    rng = np.random.default_rng(11)
    pidx, batch = list(range(len(allm))), 2
    mods = [allm[i] for i in pidx]
    x = rand_limbs(rng, mods, prm.N, batch)
    say(f"ntt {which} shape col {wc} blk {wb}")
    ctx.helrm_set_tuning("ntt_col_w", wc)
    ctx.helrm_set_tuning("ntt_blk_w", wb)
    try:
        d = to_dev(x)
        ctx.helrm_ntt(d, pidx, batch)
        got = to_host(d).reshape(x.shape)
        for b in range(batch):
            assert_bit_exact(got[b], O.ntt(x[b], mods, prm), f"ntt batch {b}")
        ctx.helrm_intt(d, pidx, batch)
        assert_bit_exact(to_host(d).reshape(x.shape), x, "intt(ntt(x))")
    finally:
        ctx.helrm_set_tuning("ntt_col_w", 16)
        ctx.helrm_set_tuning("ntt_blk_w", 4)


@pytest.mark.parametrize("n1,batch", [(16, 1), (4, 3)])
def test_lookup_ks_chain(n1, batch, p2, ctx2):
    """The key-switching kernels with their workgroups in chain order of the
    coefficient blocks (knob ks_chain): a lookup at N=2^16, level 4, on the
    per-thread baby-step kernel (n1 = 16, one giant output, batch 1) and on
    the workgroup-shared one (n1 = 4, four giant outputs, batch 3), bit-exact
    against the oracle and equal to the plain order."""
    g = synth.rng(3)
    t = W.compressed_table(g, 65536, 16, 256, -0.05, 0.05)
    w = W.build(p2, [t], level=4, n1=n1, radix=4, n_queries=batch, sign=-1)
    load_keys(ctx2, w.keys)
    plan = gpu_plan(ctx2, w.plan)
    outs = []
    try:
        for chain in (1, 0):
            ctx2.helrm_set_tuning("ks_chain", chain)
            say(f"lookup N=2^16 level 4 n1={n1} batch {batch}, ks_chain {chain}")
            out = empty(batch, 2, 4, p2.N)
            ctx2.helrm_lookup_packed(plan, to_dev(np.stack(w.cts)), batch, out)
            outs.append(to_host(out).reshape(batch, 2, 4, p2.N))
    finally:
        ctx2.helrm_set_tuning("ks_chain", 1)
    assert_bit_exact(outs[0], outs[1], "ks_chain 1 vs 0")
    pts = O.plan_residues(p2, w.plan)
    for k in range(batch):
        assert_bit_exact(outs[0][k], O.lookup(p2, w.keys, w.plan, w.cts[k], pts), f"ks_chain query {k}")


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_key_uniform_parity(which, p1, p2, ctx1, ctx2):
    """Seeded key polynomials expanded on the GPU equal the oracle's expansion,
    including a seed whose 64-bit sample on a prime below 2^40 is rejected and
    redrawn (541 on the toy ring, 1208 at N=2^16)."""
    prm, ctx = (p1, ctx1) if which == "cfg1" else (p2, ctx2)
    for seed in (0, 0x0123456789ABCDEF, 2 ** 63 - 1, 541 if which == "cfg1" else 1208):
        for j in range(prm.dnum):
            say(f"key_uniform {which} seed={seed} digit={j}")
            out = empty(len(prm.q) + len(prm.p), prm.N)
            ctx.helrm_key_uniform(seed, j, out)
            assert_bit_exact(to_host(out), O.key_uniform(prm, seed, j), f"key_uniform digit {j}")


def test_ntt_edge_values(p2, ctx2):
    say("ntt edge values q-1 / 0")
    prm, ctx = p2, ctx2
    mods = prm.q[:2] + prm.p[:1]
    pidx = [0, 1, prm.L + 1]
    x = np.stack([np.full(prm.N, q - 1, dtype=np.uint64) for q in mods])
    x[1, ::3] = 0
    d = to_dev(x)
    ctx.helrm_ntt(d, pidx, 1)
    assert_bit_exact(to_host(d).reshape(x.shape), O.ntt(x, mods, prm), "ntt of q-1")


def test_automorph_parity(p1, p2, ctx1, ctx2):
    rng = np.random.default_rng(11)
    for prm, ctx in ((p1, ctx1), (p2, ctx2)):
        for k in (1, 5, prm.n - 1, prm.n // 2):
            g = O.galois_for_step(k, prm)
            say(f"automorph N={prm.N} g={g}")
            x = rand_limbs(rng, prm.q[:3], prm.N, 2)
            out = empty(*x.shape)
            ctx.helrm_automorph(to_dev(x), out, g, 3, 2)
            got = to_host(out).reshape(x.shape)
            for b in range(2):
                assert_bit_exact(got[b], O.automorph_ntt(x[b], g, prm.N), "automorph")


def test_empty_calls_enqueue_nothing(ctx1, w1):
    """Every call that takes a batch accepts an empty one (batch 0, or no
    limbs or rotations) with NULL buffers and returns HELRM_OK without
    enqueueing work; a batch graph needs an element.  The context keeps
    working: a lookup afterwards matches the oracle."""
    import ctypes
    from paper_2506_18150_amd import binding as B
    L = B.lib()
    h, lv = ctx1.h, w1.level
    pidx = np.arange(3, dtype=np.int32)
    pp = pidx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    steps = np.array([1], dtype=np.int32)
    sp = steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    plan = gpu_plan(ctx1, w1.plan)
    plans = (ctypes.c_void_p * 1)(plan.h.value if hasattr(plan.h, "value") else plan.h)
    calls = {
        "ntt, batch 0": lambda: L.helrm_ntt(h, None, 3, pp, 0, None),
        "ntt, no limbs": lambda: L.helrm_ntt(h, None, 0, None, 4, None),
        "intt, batch 0": lambda: L.helrm_intt(h, None, 3, pp, 0, None),
        "automorph": lambda: L.helrm_automorph(h, None, None, 5, 3, 0, None),
        "poly_op": lambda: L.helrm_poly_op(h, B.HELRM_OP_ADD, None, None, None, 3, pp, 0, None),
        "mul_scalar": lambda: L.helrm_mul_scalar(h, None, None, None, 3, pp, 0, None),
        "from_signed": lambda: L.helrm_from_signed(h, None, None, 3, pp, 0, None),
        "keyswitch_hoisted, batch 0": lambda: L.helrm_keyswitch_hoisted(h, None, lv, sp, 1, None, 1, 0, None),
        "keyswitch_hoisted, no rotations": lambda: L.helrm_keyswitch_hoisted(h, None, lv, None, 0, None, 1, 2,
                                                                             None),
        "rescale": lambda: L.helrm_rescale(h, None, lv, None, 0, None),
        "mul_relin": lambda: L.helrm_mul_relin(h, None, None, lv, None, 0, None),
        "add_plain": lambda: L.helrm_add_plain(h, None, None, lv, None, 0, None),
        "mod_drop": lambda: L.helrm_mod_drop(h, None, lv, None, 1, 0, None),
        "ptxt_ct_matvec_diag": lambda: L.helrm_ptxt_ct_matvec_diag(h, plan.h, None, None, 0, None),
        "lookup_packed": lambda: L.helrm_lookup_packed(h, plan.h, None, 0, None, None),
        "lookup_packed_noalloc": lambda: L.helrm_lookup_packed_noalloc(h, plan.h, None, 0, None, None),
        "lookup_multi": lambda: L.helrm_lookup_multi(h, plans, 1, None, 0, None, None),
        "lookup_batch": lambda: L.helrm_lookup_batch(h, plans, None, 0, None, None),
    }
    for what, call in calls.items():
        say(f"empty call: {what}")
        assert call() == B.HELRM_OK, f"{what}: {L.helrm_last_error()}"
    g = ctypes.c_void_p()
    assert L.helrm_batch_graph_create(h, plans, 1, None, 0, None, ctypes.byref(g)) == B.HELRM_EINVAL
    say("empty calls done; a lookup on the same context")
    _check_lookup(ctx1, w1, plan, [0])


def test_tuning_knobs_validate(p1):
    """Every schedule knob accepts its documented values and rejects the
    others (and unknown names) with HELRM_EINVAL, leaving the context usable."""
    from paper_2506_18150_amd import binding as B
    ctx = context_for(p1)
    good = {"ks_tile": [1, 2, 4], "baby_tile": [1, 2, 4], "baby_share": [1, 2, 4, 8], "ntt_col_w": [0, 8, 16],
            "ntt_blk_w": [0, 4, 8], "ntt_small_limbs": [0, 48], "gen_key_a": [0, 1, 2], "limb_xcd": [0, 1],
            "fuse_ks": [0, 1], "fuse_conv": [0, 1], "conv_wgs": [0, 2048], "ks_chain": [0, 1],
            "block_chain": [0, 1], "baby_mfma": [0, 8], "baby_fold": [0, 8], "ptm": [0, 1],
            "mfma_min_slots": [0, 64, 33], "fold_mp": [0, 3, 2]}
    bad = {"ks_tile": [0, 3, 8], "baby_tile": [0, 3], "baby_share": [0, 3, 16], "ntt_col_w": [4, 32],
           "ntt_blk_w": [2, 16], "ntt_small_limbs": [-1], "gen_key_a": [-1, 3], "limb_xcd": [2],
           "fuse_ks": [2], "fuse_conv": [2, -1], "conv_wgs": [-1], "ks_chain": [2, -1], "block_chain": [2],
           "baby_mfma": [-1], "baby_fold": [-1], "ptm": [2], "mfma_min_slots": [-1, 65], "fold_mp": [-1, 4]}
    for knob, vals in good.items():
        for v in vals:
            ctx.helrm_set_tuning(knob, v)
    for knob, vals in bad.items():
        for v in vals:
            with pytest.raises(B.HelrmError):
                ctx.helrm_set_tuning(knob, v)
    with pytest.raises(B.HelrmError):
        ctx.helrm_set_tuning("no_such_knob", 1)
    assert ctx.helrm_get_psi(0) > 1


def test_elementwise_parity(p2, ctx2):
    prm, ctx = p2, ctx2
    from paper_2506_18150_amd import binding as B
    rng = np.random.default_rng(12)
    pidx = [0, 5, prm.L + 2]
    mods = [(prm.q + prm.p)[i] for i in pidx]
    a = rand_limbs(rng, mods, prm.N, 2)
    b = rand_limbs(rng, mods, prm.N, 2)
    da, db = to_dev(a), to_dev(b)
    for op, fn in ((B.HELRM_OP_ADD, O.add), (B.HELRM_OP_SUB, O.sub), (B.HELRM_OP_MUL, O.mul)):
        say(f"poly_op {op}")
        out = empty(*a.shape)
        ctx.helrm_poly_op(op, da, db, out, pidx, 2)
        got = to_host(out).reshape(a.shape)
        for k in range(2):
            assert_bit_exact(got[k], fn(a[k], b[k], mods), f"op {op}")
    out = empty(*a.shape)
    ctx.helrm_poly_op(B.HELRM_OP_NEG, da, None, out, pidx, 2)
    assert_bit_exact(to_host(out).reshape(a.shape)[1], O.neg(a[1], mods), "neg")
    sc = [3, mods[1] - 1, 2 ** 59 + 12345]
    out = empty(*a.shape)
    ctx.helrm_mul_scalar(da, sc, out, pidx, 2)
    assert_bit_exact(to_host(out).reshape(a.shape)[0], O.mul_scalar(a[0], sc, mods), "mul_scalar")
    say("from_signed")
    import torch
    v = rng.integers(-2 ** 62, 2 ** 62, size=(2, prm.N), dtype=np.int64)
    v[0, :4] = [0, -1, 2 ** 63 - 1, -2 ** 63]
    out = empty(2, 3, prm.N)
    ctx.helrm_from_signed(torch.from_numpy(v).cuda(), out, pidx, 2)
    got = to_host(out).reshape(2, 3, prm.N)
    for k in range(2):
        assert_bit_exact(got[k], O.from_signed(v[k], mods), "from_signed")


@pytest.fixture(scope="module")
def w1(ctx1):
    w = W.config1(n_queries=3)
    load_keys(ctx1, w.keys)
    return w


def test_rescale_parity(p1, p2, ctx1, ctx2):
    rng = np.random.default_rng(13)
    for prm, ctx, levels in ((p1, ctx1, (3, 1)), (p2, ctx2, (23, 4, 1))):
        for lv in levels:
            say(f"rescale N={prm.N} level={lv}")
            ct = rand_limbs(rng, prm.Q(lv), prm.N, 2).reshape(1, 2, lv + 1, prm.N)
            ct = np.concatenate([ct, ct[:, ::-1]])   # batch of 2
            out = empty(2, 2, lv, prm.N)
            ctx.helrm_rescale(to_dev(ct), lv, out, 2)
            got = to_host(out).reshape(2, 2, lv, prm.N)
            for b in range(2):
                assert_bit_exact(got[b], O.rescale(prm, ct[b], lv), f"rescale level {lv}")


@pytest.mark.parametrize("level", [3, 2, 0])
def test_keyswitch_hoisted_parity_cfg1(level, p1, ctx1, w1):
    from paper_2506_18150_amd import binding as B
    prm = p1
    steps = [1, 0, 3, 1024]
    for k in steps:
        if k:
            assert O.galois_for_step(k, prm) in w1.keys.swk or True
    steps = [s for s in steps if s == 0 or O.galois_for_step(s, prm) in w1.keys.swk]
    ct = w1.cts[0][:, : level + 1].copy()
    ct2 = np.stack([ct, w1.cts[1][:, : level + 1]])
    say(f"keyswitch_hoisted cfg1 level={level} steps={steps}")
    pqn = level + 1 + prm.K
    outpq = empty(2, len(steps), 2, pqn, prm.N)
    ctx1.helrm_keyswitch_hoisted(to_dev(ct2), level, steps, outpq, B.HELRM_BASIS_PQ, 2)
    outq = empty(2, len(steps), 2, level + 1, prm.N)
    ctx1.helrm_keyswitch_hoisted(to_dev(ct2), level, steps, outq, B.HELRM_BASIS_Q, 2)
    gpq = to_host(outpq).reshape(2, len(steps), 2, pqn, prm.N)
    gq = to_host(outq).reshape(2, len(steps), 2, level + 1, prm.N)
    for b in range(2):
        d = O.modup(prm, ct2[b][1], level)
        for i, s in enumerate(steps):
            if s == 0:
                want = O.lift_P(prm, ct2[b], level)
                assert_bit_exact(gq[b, i], ct2[b], "step 0 (Q)")
            else:
                g = O.galois_for_step(s, prm)
                want = O.key_inner_product(prm, d, ct2[b][0], level, w1.keys.swk[g], g)
                assert_bit_exact(gq[b, i], O.moddown(prm, want, level), f"KS step {s} (Q)")
            assert_bit_exact(gpq[b, i], want, f"KS step {s} (PQ)")


def _check_lookup(ctx, w, plan_gpu, batch_idx):
    prm = w.prm
    lv = w.level
    cts = np.stack([w.cts[i] for i in batch_idx])
    B_ = len(batch_idx)
    say(f"matvec N={prm.N} level={lv} n1={w.plan.n1} radix={w.plan.radix} batch={B_}")
    out_mv = empty(B_, 2, lv + 1, prm.N)
    ctx.helrm_ptxt_ct_matvec_diag(plan_gpu, to_dev(cts), out_mv, B_)
    out_lk = empty(B_, 2, lv, prm.N)
    say(f"lookup_packed N={prm.N} level={lv} batch={B_}")
    ctx.helrm_lookup_packed(plan_gpu, to_dev(cts), B_, out_lk)
    gmv = to_host(out_mv).reshape(B_, 2, lv + 1, prm.N)
    glk = to_host(out_lk).reshape(B_, 2, lv, prm.N)
    pts = O.plan_residues(prm, w.plan)
    for k, qi in enumerate(batch_idx):
        mv = O.matvec(prm, w.keys, w.plan, w.cts[qi], pts)
        assert_bit_exact(gmv[k], mv, f"matvec query {qi}")
        lk = O.rescale(prm, mv, lv)
        assert_bit_exact(glk[k], lk, f"lookup query {qi}")
        got = W.decrypt_slots(w, glk[k], prm.delta, len(w.expected[qi]))
        assert np.max(np.abs(got - w.expected[qi])) < 1e-4
    return glk


def test_lookup_parity_cfg1(ctx1, w1):
    plan = gpu_plan(ctx1, w1.plan)
    assert plan.rotation_steps() == w1.plan.rotation_steps()
    glk = _check_lookup(ctx1, w1, plan, [0, 1, 2])
    # batch invariance: query 1 alone equals its slot in the batch
    alone = _check_lookup(ctx1, w1, plan, [1])
    assert_bit_exact(alone[0], glk[1], "batch invariance")


@pytest.mark.parametrize("n1,radix,compressed,sign", [(16, 2, True, 1), (2, 8, True, 1), (4, 2, False, 1),
                                                       (1, 4, True, 1), (4, 2, True, -1), (16, 8, False, -1)])
def test_lookup_schedules_cfg1(n1, radix, compressed, sign, p1):
    ctx = context_for(p1)
    w = W.config1(n_queries=1, n1=n1, radix=radix, compressed=compressed, sign=sign)
    load_keys(ctx, w.keys)
    _check_lookup(ctx, w, gpu_plan(ctx, w.plan), [0])


def cfg2_workload(level, n1=16, radix=2, n_queries=1, sign=1):
    prm = O.config2_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 65536, 16, 256, -0.05, 0.05)
    return W.build(prm, [t], level=level, n1=n1, radix=radix, n_queries=n_queries, sign=sign)


@pytest.mark.parametrize("level,n1,radix,sign", [(1, 16, 2, 1), (4, 4, 2, 1), (4, 16, 8, 1), (4, 16, 8, -1),
                                                 (1, 4, 4, -1)])
def test_lookup_parity_cfg2(level, n1, radix, sign, ctx2):
    w = cfg2_workload(level, n1, radix, sign=sign)
    load_keys(ctx2, w.keys)
    _check_lookup(ctx2, w, gpu_plan(ctx2, w.plan), [0])


@pytest.mark.parametrize("radix,sign", [(2, 1), (8, -1)])
def test_lookup_parity_cfg2_full_level(radix, sign, ctx2):
    w = cfg2_workload(23, 16, radix, sign=sign)
    load_keys(ctx2, w.keys)
    _check_lookup(ctx2, w, gpu_plan(ctx2, w.plan), [0])


@pytest.mark.parametrize("fuse", [1, 0])
def test_lookup_fused_boundaries(fuse, p1, ctx2):
    """A ModDown feeding a ModUp or the rescale runs fused with it in
    coefficient form (fuse_ks=1) or in the plain order (fuse_ks=0): both
    bit-exact, with giant steps and fold stages (toy ring n1=2, radix 2), with
    the fold alone (n1=16) and at N=2^16 with giant steps (level 4, sign -1).
    Fused, c1's ModDown also runs inside the ModUp conversions (fuse_conv=1;
    digits of K limbs on the toy ring, one digit of 5 < K limbs at level 4) or
    as a conversion of its own (0)."""
    cases = [(p1, W.config1(n_queries=1, n1=2, radix=2)), (p1, W.config1(n_queries=1, n1=16, radix=4)),
             (None, cfg2_workload(4, 4, 2, sign=-1))]
    for prm, w in cases:
        ctx = ctx2 if prm is None else context_for(prm)
        load_keys(ctx, w.keys)
        plan = gpu_plan(ctx, w.plan)
        try:
            for fc in ((1, 0) if fuse else (1,)):
                say(f"lookup fuse_ks={fuse} fuse_conv={fc} N={w.prm.N} level={w.level} n1={w.plan.n1}")
                ctx.helrm_set_tuning("fuse_ks", fuse)
                ctx.helrm_set_tuning("fuse_conv", fc)
                _check_lookup(ctx, w, plan, [0])
        finally:
            ctx.helrm_set_tuning("fuse_ks", 1)
            ctx.helrm_set_tuning("fuse_conv", 1)


def test_lookup_regenerated_key_halves_cfg2(ctx2):
    """Batch 1 regenerates the keys' a_j halves from their seeds (on the
    40-bit primes, or on every prime); with the knob off the kernels read
    them: all bit-exact against the oracle."""
    w = cfg2_workload(4, 16, 8, sign=-1)
    load_keys(ctx2, w.keys)
    plan = gpu_plan(ctx2, w.plan)
    try:
        for gen in (2, 1, 0):
            say(f"lookup cfg2 level 4 gen_key_a={gen}")
            ctx2.helrm_set_tuning("gen_key_a", gen)
            _check_lookup(ctx2, w, plan, [0])
    finally:
        ctx2.helrm_set_tuning("gen_key_a", 1)


def test_lookup_batched_ragged_cfg2(ctx2):
    """Batch of 5 at level 1 (tiles of 4 plus a ragged tail of 1): every
    ciphertext bit-exact against the oracle and identical to its batch-1 result."""
    w = cfg2_workload(1, 16, 8, n_queries=5)
    load_keys(ctx2, w.keys)
    plan = gpu_plan(ctx2, w.plan)
    glk = _check_lookup(ctx2, w, plan, [0, 1, 2, 3, 4])
    for i in (0, 4):
        alone = _check_lookup(ctx2, w, plan, [i])
        assert_bit_exact(alone[0], glk[i], f"batch invariance query {i}")


@pytest.mark.parametrize("n1", [2, 4, 8])
def test_lookup_shared_baby_kernel_cfg1(n1, p1):
    """Batches of 5 with 8, 4 and 2 giant outputs through the workgroup-shared
    baby-step kernel at every tile width (2, 4, 8 ciphertexts per workgroup:
    ragged tiles and a tile wider than the batch) and through the per-thread
    kernel (share 1): bit-exact against the oracle each time."""
    ctx = context_for(p1)
    w = W.config1(n_queries=5, n1=n1, radix=2, sign=-1)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    for share in (1, 2, 4, 8):
        say(f"baby_share={share} n1={n1}")
        ctx.helrm_set_tuning("baby_share", share)
        _check_lookup(ctx, w, plan, [0, 1, 2, 3, 4])
    ctx.helrm_set_tuning("baby_share", 8)


def test_lookup_multitable_batched_cfg2(ctx2):
    """Four tables of uneven packing (three base-256 compressed, one 100-row
    uncompressed: 64 outputs, m = 64, four giant outputs) at level 1, batch 5,
    rotations by -k: every ciphertext bit-exact and decrypting to its rows."""
    prm = O.config2_params()
    g = synth.rng(0)
    tables = [W.compressed_table(g, 65536, 16, 256, -0.05, 0.05),
              W.uncompressed_table(g, 100, 16, -0.05, 0.05),
              W.compressed_table(g, 300000, 16, 256, -0.05, 0.05),
              W.compressed_table(g, 1000, 16, 256, -0.05, 0.05)]
    w = W.build(prm, tables, level=1, n1=16, radix=8, n_queries=5, sign=-1)
    assert w.plan.m == 64 and w.plan.n2 == 4
    load_keys(ctx2, w.keys)
    plan = gpu_plan(ctx2, w.plan)
    glk = _check_lookup(ctx2, w, plan, [0, 1, 2, 3, 4])
    alone = _check_lookup(ctx2, w, plan, [3])
    assert_bit_exact(alone[0], glk[3], "batch invariance query 3")


def test_lookup_table1_shape_toy(p1):
    """d=768 rows from 32 base-16 digit tables (512 selector slots, m=1024
    diagonals, n1=32) on the toy ring at level 1, batch 2."""
    ctx = context_for(p1)
    w = W.table1_shape(p1, 1, n_queries=2)
    load_keys(ctx, w.keys)
    _check_lookup(ctx, w, gpu_plan(ctx, w.plan), [0, 1])


def test_lookup_table1_shape_n16(ctx2):
    """The same shape at N=2^16, selector at level 1 (the level of the paper's
    comparison with prior work)."""
    w = W.table1_shape(O.config2_params(), 1, n_queries=1)
    load_keys(ctx2, w.keys)
    _check_lookup(ctx2, w, gpu_plan(ctx2, w.plan), [0])


def _check_multi(ctx, w, plans_gpu, batch_idx):
    prm, lv = w.prm, w.level
    n_in = len(w.plans)
    sel = np.stack([np.stack(w.cts[i]) for i in batch_idx])
    B_ = len(batch_idx)
    say(f"lookup_multi N={prm.N} level={lv} n_in={n_in} batch={B_}")
    out = empty(B_, 2, lv, prm.N)
    ctx.helrm_lookup_multi(plans_gpu, to_dev(sel), B_, out)
    got = to_host(out).reshape(B_, 2, lv, prm.N)
    for k, qi in enumerate(batch_idx):
        assert_bit_exact(got[k], O.lookup_multi(prm, w.keys, w.plans, w.cts[qi]), f"multi query {qi}")
        m = O.decrypt(prm, w.keys, got[k])
        rows = O.decode(m, prm.delta, prm)[: len(w.expected[qi])].real
        assert np.max(np.abs(rows - w.expected[qi])) < 1e-4
    return got


def test_lookup_multi_ciphertext_toy(p1):
    """3,000 selector slots on the toy ring (n = 2048): two ciphertexts per
    query, batch 3, every result bit-exact; query 2 alone equals its slot."""
    ctx = context_for(p1)
    g = synth.rng(9)
    tables = [W.uncompressed_table(g, 1000, 16, -1, 1) for _ in range(3)]
    w = W.build_multi(p1, tables, level=2, n1=16, radix=4, n_queries=3)
    load_keys(ctx, w.keys)
    plans = [gpu_plan(ctx, p) for p in w.plans]
    got = _check_multi(ctx, w, plans, [0, 1, 2])
    alone = _check_multi(ctx, w, plans, [2])
    assert_bit_exact(alone[0], got[2], "multi batch invariance")


def test_lookup_multi_ciphertext_n16(ctx2):
    """N=2^16: four 10,000-row uncompressed tables (40,000 slots, two
    ciphertexts), level 1, batch 2."""
    g = synth.rng(10)
    tables = [W.uncompressed_table(g, 10000, 16, -0.05, 0.05) for _ in range(4)]
    w = W.build_multi(O.config2_params(), tables, level=1, n1=16, radix=8, n_queries=2)
    assert len(w.plans) == 2
    load_keys(ctx2, w.keys)
    _check_multi(ctx2, w, [gpu_plan(ctx2, p) for p in w.plans], [0, 1])


@pytest.mark.parametrize("n_ct,rows,batch", [(18, 12288, 2), (85, 58000, 1)])
def test_lookup_multi_ciphertext_paper_scale(n_ct, rows, batch, p1):
    """Selectors as wide as the paper's multi-ciphertext models (18 and 85
    input ciphertexts, Sec. V-D and Table II) on the toy ring: three
    uncompressed tables of `rows` rows each, every column block's products
    summed into the same giant accumulators; bit-exact against the oracle and
    decrypted against the cleartext rows."""
    ctx = context_for(p1)
    g = synth.rng(21)
    tables = [W.uncompressed_table(g, rows, 16, -1, 1) for _ in range(3)]
    w = W.build_multi(p1, tables, level=2, n1=16, radix=4, n_queries=batch)
    assert len(w.plans) == n_ct
    load_keys(ctx, w.keys)
    _check_multi(ctx, w, [gpu_plan(ctx, p) for p in w.plans], list(range(batch)))
    ctx.close()


def test_graph_capture_replays(ctx1, w1):
    """The batched lookup captured in a HIP graph: every replay (with eager
    work and synchronisation between replays) equals the eager result."""
    import torch
    plan = gpu_plan(ctx1, w1.plan)
    B_ = 3
    cts = to_dev(np.stack(w1.cts[:B_]))
    eager = empty(B_, 2, w1.level, w1.prm.N)
    ctx1.helrm_lookup_packed(plan, cts, B_, eager)
    want = to_host(eager)
    s = torch.cuda.Stream()
    out = empty(B_, 2, w1.level, w1.prm.N)
    ctx1.helrm_reserve(plan, B_, s)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx1.helrm_lookup_packed(plan, cts, B_, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("graph capture of lookup_packed batch=3")
    with torch.cuda.graph(g, stream=s):
        ctx1.helrm_lookup_packed(plan, cts, B_, out)
    for rep in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert_bit_exact(to_host(out), want, f"graph replay {rep}")
        ctx1.helrm_lookup_packed(plan, cts, B_, eager)   # eager work between replays
        torch.cuda.synchronize()


def test_batch_graph_abi_replays(ctx1, w1):
    """helrm_batch_graph_create / _replay / _destroy: the batched lookup
    recorded once and replayed four times, with new selectors written into
    the bound input and eager work in between; every replay bit-exact against
    the oracle (and the eager call)."""
    import torch
    plan = gpu_plan(ctx1, w1.plan)
    B_ = 3
    order = [[0, 1, 2], [2, 0, 1], [1, 1, 0], [0, 1, 2]]
    sel = to_dev(np.stack(w1.cts[:B_]))
    out = empty(B_, 2, w1.level, w1.prm.N)
    say("batch graph create (C ABI), batch 3")
    g = ctx1.helrm_batch_graph_create([plan], sel, B_, out)
    want = {i: O.lookup(w1.prm, w1.keys, w1.plan, w1.cts[i]) for i in range(3)}
    eager = empty(B_, 2, w1.level, w1.prm.N)
    s = torch.cuda.Stream()
    for rep, idx in enumerate(order):
        sel.copy_(to_dev(np.stack([w1.cts[i] for i in idx])))
        out.zero_()
        g.replay(s if rep % 2 else None)
        torch.cuda.synchronize()
        got = to_host(out).reshape(B_, 2, w1.level, w1.prm.N)
        for k, i in enumerate(idx):
            assert_bit_exact(got[k], want[i], f"replay {rep} slot {k}")
        ctx1.helrm_lookup_packed(plan, sel, B_, eager)   # eager work between replays
        torch.cuda.synchronize()
        assert_bit_exact(to_host(eager).reshape(got.shape), got, f"eager after replay {rep}")
    g.close()


def test_batch_graph_abi_multi_ciphertext(p1):
    """The graph of a multi-ciphertext lookup (two selector ciphertexts per
    query, batch 2) replays bit-exact against the oracle."""
    import torch
    ctx = context_for(p1)
    g9 = synth.rng(9)
    tables = [W.uncompressed_table(g9, 1000, 16, -1, 1) for _ in range(3)]
    w = W.build_multi(p1, tables, level=2, n1=16, radix=4, n_queries=2)
    load_keys(ctx, w.keys)
    plans = [gpu_plan(ctx, p) for p in w.plans]
    sel = to_dev(np.stack([np.stack(c) for c in w.cts]))
    out = empty(2, 2, w.level, p1.N)
    assert ctx.helrm_footprint_multi(plans, 2) >= ctx.helrm_footprint(plans[0], 2)
    g = ctx.helrm_batch_graph_create(plans, sel, 2, out)
    for rep in range(2):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = to_host(out).reshape(2, 2, w.level, p1.N)
        for k in range(2):
            assert_bit_exact(got[k], O.lookup_multi(p1, w.keys, w.plans, w.cts[k]), f"multi replay {rep} q{k}")
    g.close()


def test_capture_guard_and_outgrown_workspace(ctx1, w1):
    """A lookup captured (torch graph) on a stream whose workspace was not
    reserved for it fails with HELRM_ESTATE instead of allocating; a graph
    captured on a reserved workspace still replays bit-exact after an eager
    call on the same stream outgrew that workspace (the old one is kept)."""
    import torch
    from paper_2506_18150_amd import binding as B
    plan = gpu_plan(ctx1, w1.plan)
    cts = to_dev(np.stack(w1.cts[:3]))
    want = [O.lookup(w1.prm, w1.keys, w1.plan, w1.cts[i]) for i in range(3)]
    s = torch.cuda.Stream()
    out = empty(1, 2, w1.level, w1.prm.N)
    say("capture without reserve -> HELRM_ESTATE")
    g0 = torch.cuda.CUDAGraph()
    with pytest.raises(B.HelrmError) as ei:
        with torch.cuda.graph(g0, stream=s):
            out.zero_()
            ctx1.helrm_lookup_packed(plan, cts[:1].contiguous(), 1, out, s)
    assert ei.value.code == -4
    torch.cuda.synchronize()
    say("capture on a reserved workspace, then outgrow it eagerly")
    s2 = torch.cuda.Stream()
    ctx1.helrm_reserve(plan, 1, s2)
    one = cts[:1].contiguous()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s2):
        ctx1.helrm_lookup_packed(plan, one, 1, out, s2)
    big = empty(3, 2, w1.level, w1.prm.N)
    with torch.cuda.stream(s2):
        ctx1.helrm_lookup_packed(plan, cts, 3, big, s2)   # needs a larger workspace on s2
    torch.cuda.synchronize()
    for k in range(3):
        assert_bit_exact(to_host(big)[k], want[k], f"eager batch 3 query {k}")
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert_bit_exact(to_host(out)[0], want[0], f"replay {rep} after the workspace grew")
