"""GPU parity for the small-DLRM pieces (Appendix A "Multiplication",
"Addition"; Sec. II-B, Sec. V-C): ciphertext product with relinearisation,
plaintext addition and level drop against the oracle, bit-exact on every
residue, and the whole encrypted forward pass (oracle-built plans and biases
driven through the product's pipeline) bit-exact against the oracle's pass and
within 1e-4 of the fp64 model after decryption."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def load_all_keys(ctx, keys):
    import torch
    from paper_2506_18150_amd import binding as B
    load_keys(ctx, keys)
    ctx.helrm_load_eval_keys([0], B.device_u64(keys.relin), [keys.seeds[0]])
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def cfg1():
    prm = O.config1_params()
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, [], relin=True))
    ctx = context_for(prm)
    load_all_keys(ctx, keys)
    return prm, keys, ctx


def _cts(prm, keys, level, n, seed):
    g = synth.rng(seed)
    return np.stack([O.encrypt(prm, keys, O.encode(g.uniform(-1, 1, prm.n), prm.delta, prm), level,
                               synth.enc_draws(g, prm.N)) for _ in range(n)])


@pytest.mark.parametrize("level", [3, 1, 0])
def test_mul_relin_parity(cfg1, level):
    prm, keys, ctx = cfg1
    a = _cts(prm, keys, level, 3, 40 + level)
    b = _cts(prm, keys, level, 3, 50 + level)
    say(f"mul_relin N={prm.N} level={level} batch=3")
    out = empty(3, 2, level + 1, prm.N)
    ctx.helrm_mul_relin(to_dev(a), to_dev(b), level, out, 3)
    sq = empty(3, 2, level + 1, prm.N)
    da = to_dev(a)
    ctx.helrm_mul_relin(da, da, level, sq, 3)
    got, gsq = to_host(out), to_host(sq)
    for k in range(3):
        assert_bit_exact(got[k], O.mul_relin(prm, keys, a[k], b[k], level), f"mul_relin {k}")
        assert_bit_exact(gsq[k], O.mul_relin(prm, keys, a[k], a[k], level), f"square {k}")
    # out aliasing an input
    ctx.helrm_mul_relin(da, da, level, da, 3)
    assert_bit_exact(to_host(da), gsq, "square in place")


def test_add_plain_and_mod_drop_parity(cfg1):
    prm, keys, ctx = cfg1
    level = 3
    a = _cts(prm, keys, level, 2, 60)
    pt = O.plain_residues(prm, synth.rng(61).uniform(-1, 1, prm.n), prm.delta, level)
    out = empty(2, 2, level + 1, prm.N)
    ctx.helrm_add_plain(to_dev(a), to_dev(pt), level, out, 2)
    got = to_host(out)
    for k in range(2):
        assert_bit_exact(got[k], O.add_plain(prm, a[k], pt, level), f"add_plain {k}")
    for lo in (2, 0):
        dropped = empty(2, 2, lo + 1, prm.N)
        ctx.helrm_mod_drop(out, level, dropped, lo, 2)
        gd = to_host(dropped)
        for k in range(2):
            assert_bit_exact(gd[k], O.mod_drop(got[k], lo), f"mod_drop {k} to {lo}")


def gpu_schedule(ctx, sch):
    from paper_2506_18150_amd import dlrm
    return dlrm.Schedule(level0=sch.level0, emb=gpu_plan(ctx, sch.emb), bottom=[gpu_plan(ctx, p) for p in sch.bottom],
                         bias_bottom=[to_dev(b) for b in sch.bias_bottom], top=[gpu_plan(ctx, p) for p in sch.top],
                         bias_top=[to_dev(b) for b in sch.bias_top], concat_level=sch.concat_level,
                         out_level=sch.out_level)


def _dlrm_case(prm, level0, n_queries, seed, check_oracle):
    from paper_2506_18150_amd import dlrm
    model = W.small_dlrm(0)
    sch = O.dlrm_schedule(prm, model, level0=level0, n1=16, radix=8, sign=-1)
    gals = [O.galois_for_step(k, prm) for k in sch.rotation_steps()]
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals, relin=True))
    ctx = context_for(prm)
    load_all_keys(ctx, keys)
    g = synth.rng(seed)
    cts, want = [], []
    for _ in range(n_queries):
        dense = synth.dense_features(g, model.n_dense)
        idx = synth.indices(g, [t.rows for t in model.tables])
        cts.append(O.encrypt(prm, keys, O.encode(model.input_slots(dense, idx), prm.delta, prm), level0,
                             synth.enc_draws(g, prm.N)))
        want.append(O.dlrm_cleartext(model, dense, idx)[0])
    gs = gpu_schedule(ctx, sch)
    say(f"dlrm forward N={prm.N} level0={level0} batch={n_queries}")
    out = dlrm.forward(ctx, gs, to_dev(np.stack(cts)), n_queries)
    got = to_host(out)
    assert got.shape == (n_queries, 2, sch.out_level + 1, prm.N)
    for k in check_oracle:
        assert_bit_exact(got[k], O.dlrm_forward(prm, keys, sch, cts[k]), f"dlrm query {k}")
    for k in range(n_queries):
        logit = O.decode(O.decrypt(prm, keys, got[k]), prm.delta, prm).real[0]
        assert abs(logit - want[k]) < 1e-4


def test_dlrm_forward_toy_ring():
    """N=2^12, 8 levels, batch 3: every query bit-exact against the oracle."""
    _dlrm_case(W.dlrm_params_toy(), 8, 3, 70, check_oracle=[0, 1, 2])


def test_dlrm_forward_n16():
    """N=2^16 with the 24-prime chain, input at level 8, batch 4: every query
    bit-exact against the oracle, every logit within 1e-4 of fp64."""
    _dlrm_case(O.config2_params(), 8, 4, 71, check_oracle=[0, 1, 2, 3])
