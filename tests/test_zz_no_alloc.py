"""helrm_lookup_packed_noalloc (the lookup for callers that cannot allocate,
its workspace a static device array) against helrm_lookup_packed on the same
inputs, bit-exact on every residue, on two calls in a row, the second with a
smaller input; and its refusal of a lookup whose workspace exceeds the array.
Encrypted packed lookup: Sec. IV-B."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W
from tests.gpu_helpers import assert_bit_exact, context_for, empty, gpu_plan, load_keys, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _both(ctx, plan, cts, level, N):
    """The no-allocation call and the plain call on the same selectors."""
    B = len(cts)
    sel = to_dev(np.stack(cts))
    out_na = empty(B, 2, level, N)
    out = empty(B, 2, level, N)
    ctx.helrm_lookup_packed_noalloc(plan, sel, B, out_na)
    ctx.helrm_lookup_packed(plan, sel, B, out)
    return (to_host(out_na).reshape(B, 2, level, N), to_host(out).reshape(B, 2, level, N))


@pytest.mark.timeout(300)
def test_noalloc_matches_lookup_toy_ring():
    """Toy ring N=2^12 (level 3, n1=4, radix 2): batch 3, then batch 1; the
    first result also against the oracle."""
    w = W.config1(n_queries=3)
    ctx = context_for(w.prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    for batch in (3, 1):
        say(f"noalloc toy ring batch={batch}")
        got, want = _both(ctx, plan, w.cts[:batch], w.level, w.prm.N)
        assert_bit_exact(got, want, f"noalloc vs lookup_packed, batch {batch}")
    assert_bit_exact(got[0], O.lookup(w.prm, w.keys, w.plan, w.cts[0]), "noalloc vs oracle")
    ctx.close()


@pytest.mark.timeout(300)
def test_noalloc_matches_lookup_n16():
    """N=2^16, one 65,536-row table, selector at level 4 with the headline
    schedule (n1=16, fold radix 8, sign -1: baby steps and fold stages):
    batch 2, then batch 1."""
    prm = O.config2_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 65536, 16, 256, -0.05, 0.05)
    w = W.build(prm, [t], level=4, n1=16, radix=8, n_queries=2, sign=-1)
    ctx = context_for(prm)
    load_keys(ctx, w.keys)
    plan = gpu_plan(ctx, w.plan)
    from paper_2506_18150_amd import binding as B
    for batch in (2, 1):
        need = ctx.helrm_footprint(plan, batch)
        assert need <= B.HELRM_NOALLOC_MAX_BYTES, need
        say(f"noalloc N=2^16 level 4 batch={batch} scratch={need}")
        got, want = _both(ctx, plan, w.cts[:batch], 4, prm.N)
        assert_bit_exact(got, want, f"noalloc vs lookup_packed, batch {batch}")
        rows = W.decrypt_slots(w, got[0], prm.delta, 16)
        assert np.max(np.abs(rows - w.expected[0])) < 1e-4
    ctx.close()


@pytest.mark.timeout(300)
def test_noalloc_refuses_oversized_lookup():
    """A level-23 lookup at N=2^16 needs more workspace than the static array
    holds: the call fails on the host with HELRM_EINVAL (nothing launched)."""
    from paper_2506_18150_amd import binding as B
    prm = O.config2_params()
    g = synth.rng(0)
    t = W.compressed_table(g, 65536, 16, 256, -0.05, 0.05)
    M = O.pack_tables([t])
    plan_o = O.make_plan(prm, M, 23, 16, 8, -1)
    ctx = context_for(prm)
    plan = gpu_plan(ctx, plan_o)
    assert ctx.helrm_footprint(plan, 1) > B.HELRM_NOALLOC_MAX_BYTES
    sel = empty(1, 2, 24, prm.N)
    out = empty(1, 2, 23, prm.N)
    say("noalloc oversized lookup (host-side refusal)")
    with pytest.raises(B.HelrmError) as e:
        ctx.helrm_lookup_packed_noalloc(plan, sel, 1, out)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    ctx.close()
