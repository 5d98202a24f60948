"""Host-side pieces of the product (parameter rule, encoding, planner,
selector) against the oracle's independent implementations and against the
paper's worked example -- CPU only."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from paper_2506_18150_amd import encoding, params, planner


def test_param_sets_match_oracle_rule():
    for mine, theirs in ((params.toy(), O.config1_params()), (params.n16(), O.config2_params())):
        assert mine.q == theirs.q and mine.p == theirs.p
        assert (mine.N, mine.L, mine.K, mine.alpha, mine.dnum) == (theirs.N, theirs.L, theirs.K, theirs.alpha,
                                                                  theirs.dnum)


@pytest.mark.parametrize("N", [64, 4096])
def test_encoding_matches_oracle(N):
    prm = O.make_params(N=N, L=1, K=1, alpha=1)
    rng = np.random.default_rng(N)
    for scale in (2.0 ** 40, float(prm.q[1])):
        z = rng.uniform(-1, 1, N // 2)
        mine = encoding.encode(z, scale, N)
        theirs = O.encode(z, scale, prm)
        # two different FFT routes: rounding may differ only at exact .5 ties
        assert np.max(np.abs(mine - theirs)) <= 1
        assert np.mean(mine != theirs) < 1e-3
        back = encoding.decode(mine, scale, N)
        assert np.max(np.abs(back.real - z)) < 1e-9


def test_digits_worked_example():
    assert planner.n_digits(16, 4) == 2 and planner.digits(14, 4, 2) == [2, 3]
    assert planner.n_digits(65536, 256) == 2 and planner.n_digits(65537, 256) == 3
    assert planner.n_digits(1, 256) == 1


def test_plan_matches_oracle_diagonals():
    rng = synth.rng(3)
    M = rng.uniform(-1, 1, (24, 300))
    for n1, sign in ((4, 1), (16, 1), (4, -1), (16, -1)):
        m, n2, vals = planner.bsgs_diagonals(M, 512, n1, sign)
        om, on2, ovals = O.bsgs_plan_values(M, 512, n1, sign)
        assert (m, n2) == (om, on2)
        assert sorted(vals) == sorted(g * n1 + b for (g, b) in ovals)
        for (g, b), v in ovals.items():
            assert np.array_equal(vals[g * n1 + b], v)
    assert planner.fold_stages(32768, 16, 8) == O.fold_stages(32768, 16, 8)
    for sign in (1, -1):
        assert planner.fold_span(24, 300, 512, sign) == O.fold_span(M, 512, sign)


def test_selector_and_rows_match_oracle():
    g = synth.rng(5)
    parts = [synth.uniform_table(g, 16, 4, -1, 1) for _ in range(3)]
    E = synth.uniform_table(g, 7, 4, -1, 1)
    mine = [planner.Table(rows=4000, d=4, base=16, parts=parts), planner.Table(rows=7, d=4, full=E)]
    theirs = [O.TableSpec(rows=4000, d=4, base=16, C=parts), O.TableSpec(rows=7, d=4, E=E)]
    assert np.array_equal(planner.packed_matrix(mine), O.pack_tables(theirs))
    for idx in ([0, 0], [3999, 6], [1234, 3]):
        assert np.array_equal(planner.packed_selector(mine, idx), O.pack_selector(theirs, idx))
        assert np.allclose(np.concatenate([t.row(i) for t, i in zip(mine, idx)]),
                           np.concatenate([t.lookup(i) for t, i in zip(theirs, idx)]))


def test_plan_spec_rotation_steps():
    M = np.ones((16, 512))
    spec = planner.make_plan(M, 1 << 16, 23, 2.0 ** 40, 16, 2, sign=1)
    assert spec.m == 16 and spec.n2 == 1 and len(spec.stages) == 11
    assert len(spec.rotation_steps()) == 26
    spec = planner.make_plan(M, 1 << 16, 23, 2.0 ** 40, 16, 8, sign=-1)
    assert spec.span == 1024 and spec.stages == [(128, 8), (16, 8)]
    assert spec.rotation_steps()[:15] == list(range(-15, 0))
    assert len(spec.rotation_steps()) == 15 + 14
    assert planner.compress_rule(501, 500) and not planner.compress_rule(500, 500)


def test_dlrm_layout_matches_oracle():
    """The product's slot layout of the small DLRM equals the oracle's."""
    from paper_2506_18150_amd import dlrm
    d = synth.small_dlrm_draws(0)
    w = dlrm.DLRMWeights(tables=d.tables, bottom=list(d.bottom), top=list(d.top), n_dense=d.n_dense)
    model = O.SmallDLRM(tables=[O.TableSpec(rows=r, d=t.shape[1], E=t) for r, t in zip(d.table_rows, d.tables)],
                        bottom=list(d.bottom), top=list(d.top), n_dense=d.n_dense)
    emb, bottom, bb, top, bt = dlrm.layer_matrices(w)
    lay = O.dlrm_layout(model)
    assert np.array_equal(emb, lay.emb)
    for a, b in zip(bottom + bb + top + bt, lay.bottom + lay.bias_bottom + lay.top + lay.bias_top):
        assert np.array_equal(a, b)
    g = synth.rng(2)
    dense = synth.dense_features(g, d.n_dense)
    idx = synth.indices(g, d.table_rows)
    assert np.array_equal(w.input_slots(dense, idx), model.input_slots(dense, idx))
    assert np.allclose(w.cleartext(dense, idx), O.dlrm_cleartext(model, dense, idx), atol=1e-14)


def test_multi_plan_matches_oracle():
    """Column blocks of a selector wider than one ciphertext: the product's
    per-block plans and shared fold equal the oracle's."""
    prm = O.config1_params()
    g = synth.rng(9)
    E = [synth.uniform_table(g, 1000, 16, -1, 1) for _ in range(3)]
    mine = planner.packed_matrix([planner.Table(rows=1000, d=16, full=e) for e in E])
    theirs = O.pack_tables([O.TableSpec(rows=1000, d=16, E=e) for e in E])
    assert np.array_equal(mine, theirs)
    specs = planner.make_multi_plan(mine, prm.N, 2, float(prm.q[2]), 16, 4, -1)
    plans = O.make_multi_plan(prm, theirs, 2, 16, 4, -1)
    assert len(specs) == len(plans) == 2
    for sp, p in zip(specs, plans):
        assert (sp.m, sp.n1, sp.n2, sp.span, sp.stages) == (p.m, p.n1, p.n2, p.span, p.stages)
        assert sp.diag == sorted(gg * p.n1 + b for (gg, b) in p.coeffs)
        assert sp.rotation_steps() == p.rotation_steps()


def test_plan_device_bytes():
    """Plan memory as the request loop counts it: 13 bytes per stored word
    over PQ_level, plus the matrix-core operands (4 KiB per limb, coefficient
    and giant tile of 8) only for plans with several giant steps and at least
    33 distinct baby steps among their stored diagonals."""
    from types import SimpleNamespace

    from paper_2506_18150_amd.session import plan_device_bytes
    prm = params.n16()
    pqn = 24 + prm.K
    word = pqn * prm.N
    w2 = SimpleNamespace(diag=list(range(16)), n1=16, n2=1)
    assert plan_device_bytes(prm, 23, w2) == 16 * word * 13
    w3 = SimpleNamespace(diag=list(range(512)), n1=64, n2=8)
    assert plan_device_bytes(prm, 23, w3) == 512 * word * 13 + word * 4096
    group = SimpleNamespace(diag=list(range(64)), n1=16, n2=4)
    assert plan_device_bytes(prm, 23, group) == 64 * word * 13
    wide = SimpleNamespace(diag=[g * 40 + b for g in range(9) for b in range(33)], n1=40, n2=9)
    assert plan_device_bytes(prm, 23, wide) == 9 * 33 * word * 13 + 2 * word * 4096
    few = SimpleNamespace(diag=[g * 40 + b for g in range(9) for b in range(32)], n1=40, n2=9)
    assert plan_device_bytes(prm, 23, few) == 9 * 32 * word * 13
    assert plan_device_bytes(prm, 4, w2) == 16 * (5 + prm.K) * prm.N * 13
