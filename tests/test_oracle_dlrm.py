"""Pins for the ciphertext product, relinearisation and the small-DLRM forward
pass on the oracle (Appendix A "Multiplication", Sec. II-B, Sec. V-C): the
tensor product against a big-integer negacyclic product of the two phases,
relinearisation against the phase of the tensor within the key-switching
noise and against the add-after-ModDown order, the square activation by
decryption, the layer layout against the fp64 model, and the encrypted
forward pass against the fp64 logit."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import workloads as W


def _phase(prm, keys, parts, level):
    """CRT value of sum_i parts[i] s^i over Q_level, centred (Python ints)."""
    Q = prm.Q(level)
    s = keys.s[: level + 1]
    acc = parts[0].copy()
    sp = s.copy()
    for c in parts[1:]:
        acc = O.add(acc, O.mul(c, sp, Q), Q)
        sp = O.mul(sp, s, Q)
    return O.crt_centered(O.intt(acc, Q, prm), Q)


def _negacyclic(a, b, N):
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += a[i] * b[j]
            else:
                out[k - N] -= a[i] * b[j]
    return out


def test_tensor_is_product_of_phases():
    """(a0 + a1 s)(b0 + b1 s) = d0 + d1 s + d2 s^2 in Z_Q[X]/(X^N+1)."""
    prm = O.make_params(N=16, L=3, K=2, alpha=2)
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, [], relin=True))
    rng = np.random.default_rng(3)
    for level in (prm.L, 1):
        Q = prm.Q(level)
        Qv = 1
        for q in Q:
            Qv *= q
        a = np.stack([np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in Q]) for _ in range(2)])
        b = np.stack([np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in Q]) for _ in range(2)])
        d = O.tensor(prm, a, b, level)
        A = _phase(prm, keys, list(a), level)
        B = _phase(prm, keys, list(b), level)
        D = _phase(prm, keys, list(d), level)
        want = _negacyclic(A, B, prm.N)
        assert all((x - y) % Qv == 0 for x, y in zip(D, want))


@pytest.fixture(scope="module")
def relin_keys():
    prm = O.config1_params()
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, [], relin=True))
    return prm, keys


def test_relinearize_noise_and_order(relin_keys):
    prm, keys = relin_keys
    g = synth.rng(21)
    z = g.uniform(-1, 1, prm.n)
    w = g.uniform(-1, 1, prm.n)
    for level in (prm.L, 2):
        a = O.encrypt(prm, keys, O.encode(z, prm.delta, prm), level, synth.enc_draws(g, prm.N))
        b = O.encrypt(prm, keys, O.encode(w, prm.delta, prm), level, synth.enc_draws(g, prm.N))
        d = O.tensor(prm, a, b, level)
        r = O.relinearize(prm, keys, d, level)
        # adding (d0, d1) after the ModDown gives the same residues
        zero = np.zeros((level + 1, prm.N), dtype=np.uint64)
        ks = O.moddown(prm, O.key_inner_product(prm, O.modup(prm, d[2], level), zero, level, keys.relin, 1),
                       level)
        Q = prm.Q(level)
        assert np.array_equal(r, np.stack([O.add(d[0], ks[0], Q), O.add(d[1], ks[1], Q)]))
        # phase of the result = phase of the tensor + key-switching noise:
        # sum_j digit_j e_j / P over dnum digits plus the ModDown floor times s
        got = _phase(prm, keys, list(r), level)
        want = _phase(prm, keys, list(d), level)
        bound = prm.dnum * prm.N * 19 * 2 + prm.N * (prm.K + 2)
        assert max(abs(x - y) for x, y in zip(got, want)) < bound
        assert max(abs(x) for x in want) > 2 ** 60   # the product itself is far above the noise


def test_square_rescale_decodes(relin_keys):
    prm, keys = relin_keys
    g = synth.rng(22)
    z = g.uniform(-1, 1, prm.n)
    level = prm.L
    ct = O.encrypt(prm, keys, O.encode(z, prm.delta, prm), level, synth.enc_draws(g, prm.N))
    sq = O.rescale(prm, O.mul_relin(prm, keys, ct, ct, level), level)
    scale = float(prm.delta) ** 2 / prm.q[level]
    got = O.decode(O.decrypt(prm, keys, sq), scale, prm).real
    assert np.max(np.abs(got - z * z)) < 1e-6


def test_add_plain_and_mod_drop(relin_keys):
    prm, keys = relin_keys
    g = synth.rng(23)
    z = g.uniform(-1, 1, prm.n)
    b = g.uniform(-1, 1, prm.n)
    level = prm.L
    ct = O.encrypt(prm, keys, O.encode(z, prm.delta, prm), level, synth.enc_draws(g, prm.N))
    out = O.add_plain(prm, ct, O.plain_residues(prm, b, prm.delta, level), level)
    dropped = O.mod_drop(out, 1)
    assert dropped.shape == (2, 2, prm.N)
    for c, lv in ((out, level), (dropped, 1)):
        got = O.decode(O.decrypt(prm, keys, c), prm.delta, prm).real
        assert np.max(np.abs(got - (z + b))) < 1e-6


def test_dlrm_layout_matches_model():
    """The slot layout (embedding rows then bottom output, one matrix per layer)
    reproduces the fp64 model, both directly and through the BSGS schedule."""
    model = W.small_dlrm(0)
    lay = O.dlrm_layout(model)
    n = 2048
    rng = np.random.default_rng(4)
    for _ in range(3):
        dense = synth.dense_features(rng, model.n_dense)
        idx = synth.indices(rng, [t.rows for t in model.tables])
        x = model.input_slots(dense, idx)
        h = x[: model.n_dense]
        for k, (M, b) in enumerate(zip(lay.bottom, lay.bias_bottom)):
            h = (M @ h + b) ** 2
        z = lay.emb @ x + h
        assert np.allclose(z[: model.emb_dim], np.concatenate([t.lookup(i) for t, i in zip(model.tables, idx)]))
        for k, (M, b) in enumerate(zip(lay.top, lay.bias_top)):
            z = M @ z + b
            if k + 1 < len(lay.top):
                z = z ** 2
        assert np.allclose(z, O.dlrm_cleartext(model, dense, idx), atol=1e-12)
        # the schedule replay of the embedding product is exact on the rows it
        # writes and zero on the bottom-output rows
        xs = np.zeros(n)
        xs[: len(x)] = x
        ze = O.cleartext_bsgs(lay.emb, xs, n, 16, 8, -1)
        assert np.allclose(ze[: lay.emb.shape[0]], lay.emb @ x, atol=1e-12)
        assert np.allclose(ze[model.emb_dim: O.next_pow2(lay.emb.shape[0])], 0, atol=1e-12)


@pytest.fixture(scope="module")
def toy_dlrm():
    prm = W.dlrm_params_toy()
    model = W.small_dlrm(0)
    sch = O.dlrm_schedule(prm, model, level0=prm.L, n1=16, radix=8, sign=-1)
    gals = [O.galois_for_step(k, prm) for k in sch.rotation_steps()]
    keys = O.keygen(prm, synth.key_draws(0, prm.N, prm.q, prm.p, prm.dnum, gals, relin=True))
    return prm, model, sch, keys


def test_dlrm_schedule_levels(toy_dlrm):
    prm, model, sch, _ = toy_dlrm
    # bottom: 2 x (matvec + square), top: matvec + square + matvec -> 7 levels
    assert [p.level for p in sch.bottom] == [8, 6]
    assert [p.level for p in sch.top] == [4, 2]
    assert sch.emb.level == 8 and sch.concat_level == 4 and sch.out_level == 1
    assert sch.emb.m == 256 and sch.bottom[1].m == 256


def test_dlrm_encrypted_forward_matches_fp64(toy_dlrm):
    prm, model, sch, keys = toy_dlrm
    g = synth.rng(31)
    for _ in range(2):
        dense = synth.dense_features(g, model.n_dense)
        idx = synth.indices(g, [t.rows for t in model.tables])
        ct = O.encrypt(prm, keys, O.encode(model.input_slots(dense, idx), prm.delta, prm), sch.level0,
                       synth.enc_draws(g, prm.N))
        out = O.dlrm_forward(prm, keys, sch, ct)
        assert out.shape == (2, sch.out_level + 1, prm.N)
        got = O.decode(O.decrypt(prm, keys, out), prm.delta, prm).real[0]
        want = O.dlrm_cleartext(model, dense, idx)[0]
        assert abs(got - want) < 1e-4
