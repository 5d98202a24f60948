"""Pins for the oracle's CKKS layer (Appendix A): encoding against its defining
sum and the ring-homomorphism property, encryption/decryption noise, rotation
direction, hoisted key switching and rescale by decrypting."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


@pytest.fixture(scope="module")
def prm1():
    return O.config1_params()


def test_encode_matches_defining_sum():
    prm = O.make_params(N=64, L=1, K=1, alpha=1)
    rng = np.random.default_rng(1)
    z = rng.uniform(-1, 1, prm.n) + 1j * rng.uniform(-1, 1, prm.n)
    assert np.array_equal(O.encode(z, 2.0 ** 30, prm), O.encode_direct(z, 2.0 ** 30, prm))


def test_encode_constant_is_constant_polynomial(prm1):
    for c in (0.5, -0.3125, 1.0):
        m = O.encode(np.full(prm1.n, c), prm1.delta, prm1)
        assert m[0] == round(c * prm1.delta)
        assert not np.any(m[1:])


def test_encode_decode_roundtrip(prm1):
    rng = np.random.default_rng(2)
    z = rng.uniform(-1, 1, prm1.n)
    back = O.decode(O.encode(z, prm1.delta, prm1), prm1.delta, prm1)
    assert np.max(np.abs(back - z)) < 2.0 ** -28
    assert np.max(np.abs(back.imag)) < 2.0 ** -28


def test_canonical_embedding_is_ring_homomorphism():
    """decode(a * b mod X^N+1) = decode(a) (.) decode(b): pins the slot roots,
    and X -> X^5 rotates slots left by one: pins the rotation direction."""
    prm = O.make_params(N=32, L=1, K=1, alpha=1)
    rng = np.random.default_rng(3)
    a = rng.integers(-50, 50, prm.N)
    b = rng.integers(-50, 50, prm.N)
    prod = np.zeros(prm.N, dtype=np.int64)
    for i in range(prm.N):
        for j in range(prm.N):
            if i + j < prm.N:
                prod[i + j] += a[i] * b[j]
            else:
                prod[i + j - prm.N] -= a[i] * b[j]
    za, zb, zp = (O.decode(v, 1.0, prm) for v in (a, b, prod))
    assert np.allclose(zp, za * zb, atol=1e-6)
    for k in (1, 3):
        g = O.galois_for_step(k, prm)
        rotated = np.zeros(prm.N, dtype=np.int64)
        for c in range(prm.N):
            e = c * g % (2 * prm.N)
            if e < prm.N:
                rotated[e] += a[c]
            else:
                rotated[e - prm.N] -= a[c]
        assert np.allclose(O.decode(rotated, 1.0, prm), np.roll(za, -k), atol=1e-6)


@pytest.fixture(scope="module")
def keyed(prm1):
    steps = [1, 2, 5, 100, 1024]
    gals = [O.galois_for_step(k, prm1) for k in steps]
    draws = synth.key_draws(0, prm1.N, prm1.q, prm1.p, prm1.dnum, gals, relin=True)
    return O.keygen(prm1, draws), steps, draws


def test_public_key_relation(prm1, keyed):
    keys, _, draws = keyed
    # b + a s = e on every Q limb
    Q = prm1.q
    e = O.add(keys.pk[0], O.mul(keys.pk[1], keys.s[: prm1.L + 1], Q), Q)
    ec = O.intt(e, Q, prm1)
    for li, q in enumerate(Q):
        got = np.array([int(x) - q if int(x) > q // 2 else int(x) for x in ec[li]])
        assert np.array_equal(got, draws.pk_e)


def test_encrypt_decrypt_noise(prm1, keyed):
    keys, _, _ = keyed
    g = synth.rng(5)
    z = g.uniform(-1, 1, prm1.n)
    m = O.encode(z, prm1.delta, prm1)
    for level in (prm1.L, 1):
        ct = O.encrypt(prm1, keys, m, level, synth.enc_draws(g, prm1.N))
        got = O.decrypt(prm1, keys, ct)
        # noise v e + e0 + e1 s is bounded by N * 19 * 2 + 19
        assert np.max(np.abs(got - m)) < 2 * 19 * prm1.N + 19
        assert np.max(np.abs(O.decode(got, prm1.delta, prm1).real - z)) < 1e-6


def test_rotation_and_hoisting_decrypt(prm1, keyed):
    keys, steps, _ = keyed
    g = synth.rng(6)
    z = g.uniform(-1, 1, prm1.n)
    m = O.encode(z, prm1.delta, prm1)
    level = prm1.L
    ct = O.encrypt(prm1, keys, m, level, synth.enc_draws(g, prm1.N))
    hoisted = O.hoisted_rotations(prm1, keys, ct, level, steps)
    for k, R in zip(steps, hoisted):
        full = O.rotate(prm1, keys, ct, k, level)
        assert np.array_equal(O.moddown(prm1, R, level), full)
        got = O.decode(O.decrypt(prm1, keys, full), prm1.delta, prm1).real
        assert np.max(np.abs(got - np.roll(z, -k))) < 1e-6
    # at a lower level the full-level keys still work
    ct1 = O.encrypt(prm1, keys, m, 1, synth.enc_draws(g, prm1.N))
    got = O.decode(O.decrypt(prm1, keys, O.rotate(prm1, keys, ct1, 5, 1)), prm1.delta, prm1).real
    assert np.max(np.abs(got - np.roll(z, -5))) < 1e-6


def test_plaintext_mult_rescale(prm1, keyed):
    keys, _, _ = keyed
    g = synth.rng(7)
    z = g.uniform(-1, 1, prm1.n)
    w = g.uniform(-1, 1, prm1.n)
    level = prm1.L
    Q = prm1.Q(level)
    ct = O.encrypt(prm1, keys, O.encode(z, prm1.delta, prm1), level, synth.enc_draws(g, prm1.N))
    pt = O.ntt(O.from_signed(O.encode(w, prm1.q[level], prm1), Q), Q, prm1)
    prod = np.stack([O.mul(ct[c], pt, Q) for c in range(2)])
    out = O.rescale(prm1, prod, level)
    got = O.decode(O.decrypt(prm1, keys, out), prm1.delta, prm1).real
    assert np.max(np.abs(got - z * w)) < 1e-6
