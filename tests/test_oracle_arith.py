"""Pins for the oracle's modular arithmetic against facts outside the oracle:
sympy primality, the evaluation definition of the NTT, the schoolbook
negacyclic product, polynomial evaluation, and big-integer closed forms for
ModUp / ModDown / rescale (Appendix A "Key-switching", "Multiplication")."""
import random

import numpy as np
import pytest
import sympy

from oracle import oracle as O


@pytest.fixture(scope="module")
def tiny():
    # N=16, four Q primes, two special primes, two primes per digit
    return O.make_params(N=16, L=3, K=2, alpha=2)


def rand_res(rng, moduli, N):
    return np.stack([rng.integers(0, q, size=N, dtype=np.uint64) for q in moduli])


def test_prime_rule_config1_and_2():
    for prm in (O.config1_params(), O.config2_params()):
        twoN = 2 * prm.N
        allm = prm.q + prm.p
        assert len(set(allm)) == len(allm)
        for q in allm:
            assert q % twoN == 1
            assert sympy.isprime(q)
        assert prm.q[0] < 2 ** 60 and prm.q[0] > 2 ** 59
        assert all(2 ** 39 < q < 2 ** 40 for q in prm.q[1:])
        # greedy from the top: every skipped candidate between chosen primes is composite
        tops = sorted([prm.q[0]] + prm.p, reverse=True)
        for hi, lo in zip([2 ** 60] + tops[:-1], tops):
            c = hi - 1 - ((hi - 2) % twoN)
            while c > lo:
                if c < hi:
                    assert not sympy.isprime(c)
                c -= twoN
        assert prm.q[1:] == sorted(prm.q[1:], reverse=True)
        assert prm.p == sorted(prm.p, reverse=True)
        assert prm.p[0] < prm.q[0]


def test_psi_is_primitive_2N_root():
    for prm in (O.config1_params(), O.config2_params()):
        for q in prm.q + prm.p:
            psi = prm.psi[q]
            assert pow(psi, prm.N, q) == q - 1
            assert pow(psi, 2 * prm.N, q) == 1
            # psi comes from the smallest quadratic non-residue
            x = 2
            while sympy.legendre_symbol(x, q) != -1:
                x += 1
            assert psi == pow(x, (q - 1) // (2 * prm.N), q)


@pytest.mark.parametrize("N", [8, 16, 64, 256, 1024])
def test_ntt_equals_evaluation_definition(N):
    prm = O.make_params(N=N, L=2, K=1, alpha=1)
    rng = np.random.default_rng(N)
    lg = N.bit_length() - 1
    for q in prm.q + prm.p:
        a = rng.integers(0, q, size=N, dtype=np.uint64)
        fast = O.ntt(a[None], [q], prm)[0]
        if N <= 256:
            # the definition, evaluated with Python integers
            psi = prm.psi[q]
            for j in range(N):
                x = pow(psi, 2 * int(f"{j:0{lg}b}"[::-1], 2) + 1, q)
                assert int(fast[j]) == sum(int(a[c]) * pow(x, c, q) for c in range(N)) % q
        assert np.array_equal(fast, O.ntt_definition(a, q, prm.psi[q]))
        assert np.array_equal(O.intt(fast[None], [q], prm)[0], a)


@pytest.mark.parametrize("N", [8, 32, 128])
def test_ntt_pointwise_product_is_negacyclic_convolution(N):
    prm = O.make_params(N=N, L=2, K=1, alpha=1)
    rng = np.random.default_rng(7 + N)
    for q in prm.q + prm.p:
        a = rng.integers(0, q, size=N, dtype=np.uint64)
        b = rng.integers(0, q, size=N, dtype=np.uint64)
        # independent schoolbook with Python integers
        ref = [0] * N
        for i in range(N):
            for j in range(N):
                t = int(a[i]) * int(b[j])
                if i + j < N:
                    ref[i + j] += t
                else:
                    ref[i + j - N] -= t
        ref = np.array([x % q for x in ref], dtype=np.uint64)
        assert np.array_equal(O.schoolbook(a, b, q), ref)
        fa, fb = O.ntt(a[None], [q], prm), O.ntt(b[None], [q], prm)
        prod = O.intt(O.mul(fa, fb, [q]), [q], prm)[0]
        assert np.array_equal(prod, ref)


def test_ntt_full_size_sampled_points():
    prm = O.config2_params()
    rng = np.random.default_rng(3)
    for q in (prm.q[0], prm.q[5], prm.p[-1]):
        a = rng.integers(0, q, size=prm.N, dtype=np.uint64)
        fast = O.ntt(a[None], [q], prm)[0]
        for j in rng.integers(0, prm.N, size=24):
            assert int(fast[j]) == O.ntt_definition_at(a, q, prm.psi[q], int(j))
        assert np.array_equal(O.intt(fast[None], [q], prm)[0], a)


def test_automorphism_forms(tiny):
    prm = tiny
    rng = np.random.default_rng(11)
    Q = prm.Q(prm.L)
    a = rand_res(rng, Q, prm.N)
    for k in (1, 2, 3, 5, prm.n - 1):
        g = O.galois_for_step(k, prm)
        co = O.automorph_coeff(a, g, Q)
        # sigma_g(a)(x) = a(x^g) at roots x of X^N + 1 (x = psi^odd), by Python evaluation
        for li, q in enumerate(Q):
            for e in rng.integers(0, prm.N, size=3):
                x = pow(prm.psi[q], 2 * int(e) + 1, q)
                lhs = sum(int(co[li, c]) * pow(x, c, q) for c in range(prm.N)) % q
                xg = pow(x, g, q)
                rhs = sum(int(a[li, c]) * pow(xg, c, q) for c in range(prm.N)) % q
                assert lhs == rhs
        # evaluation-form permutation equals the coefficient form
        ev = O.automorph_ntt(O.ntt(a, Q, prm), g, prm.N)
        assert np.array_equal(O.intt(ev, Q, prm), co)
    # sigma_g sigma_h = sigma_gh
    g, h = O.galois_for_step(3, prm), O.galois_for_step(5, prm)
    A = O.ntt(a, Q, prm)
    lhs = O.automorph_ntt(O.automorph_ntt(A, h, prm.N), g, prm.N)
    assert np.array_equal(lhs, O.automorph_ntt(A, g * h % (2 * prm.N), prm.N))


def test_modup_closed_form(tiny):
    prm = tiny
    rng = np.random.default_rng(5)
    for level in (prm.L, 2, 0):
        Q = prm.Q(level)
        PQ = prm.PQ(level)
        c1 = rand_res(rng, Q, prm.N)
        digits = O.modup(prm, c1, level)
        xc = O.intt(c1, Q, prm)
        assert len(digits) == prm.n_digits(level)
        for j, d in enumerate(digits):
            Dj = prm.digit(j, level)
            Qj = 1
            for i in Dj:
                Qj *= Q[i]
            x = O.crt(xc[Dj], [Q[i] for i in Dj])
            dv = O.crt(O.intt(d, PQ, prm), PQ)
            for c in range(prm.N):
                u, r = divmod(dv[c] - x[c], Qj)
                assert r == 0 and 0 <= u < len(Dj)


def test_moddown_closed_form(tiny):
    prm = tiny
    rng = np.random.default_rng(6)
    P = 1
    for p in prm.p:
        P *= p
    for level in (prm.L, 1):
        Q, PQ = prm.Q(level), prm.PQ(level)
        Qv = 1
        for q in Q:
            Qv *= q
        X = rand_res(rng, PQ, prm.N)[None]
        out = O.moddown(prm, X, level)[0]
        xv = O.crt(O.intt(X[0], PQ, prm), PQ)
        ov = O.crt(O.intt(out, Q, prm), Q)
        for c in range(prm.N):
            u = (xv[c] // P - ov[c]) % Qv
            assert 0 <= u < prm.K


def test_rescale_closed_form(tiny):
    prm = tiny
    rng = np.random.default_rng(8)
    for level in (prm.L, 1):
        Q = prm.Q(level)
        ct = rand_res(rng, Q, prm.N)[None]
        out = O.rescale(prm, ct, level)[0]
        ql = Q[level]
        Qm = 1
        for q in Q[:level]:
            Qm *= q
        C = O.crt(O.intt(ct[0], Q, prm), Q)
        got = O.crt(O.intt(out, Q[:level], prm), Q[:level])
        for c in range(prm.N):
            assert got[c] == ((C[c] + ql // 2) // ql) % Qm


def test_basis_convert_exact_integer(tiny):
    prm = tiny
    rng = np.random.default_rng(9)
    qin = prm.q[:3]
    qout = prm.p + [prm.q[3]]
    x = rand_res(rng, qin, prm.N)
    out = O.basis_convert(x, qin, qout)
    Qin = qin[0] * qin[1] * qin[2]
    xv = O.crt(x, qin)
    for c in range(prm.N):
        # the converted value is x + u Qin for one integer 0 <= u < 3, the same for every output prime
        us = set()
        for r, qr in enumerate(qout):
            for u in range(3):
                if (xv[c] + u * Qin) % qr == int(out[r, c]):
                    us.add(u)
        assert len(us) >= 1
        assert any(all((xv[c] + u * Qin) % qr == int(out[r, c]) for r, qr in enumerate(qout)) for u in us)


def test_splitmix64_published_outputs():
    """The counter-based generator behind seeded key polynomials reproduces
    the published SplitMix64 outputs (output n of seed s is the n-th draw)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")) as f:
        g = json.load(f)
    for case in g["outputs"]:
        for n, v in enumerate(case["values"], start=1):
            assert O.splitmix64(case["seed"], n) == int(v, 0)


def test_key_uniform_definition_and_spread(tiny):
    """a = (X mod q) 2^-128 mod q, c = x + 2^16 p + 2^24 j, with
    X = out_{2c+2} 2^64 + out_{2c+1} on primes of 40 bits or more and, below
    2^40, the first of out_{2c+1}, out_{2^32+4c+t} (t = 1..3) below
    2^64 - (2^64 mod q); values cover [0, q) evenly."""
    prm = tiny
    seed = 0x1234_5678_9ABC_DEF0
    allm = prm.q + prm.p
    for j in range(prm.dnum):
        a = O.key_uniform(prm, seed, j)
        for p, q in enumerate(allm):
            for x in (0, 1, prm.N - 1):
                c = x + (p << 16) + (j << 24)
                if q >= 2 ** 40:
                    X = (O.splitmix64(seed, 2 * c + 2) << 64) | O.splitmix64(seed, 2 * c + 1)
                else:
                    X = O.splitmix64(seed, 2 * c + 1)
                    assert X < 2 ** 64 - 2 ** 64 % q   # no rejection at these coefficients
                assert int(a[p, x]) == (X % q) * pow(pow(2, 128, q), -1, q) % q
    # spread: a larger ring, the fraction of values in each quarter of [0, q)
    big = O.make_params(N=4096, L=1, K=1, alpha=1)
    a = O.key_uniform(big, 7, 0)
    for p, q in enumerate(big.q + big.p):
        quarters = np.bincount((a[p].astype(object) * 4 // q).astype(np.int64), minlength=4) / big.N
        assert np.all(np.abs(quarters - 0.25) < 0.03)


# (ring, seed, digit, prime index, coefficient) where the first 64-bit
# candidate of a prime below 2^40 lies in the rejected range [2^64 - (2^64 mod
# q), 2^64); found by scanning seeds
REJECTION_CASES = [("cfg1", 541, 3, 2, 892), ("cfg2", 1208, 0, 22, 7462)]


@pytest.mark.parametrize("case", REJECTION_CASES)
def test_key_uniform_rejection(case):
    """Below 2^40 a candidate X >= 2^64 - (2^64 mod q) would make the small
    residues one count more likely than the others (2^64 is not a multiple
    of q); the sampler rejects it and takes the next candidate of its own
    counter range, so every accepted X lies in a whole number of periods of q
    (X mod q exactly uniform)."""
    ring, seed, j, p, x = case
    prm = O.config1_params() if ring == "cfg1" else O.config2_params()
    q = (prm.q + prm.p)[p]
    assert q < 2 ** 40
    lam = 2 ** 64 - 2 ** 64 % q
    assert lam % q == 0
    c = x + (p << 16) + (j << 24)
    first = O.splitmix64(seed, 2 * c + 1)
    assert first >= lam, "the case must exercise the rejection"
    second = O.splitmix64(seed, 2 ** 32 + 4 * c + 1)
    assert second < lam
    assert O.key_uniform_sample40(seed, c, q) == second
    a = O.key_uniform(prm, seed, j)
    assert int(a[p, x]) == (second % q) * pow(pow(2, 128, q), -1, q) % q
    # neighbours draw no rejection: their first candidate is kept
    for xx in (x - 1, x + 1):
        cc = xx + (p << 16) + (j << 24)
        assert O.key_uniform_sample40(seed, cc, q) == O.splitmix64(seed, 2 * cc + 1)
