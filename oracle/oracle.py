"""CPU oracle for the HE-LRM encrypted-lookup hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference of what the GPU library computes.
Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
it.  It shares no code with the GPU library: the modular loops are in
``ckks_oracle.c`` (full 128-bit products and ``%``), the orchestration below
follows the method step by step.

Paper sections followed (arXiv 2506.18150):
  * Appendix A, "Encoding"/"Encryption"/"Multiplication"/"Rotation"/
    "Key-switching": CKKS over R_Q = Z_Q[X]/(X^N+1), rescale Q_l -> Q_{l-1}.
  * Sec. II-A "System-Level Costs": rotations need a key switch with one
    evaluation key per rotation offset.
  * Sec. II-A "Neural Network Layers in FHE": diagonal (Halevi-Shoup)
    matrix-vector product and its baby-step giant-step (BSGS) form.
  * Sec. III-B "Matrix-Vector Lookup": y = E^T s costs one level; the
    double-hoisted BSGS variant is used.
  * Sec. IV-A "Deterministic digit encoding" / "Compressed embedding
    parameterization": base-p digits, y = sum_j C_j[i_j].
  * Sec. IV-B "Block-diagonal embedding matrix": M = block_diag(W_t), the
    selector is the concatenation of per-table one-hots.
  * Sec. II-B / Sec. V-C: the small DLRM (dense features and embedding
    lookups into bottom and top MLPs with a square activation), built from
    the same matvec, ciphertext products with relinearisation, plaintext
    additions and level alignment.

The paper leaves the following open; this oracle takes these readings (the
GPU library must take the same ones for bit-exact parity):
  * primes q = 1 mod 2N chosen greedily from the top (largest below 2^60 for
    q_0 and the special primes, below 2^40 for q_1..q_L); psi from the
    smallest quadratic non-residue;
  * evaluation form = values at psi^(2 brv(j)+1) (bit-reversed order);
  * rotation left by k <-> Galois element 5^k mod 2N;
  * hybrid key switching with dnum digits of alpha primes and K special
    primes; ModUp uncorrected; ModDown without a rounding offset; hoisted
    rotations apply the automorphism after ModUp; rescale rounds half up;
    the uniform part of every switching key is expanded from a 64-bit seed
    with SplitMix64 (a counter-based generator, so a key stores only b_j);
  * hybrid diagonals u_k[j] = M[j mod m][(j+k) mod n] for k < m,
    m = next_pow2(rows), summed over the m-periodic copies by a fold.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile ckks_oracle.c with gcc into liboracle.so (plain C, OpenMP)."""
    src = os.path.join(_HERE, "ckks_oracle.c")
    if force or not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(src):
        import subprocess
        tmp = _LIBPATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _LIBPATH)
    return _LIBPATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        L = ctypes.CDLL(_LIBPATH)
        u64 = ctypes.c_uint64
        ci = ctypes.c_int
        L.or_mulmod.restype = u64; L.or_mulmod.argtypes = [u64, u64, u64]
        L.or_powmod.restype = u64; L.or_powmod.argtypes = [u64, u64, u64]
        L.or_invmod.restype = u64; L.or_invmod.argtypes = [u64, u64]
        L.or_is_prime.restype = ci; L.or_is_prime.argtypes = [u64]
        L.or_primes_below.restype = ci; L.or_primes_below.argtypes = [u64, u64, ci, u64p]
        L.or_find_psi.restype = u64; L.or_find_psi.argtypes = [u64, u64]
        L.or_bitrev.restype = u64; L.or_bitrev.argtypes = [u64, ci]
        L.or_ntt_definition_at.restype = u64
        L.or_ntt_definition_at.argtypes = [u64p, ci, u64, u64, ci]
        L.or_ntt_definition.argtypes = [u64p, u64p, ci, u64, u64]
        for f in (L.or_ntt, L.or_intt):
            f.argtypes = [u64p, ci, ci, u64p, u64p]
        L.or_negacyclic_schoolbook.argtypes = [u64p, u64p, u64p, ci, u64]
        L.or_automorph_coeff.argtypes = [u64p, u64p, ci, ci, u64p, u64]
        L.or_automorph_ntt.argtypes = [u64p, u64p, ci, ci, u64]
        for f in (L.or_mul, L.or_add, L.or_sub, L.or_mul_scalar):
            f.argtypes = [u64p, u64p, u64p, ci, ci, u64p]
        L.or_from_signed.argtypes = [i64p, u64p, ci, ci, u64p]
        L.or_basis_convert.argtypes = [u64p, ci, u64p, u64p, ci, u64p, ci]
        L.or_splitmix64.restype = u64; L.or_splitmix64.argtypes = [u64, u64]
        L.or_set_threads.argtypes = [ci]
        L.or_max_threads.restype = ci; L.or_max_threads.argtypes = []
        L.or_key_uniform.argtypes = [u64, ci, ci, u64, ci, u64p]
        L.or_key_uniform_sample40.restype = u64
        L.or_key_uniform_sample40.argtypes = [u64, u64, u64]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Thread count of the C loops (OpenMP)."""
    lib().or_set_threads(int(n))


def max_threads() -> int:
    """Threads the next C loop may use."""
    return int(lib().or_max_threads())


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.uint64:
        return a.ctypes.data_as(u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(i64p)
    raise TypeError(a.dtype)


def _u(x: Sequence[int]) -> np.ndarray:
    return np.ascontiguousarray(np.array([int(v) for v in x], dtype=np.uint64))


# ------------------------------------------------------------------ scalars

def mulmod(a, b, q): return int(lib().or_mulmod(int(a), int(b), int(q)))
def powmod(a, e, q): return int(lib().or_powmod(int(a), int(e), int(q)))
def invmod(a, q): return int(lib().or_invmod(int(a) % int(q), int(q)))
def is_prime(n): return bool(lib().or_is_prime(int(n)))
def bitrev(x, bits): return int(lib().or_bitrev(int(x), int(bits)))


def primes_below(bound: int, step: int, count: int) -> List[int]:
    out = np.zeros(count, dtype=np.uint64)
    got = lib().or_primes_below(int(bound), int(step), int(count), _p(out))
    assert got == count
    return [int(v) for v in out]


def find_psi(q: int, N: int) -> int:
    return int(lib().or_find_psi(int(q), int(N)))


# ------------------------------------------------------------------ parameters

@dataclass
class Params:
    """RNS-CKKS parameters.  Q primes q_0..q_L, special primes p_0..p_{K-1},
    digits of alpha consecutive Q primes (dnum = ceil((L+1)/alpha))."""
    N: int
    L: int
    K: int
    alpha: int
    q: List[int]
    p: List[int]
    delta: float
    psi: Dict[int, int] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.N // 2

    @property
    def dnum(self) -> int:
        return -(-(self.L + 1) // self.alpha)

    @property
    def logN(self) -> int:
        return self.N.bit_length() - 1

    def Q(self, level: int) -> List[int]:
        return self.q[: level + 1]

    def PQ(self, level: int) -> List[int]:
        return self.q[: level + 1] + self.p

    def digit(self, j: int, level: int) -> List[int]:
        """Indices of the Q primes of digit j that are active at this level."""
        return [i for i in range(j * self.alpha, (j + 1) * self.alpha) if i <= level]

    def n_digits(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def key_limbs(self, level: int) -> List[int]:
        """Positions, inside a full-level PQ key, of the limbs used at this level."""
        return list(range(level + 1)) + list(range(self.L + 1, self.L + 1 + self.K))

    def P_mod(self, m: int) -> int:
        r = 1
        for pk in self.p:
            r = r * pk % m
        return r

    def psis(self, moduli: Sequence[int]) -> np.ndarray:
        return _u([self.psi[m] for m in moduli])


def make_params(N: int, L: int, K: int, alpha: int, q0_bits: int = 60, q_bits: int = 40,
                p_bits: int = 60, delta: float = 2.0 ** 40) -> Params:
    """Prime rule: q_0 and the special primes are the largest primes
    = 1 mod 2N below 2^q0_bits (q_0 first, then p_0 > p_1 > ...); q_1..q_L
    are the L largest such primes below 2^q_bits, descending."""
    twoN = 2 * N
    assert q0_bits == p_bits
    top = primes_below(1 << q0_bits, twoN, 1 + K)
    qs = primes_below(1 << q_bits, twoN, L)
    prm = Params(N=N, L=L, K=K, alpha=alpha, q=[top[0]] + qs, p=top[1:], delta=delta)
    for m in prm.q + prm.p:
        prm.psi[m] = find_psi(m, N)
    return prm


def config1_params() -> Params:
    """Toy ring N=2^12: q_0 (60-bit), three ~40-bit primes, one 60-bit special
    prime, one prime per key-switching digit."""
    return make_params(N=1 << 12, L=3, K=1, alpha=1)


def config2_params() -> Params:
    """N=2^16: q_0 (60-bit) + 23 ~40-bit primes, dnum=3 (alpha=8), K=8 special
    60-bit primes."""
    return make_params(N=1 << 16, L=23, K=8, alpha=8)


# ------------------------------------------------------------------ polynomial loops

def ntt(a: np.ndarray, moduli: Sequence[int], prm: Params) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    lib().or_ntt(_p(out), len(moduli), prm.N, _p(_u(moduli)), _p(prm.psis(moduli)))
    return out


def intt(a: np.ndarray, moduli: Sequence[int], prm: Params) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    lib().or_intt(_p(out), len(moduli), prm.N, _p(_u(moduli)), _p(prm.psis(moduli)))
    return out


def ntt_definition(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.zeros_like(a)
    lib().or_ntt_definition(_p(a), _p(out), len(a), int(q), int(psi))
    return out


def ntt_definition_at(a: np.ndarray, q: int, psi: int, j: int) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return int(lib().or_ntt_definition_at(_p(a), len(a), int(q), int(psi), int(j)))


def schoolbook(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.zeros_like(a)
    lib().or_negacyclic_schoolbook(_p(a), _p(b), _p(out), len(a), int(q))
    return out


def _ew(fn, a, b, moduli):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    fn(_p(a), _p(b), _p(out), a.shape[0], a.shape[1], _p(_u(moduli)))
    return out


def mul(a, b, moduli): return _ew(lib().or_mul, a, b, moduli)
def add(a, b, moduli): return _ew(lib().or_add, a, b, moduli)
def sub(a, b, moduli): return _ew(lib().or_sub, a, b, moduli)


def mul_scalar(a, scalars, moduli):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().or_mul_scalar(_p(a), _p(_u(scalars)), _p(out), a.shape[0], a.shape[1], _p(_u(moduli)))
    return out


def neg(a, moduli):
    return sub(np.zeros_like(a), a, moduli)


def from_signed(v: np.ndarray, moduli: Sequence[int]) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int64)
    out = np.empty((len(moduli), len(v)), dtype=np.uint64)
    lib().or_from_signed(_p(v), _p(out), len(moduli), len(v), _p(_u(moduli)))
    return out


def automorph_ntt(a: np.ndarray, g: int, N: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().or_automorph_ntt(_p(a), _p(out), a.shape[0], N, int(g))
    return out


def automorph_coeff(a: np.ndarray, g: int, moduli: Sequence[int]) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().or_automorph_coeff(_p(a), _p(out), a.shape[0], a.shape[1], _p(_u(moduli)), int(g))
    return out


def basis_convert(x: np.ndarray, qin: Sequence[int], qout: Sequence[int]) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.empty((len(qout), x.shape[1]), dtype=np.uint64)
    lib().or_basis_convert(_p(x), len(qin), _p(_u(qin)), _p(out), len(qout), _p(_u(qout)), x.shape[1])
    return out


def galois_for_step(k: int, prm: Params) -> int:
    """Rotation left by k slots <-> X -> X^(5^k mod 2N)."""
    return pow(5, k % prm.n, 2 * prm.N)


# ------------------------------------------------------------------ encoding (App. A "Encoding")

def encode(z, scale: float, prm: Params) -> np.ndarray:
    """Inverse canonical embedding times scale, rounded half away from zero.
    Slot j sits at the root zeta^(5^j mod 2N), zeta = exp(i pi/N); a vector
    shorter than N/2 is zero-padded.  Returns int64 coefficients."""
    N, n = prm.N, prm.n
    z = _pad(z, n)
    Z = np.zeros(2 * N, dtype=np.complex128)
    idx = _rot_group(prm)
    Z[idx] = scale * z
    Z[(-idx) % (2 * N)] = np.conj(scale * z)
    m = np.fft.fft(Z)[:N].real / N
    r = np.sign(m) * np.floor(np.abs(m) + 0.5)
    return r.astype(np.int64)


def encode_direct(z, scale: float, prm: Params) -> np.ndarray:
    """The same map written as its defining sum (O(N^2), for small N only):
    m_c = (2/N) sum_j Re(scale z_j zeta^(-5^j c))."""
    N, n = prm.N, prm.n
    z = _pad(z, n)
    idx = _rot_group(prm)
    c = np.arange(N)
    ang = -np.pi * np.outer(idx, c) / N
    m = (2.0 / N) * np.real((scale * z)[:, None] * np.exp(1j * ang)).sum(axis=0)
    return (np.sign(m) * np.floor(np.abs(m) + 0.5)).astype(np.int64)


def decode(coeffs, scale: float, prm: Params) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) / scale for real-valued integer coefficients."""
    N = prm.N
    m = np.zeros(2 * N, dtype=np.float64)
    m[:N] = np.asarray(coeffs, dtype=np.float64)
    ev = np.fft.ifft(m) * (2 * N)
    return ev[_rot_group(prm)] / scale


def _rot_group(prm: Params) -> np.ndarray:
    idx = np.empty(prm.n, dtype=np.int64)
    x = 1
    for j in range(prm.n):
        idx[j] = x
        x = x * 5 % (2 * prm.N)
    return idx


def _pad(z, n):
    z = np.asarray(z, dtype=np.complex128).ravel()
    out = np.zeros(n, dtype=np.complex128)
    out[: len(z)] = z
    return out


# ------------------------------------------------------------------ keys (App. A "Key-switching")

@dataclass
class Keys:
    s: np.ndarray                    # secret in evaluation form over all PQ primes [L+1+K][N]
    pk: Tuple[np.ndarray, np.ndarray]  # (b, a) over Q_L
    swk: Dict[int, np.ndarray] = field(default_factory=dict)  # galois -> uint64 [dnum][2][L+1+K][N]
    relin: Optional[np.ndarray] = None
    seeds: Dict[int, int] = field(default_factory=dict)       # galois (0: relinearisation) -> seed of a_j


def splitmix64(seed: int, n: int) -> int:
    return int(lib().or_splitmix64(int(seed) & (2 ** 64 - 1), int(n) & (2 ** 64 - 1)))


def key_uniform_sample40(seed: int, c: int, q: int) -> int:
    """The 64-bit sample X of counter c on a prime q below 2^40: SplitMix64
    outputs tried in order (2c+1, then 2^32 + 4c + t for t = 1..3), the first
    below 2^64 - (2^64 mod q) taken (ckks_oracle.c, or_key_uniform_sample40)."""
    return int(lib().or_key_uniform_sample40(int(seed) & (2 ** 64 - 1), int(c), int(q)))


def key_uniform(prm: Params, seed: int, j: int) -> np.ndarray:
    """Uniform polynomial a_j of a switching key over every prime of PQ_L
    (evaluation form), expanded from the key's seed by the counter-based
    SplitMix64 generator (ckks_oracle.c, or_key_uniform): a 128-bit sample on
    primes of 40 bits or more, a rejection-sampled 64-bit one below."""
    allm = prm.q + prm.p
    out = np.empty((len(allm), prm.N), dtype=np.uint64)
    for p, q in enumerate(allm):
        row = np.empty(prm.N, dtype=np.uint64)
        lib().or_key_uniform(int(seed), j, p, int(q), prm.N, _p(row))
        out[p] = row
    return out


def _switch_key(prm: Params, s_all: np.ndarray, s_from: np.ndarray, draws) -> np.ndarray:
    """Hybrid switching key from s_from to s: for digit j,
    b_j = -a_j s + e_j + [P Qhat_j (Qhat_j^-1 mod Q_j)] s_from over PQ_L.
    The gadget factor is [P]_{q_i} on the primes of digit j and 0 elsewhere;
    a_j is expanded from the key's seed."""
    allm = prm.q + prm.p
    out = np.zeros((prm.dnum, 2, len(allm), prm.N), dtype=np.uint64)
    for j in range(prm.dnum):
        a = key_uniform(prm, draws.a_seed, j)
        e = ntt(from_signed(draws.e[j], allm), allm, prm)
        b = add(neg(mul(a, s_all, allm), allm), e, allm)
        for i in prm.digit(j, prm.L):
            g = prm.P_mod(prm.q[i])
            b[i] = add(b[i:i + 1], mul_scalar(s_from[i:i + 1], [g], [prm.q[i]]), [prm.q[i]])[0]
        out[j, 0] = b
        out[j, 1] = a
    return out


def keygen(prm: Params, draws) -> Keys:
    """Secret, public key (-a s + e, a) and one switching key per Galois
    element in the draws (for sigma_g(s) -> s), plus relinearisation (s^2 -> s)."""
    allm = prm.q + prm.p
    s_all = ntt(from_signed(draws.s, allm), allm, prm)
    QL = prm.q
    sQ = s_all[: prm.L + 1]
    pk_a = np.ascontiguousarray(draws.pk_a, dtype=np.uint64)
    pk_e = ntt(from_signed(draws.pk_e, QL), QL, prm)
    pk_b = add(neg(mul(pk_a, sQ, QL), QL), pk_e, QL)
    keys = Keys(s=s_all, pk=(pk_b, pk_a))
    for gal, d in draws.swk.items():
        keys.swk[gal] = _switch_key(prm, s_all, automorph_ntt(s_all, gal, prm.N), d)
        keys.seeds[gal] = d.a_seed
    if draws.relin is not None:
        keys.relin = _switch_key(prm, s_all, mul(s_all, s_all, allm), draws.relin)
        keys.seeds[0] = draws.relin.a_seed
    return keys


def encrypt(prm: Params, keys: Keys, m_coeffs: np.ndarray, level: int, ed) -> np.ndarray:
    """Public-key encryption at the given level: (v b + e0 + m, v a + e1).
    Returns uint64 [2][level+1][N] in evaluation form."""
    Q = prm.Q(level)
    v = ntt(from_signed(ed.v, Q), Q, prm)
    e0 = ntt(from_signed(ed.e0, Q), Q, prm)
    e1 = ntt(from_signed(ed.e1, Q), Q, prm)
    m = ntt(from_signed(m_coeffs, Q), Q, prm)
    b, a = keys.pk[0][: level + 1], keys.pk[1][: level + 1]
    c0 = add(add(mul(v, b, Q), e0, Q), m, Q)
    c1 = add(mul(v, a, Q), e1, Q)
    return np.stack([c0, c1])


def decrypt(prm: Params, keys: Keys, ct: np.ndarray) -> np.ndarray:
    """m = c0 + c1 s on the q_0 limb, centred in (-q_0/2, q_0/2] (valid while
    |m| < q_0/2).  Returns int64 coefficients."""
    q0 = prm.q[0]
    m = add(ct[0, :1], mul(ct[1, :1], keys.s[:1], [q0]), [q0])
    m = intt(m, [q0], prm)[0].astype(object)
    m = np.where(m > q0 // 2, m - q0, m)
    return np.array([int(x) for x in m], dtype=np.int64)


def decrypt_full(prm: Params, keys: Keys, ct: np.ndarray, level: int) -> List[int]:
    """c0 + c1 s over every limb of Q_level, CRT-combined and centred (Python
    ints).  Used for invariants that must hold modulo the whole Q."""
    Q = prm.Q(level)
    m = add(ct[0], mul(ct[1], keys.s[: level + 1], Q), Q)
    m = intt(m, Q, prm)
    return crt_centered(m, Q)


def crt(res: np.ndarray, moduli: Sequence[int]) -> List[int]:
    """CRT combination of residues [limb][N] into integers in [0, prod)."""
    M = 1
    for q in moduli:
        M *= int(q)
    out = [0] * res.shape[1]
    for i, q in enumerate(moduli):
        Mi = M // int(q)
        c = Mi * pow(Mi % int(q), -1, int(q))
        col = res[i]
        for j in range(res.shape[1]):
            out[j] += int(col[j]) * c
    return [v % M for v in out]


def crt_centered(res: np.ndarray, moduli: Sequence[int]) -> List[int]:
    M = 1
    for q in moduli:
        M *= int(q)
    return [v - M if v > M // 2 else v for v in crt(res, moduli)]


# ------------------------------------------------------------------ key switching pieces

def modup(prm: Params, c1: np.ndarray, level: int) -> List[np.ndarray]:
    """Digit decomposition + fast base conversion to PQ_level (no correction).
    Returns one array [level+1+K][N] per active digit, evaluation form; the
    digit's own limbs are copied from c1."""
    Q = prm.Q(level)
    PQ = prm.PQ(level)
    x = intt(c1, Q, prm)
    digits = []
    for j in range(prm.n_digits(level)):
        Dj = prm.digit(j, level)
        targets = [r for r in range(level + 1 + prm.K) if r not in Dj]
        conv = basis_convert(x[Dj], [Q[i] for i in Dj], [PQ[r] for r in targets])
        conv = ntt(conv, [PQ[r] for r in targets], prm)
        d = np.empty((len(PQ), prm.N), dtype=np.uint64)
        for i in Dj:
            d[i] = c1[i]
        for t, r in enumerate(targets):
            d[r] = conv[t]
        digits.append(d)
    return digits


def key_inner_product(prm: Params, digits: List[np.ndarray], c0: np.ndarray, level: int,
                      key: np.ndarray, galois: int) -> np.ndarray:
    """Hoisted rotation kept in PQ (no ModDown):
       A = sum_j sigma_g(d_j) a_j,  B = sum_j sigma_g(d_j) b_j + P sigma_g(c0).
    galois == 1 means no automorphism.  Returns [2][level+1+K][N] = (B, A)."""
    PQ = prm.PQ(level)
    kl = prm.key_limbs(level)
    A = np.zeros((len(PQ), prm.N), dtype=np.uint64)
    B = np.zeros((len(PQ), prm.N), dtype=np.uint64)
    for j, d in enumerate(digits):
        ds = d if galois == 1 else automorph_ntt(d, galois, prm.N)
        kb = np.ascontiguousarray(key[j, 0][kl])
        ka = np.ascontiguousarray(key[j, 1][kl])
        B = add(B, mul(ds, kb, PQ), PQ)
        A = add(A, mul(ds, ka, PQ), PQ)
    c0s = c0 if galois == 1 else automorph_ntt(c0, galois, prm.N)
    Q = prm.Q(level)
    B[: level + 1] = add(B[: level + 1], mul_scalar(c0s, [prm.P_mod(q) for q in Q], Q), Q)
    return np.stack([B, A])


def lift_P(prm: Params, ct: np.ndarray, level: int) -> np.ndarray:
    """(P c0, P c1) over PQ_level: [P]_{q_i} c on Q limbs, 0 on the special limbs."""
    Q = prm.Q(level)
    out = np.zeros((2, level + 1 + prm.K, prm.N), dtype=np.uint64)
    sc = [prm.P_mod(q) for q in Q]
    for c in range(2):
        out[c, : level + 1] = mul_scalar(ct[c], sc, Q)
    return out


def moddown(prm: Params, X: np.ndarray, level: int) -> np.ndarray:
    """Divide by P: t = BaseConv_{P -> Q}(X mod P) from the special limbs in
    coefficient form; out_i = (X_i - t_i) P^-1 mod q_i.  X: [c][level+1+K][N]."""
    Q = prm.Q(level)
    out = np.empty((X.shape[0], level + 1, prm.N), dtype=np.uint64)
    for c in range(X.shape[0]):
        xp = intt(X[c, level + 1:], prm.p, prm)
        t = ntt(basis_convert(xp, prm.p, Q), Q, prm)
        diff = sub(X[c, : level + 1], t, Q)
        out[c] = mul_scalar(diff, [invmod(prm.P_mod(q), q) for q in Q], Q)
    return out


def rescale(prm: Params, ct: np.ndarray, level: int) -> np.ndarray:
    """Q_l -> Q_{l-1}: every coefficient C becomes floor((C + h)/q_l) with
    h = floor(q_l/2).  Per limb: (c_i - [t - h]_{q_i}) q_l^-1 with
    t = (c_l + h) mod q_l taken in coefficient form."""
    ql = prm.q[level]
    h = ql // 2
    Q = prm.Q(level - 1)
    out = np.empty((ct.shape[0], level, prm.N), dtype=np.uint64)
    for c in range(ct.shape[0]):
        cl = intt(ct[c, level:level + 1], [ql], prm)[0]
        t = (cl.astype(object) + h) % ql
        tm = np.array([int(v) - h for v in t], dtype=np.int64)
        r = ntt(from_signed(tm, Q), Q, prm)
        out[c] = mul_scalar(sub(ct[c, :level], r, Q), [invmod(ql, q) for q in Q], Q)
    return out


def rotate(prm: Params, keys: Keys, ct: np.ndarray, k: int, level: int) -> np.ndarray:
    """Full rotation left by k slots: ModUp, automorphism, key product, ModDown,
    then add the rotated c0 part (included in the key product as P sigma(c0))."""
    g = galois_for_step(k, prm)
    d = modup(prm, ct[1], level)
    return moddown(prm, key_inner_product(prm, d, ct[0], level, keys.swk[g], g), level)


def hoisted_rotations(prm: Params, keys: Keys, ct: np.ndarray, level: int,
                      steps: Sequence[int]) -> List[np.ndarray]:
    """One ModUp shared by every rotation; each output kept in PQ."""
    d = modup(prm, ct[1], level)
    out = []
    for k in steps:
        g = galois_for_step(k, prm)
        out.append(key_inner_product(prm, d, ct[0], level, keys.swk[g], g))
    return out


# ------------------------------------------------------------------ ciphertext products (App. A "Multiplication")

def tensor(prm: Params, a: np.ndarray, b: np.ndarray, level: int) -> np.ndarray:
    """(a0 + a1 s)(b0 + b1 s) = d0 + d1 s + d2 s^2 with d0 = a0 b0,
    d1 = a0 b1 + a1 b0, d2 = a1 b1, pointwise in evaluation form over Q_level.
    Returns [3][level+1][N]."""
    Q = prm.Q(level)
    d0 = mul(a[0], b[0], Q)
    d1 = add(mul(a[0], b[1], Q), mul(a[1], b[0], Q), Q)
    d2 = mul(a[1], b[1], Q)
    return np.stack([d0, d1, d2])


def relinearize(prm: Params, keys: Keys, d: np.ndarray, level: int) -> np.ndarray:
    """Switch d2 from s^2 to s with the relinearisation key and add (d0, d1):
    ModDown(P (d0, d1) + sum_j ModUp(d2)_j (b_j, a_j)).  P (d0, d1) vanishes
    modulo every special prime, so adding it before the ModDown gives the same
    residues as adding (d0, d1) after it."""
    PQ = prm.PQ(level)
    digits = modup(prm, d[2], level)
    zero = np.zeros((level + 1, prm.N), dtype=np.uint64)
    X = key_inner_product(prm, digits, zero, level, keys.relin, 1)
    Lp = lift_P(prm, d[:2], level)
    for c in range(2):
        X[c] = add(X[c], Lp[c], PQ)
    return moddown(prm, X, level)


def mul_relin(prm: Params, keys: Keys, a: np.ndarray, b: np.ndarray, level: int) -> np.ndarray:
    """Ciphertext product followed by relinearisation (no rescale)."""
    return relinearize(prm, keys, tensor(prm, a, b, level), level)


def add_plain(prm: Params, ct: np.ndarray, pt: np.ndarray, level: int) -> np.ndarray:
    """(c0 + pt, c1): pt is [level+1][N] residues in evaluation form."""
    Q = prm.Q(level)
    return np.stack([add(ct[0], pt, Q), ct[1].copy()])


def add_ct(prm: Params, a: np.ndarray, b: np.ndarray, level: int) -> np.ndarray:
    Q = prm.Q(level)
    return np.stack([add(a[0], b[0], Q), add(a[1], b[1], Q)])


def mod_drop(ct: np.ndarray, level: int) -> np.ndarray:
    """Drop the primes above q_level (the same ciphertext modulo Q_level)."""
    return np.ascontiguousarray(ct[:, : level + 1])


def plain_residues(prm: Params, z, scale: float, level: int) -> np.ndarray:
    """Slot vector z encoded at `scale`, as residues over Q_level in evaluation form."""
    Q = prm.Q(level)
    return ntt(from_signed(encode(z, scale, prm), Q), Q, prm)


# ------------------------------------------------------------------ cleartext model (Sec. IV)

def num_digits(k: int, p: int) -> int:
    """l = ceil(log_p k), computed exactly: the least l with p^l >= k (>= 1)."""
    l = 1
    while p ** l < k:
        l += 1
    return l


def digits_of(i: int, p: int, l: int) -> List[int]:
    """Little-endian base-p digits: i_j = floor(i / p^j) mod p."""
    return [(i // p ** j) % p for j in range(l)]


def ohe(i: int, k: int) -> np.ndarray:
    e = np.zeros(k)
    e[i] = 1.0
    return e


@dataclass
class TableSpec:
    """One embedding table: either compressed (l tables C_j of p x d) or
    uncompressed (E of k x d)."""
    rows: int
    d: int
    base: Optional[int] = None            # None = uncompressed
    C: Optional[List[np.ndarray]] = None  # compressed tables
    E: Optional[np.ndarray] = None        # uncompressed table

    @property
    def width(self) -> int:
        return self.base * len(self.C) if self.base is not None else self.rows

    def block(self) -> np.ndarray:
        """W = [C_0; ...; C_{l-1}]^T (d x p l), or E^T (d x k)."""
        if self.base is not None:
            return np.concatenate(self.C, axis=0).T
        return self.E.T

    def selector(self, i: int) -> np.ndarray:
        if self.base is not None:
            ds = digits_of(i, self.base, len(self.C))
            return np.concatenate([ohe(x, self.base) for x in ds])
        return ohe(i, self.rows)

    def lookup(self, i: int) -> np.ndarray:
        """Cleartext result: sum_j C_j[i_j], or E[i]."""
        if self.base is not None:
            ds = digits_of(i, self.base, len(self.C))
            return sum(self.C[j][x] for j, x in enumerate(ds))
        return self.E[i]


def block_diag(blocks: Sequence[np.ndarray]) -> np.ndarray:
    rows = sum(b.shape[0] for b in blocks)
    cols = sum(b.shape[1] for b in blocks)
    M = np.zeros((rows, cols))
    r = c = 0
    for b in blocks:
        M[r:r + b.shape[0], c:c + b.shape[1]] = b
        r += b.shape[0]
        c += b.shape[1]
    return M


def pack_tables(tables: Sequence[TableSpec]) -> np.ndarray:
    return block_diag([t.block() for t in tables])


def pack_selector(tables: Sequence[TableSpec], idx: Sequence[int]) -> np.ndarray:
    return np.concatenate([t.selector(i) for t, i in zip(tables, idx)])


def next_pow2(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def hybrid_diagonals(M: np.ndarray, n: int, sign: int = 1) -> Tuple[int, np.ndarray]:
    """u_k[j] = M'[j mod m][(j + sign k) mod n] for k < m, M' = M zero-padded to
    m x n, m = next_pow2(rows).  sum_k u_k * rot(x, sign k), folded over the
    m-periodic copies, equals M x in slots [0, rows)."""
    rows, cols = M.shape
    assert cols <= n and sign in (1, -1)
    m = next_pow2(rows)
    Mp = np.zeros((m, n))
    Mp[:rows, :cols] = M
    j = np.arange(n)
    U = np.stack([Mp[j % m, (j + sign * k) % n] for k in range(m)])
    return m, U


def fold_span(M: np.ndarray, n: int, sign: int) -> int:
    """Slots the fold must cover.  With sign -1, u_k[j] is non-zero only for
    j - k in [0, cols), so every partial sum lies in [0, cols + m - 1) and the
    fold can stop at the next power of two above that; with sign +1 the
    partial sums wrap around and the fold covers all n slots."""
    rows, cols = M.shape
    m = next_pow2(rows)
    if sign == 1:
        return n
    return min(n, next_pow2(cols + m - 1))


def rot(x: np.ndarray, k: int) -> np.ndarray:
    """Cleartext rotation left by k: rot(x, k)[j] = x[(j + k) mod n]."""
    return np.roll(x, -k)


def fold_stages(n: int, m: int, radix: int) -> List[Tuple[int, int]]:
    """Fold schedule from n slots down to period m: each stage (s, r) replaces
    z by sum_{t<r} rot(z, t s)."""
    stages = []
    span = n
    while span > m:
        r = min(radix, span // m)
        s = span // r
        stages.append((s, r))
        span = s
    return stages


@dataclass
class Plan:
    """BSGS matvec schedule over the hybrid diagonals of one packed matrix.
    sign = +1 rotates by +b and +n1 g, sign = -1 by -b and -n1 g; the fold
    runs from `span` slots down to period m."""
    m: int
    n1: int
    n2: int
    radix: int
    level: int
    rows: int
    coeffs: Dict[Tuple[int, int], np.ndarray]   # (g, b) -> int64 [N], encoded at scale q_level
    stages: List[Tuple[int, int]] = field(default_factory=list)
    sign: int = 1
    span: int = 0

    def baby_steps(self) -> List[int]:
        return sorted({b for (_, b) in self.coeffs})

    def giant_steps(self) -> List[int]:
        return sorted({g for (g, _) in self.coeffs})

    def rotation_steps(self) -> List[int]:
        st = set(self.sign * b for b in self.baby_steps() if b != 0)
        st |= {self.sign * self.n1 * g for g in self.giant_steps() if g != 0}
        for s, r in self.stages:
            st |= {t * s for t in range(1, r)}
        return sorted(st)


def bsgs_plan_values(M: np.ndarray, n: int, n1: int, sign: int = 1) -> Tuple[int, int, Dict[Tuple[int, int], np.ndarray]]:
    """Pre-rotated diagonals v_{g,b} = rot(u_{n1 g + b}, -sign n1 g) for every
    non-zero hybrid diagonal, so that
    sum_g rot(sum_b v_{g,b} rot(x, sign b), sign n1 g) = sum_k u_k rot(x, sign k)."""
    m, U = hybrid_diagonals(M, n, sign)
    n2 = -(-m // n1)
    vals = {}
    for k in range(m):
        if not np.any(U[k]):
            continue
        g, b = divmod(k, n1)
        vals[(g, b)] = rot(U[k], -sign * n1 * g)
    return m, n2, vals


def make_plan(prm: Params, M: np.ndarray, level: int, n1: int, radix: int = 2, sign: int = 1,
              scale: Optional[float] = None) -> Plan:
    """Plaintext diagonals encoded at `scale` (default q_level, which keeps the
    product at the input's scale after the rescale)."""
    m, n2, vals = bsgs_plan_values(M, prm.n, n1, sign)
    scale = prm.q[level] if scale is None else scale
    coeffs = {gb: encode(v, scale, prm) for gb, v in vals.items()}
    span = fold_span(M, prm.n, sign)
    return Plan(m=m, n1=n1, n2=n2, radix=radix, level=level, rows=M.shape[0], coeffs=coeffs,
                stages=fold_stages(span, m, radix), sign=sign, span=span)


def cleartext_bsgs(M: np.ndarray, x: np.ndarray, n: int, n1: int, radix: int, sign: int = 1) -> np.ndarray:
    """fp64 replay of the schedule: the BSGS sum followed by the fold."""
    m, n2, vals = bsgs_plan_values(M, n, n1, sign)
    xs = np.zeros(n)
    xs[: len(x)] = x
    z = np.zeros(n)
    for g in range(n2):
        inner = np.zeros(n)
        for b in range(n1):
            if (g, b) in vals:
                inner += vals[(g, b)] * rot(xs, sign * b)
        z += rot(inner, sign * n1 * g)
    for s, r in fold_stages(fold_span(M, n, sign), m, radix):
        z = sum(rot(z, t * s) for t in range(r))
    return z


# ------------------------------------------------------------------ encrypted matvec / lookup

def plan_residues(prm: Params, plan: Plan) -> Dict[Tuple[int, int], np.ndarray]:
    """Plaintext diagonals reduced over PQ_level and taken to evaluation form."""
    PQ = prm.PQ(plan.level)
    return {gb: ntt(from_signed(c, PQ), PQ, prm) for gb, c in plan.coeffs.items()}


def matvec(prm: Params, keys: Keys, plan: Plan, ct: np.ndarray,
           pts: Optional[Dict[Tuple[int, int], np.ndarray]] = None) -> np.ndarray:
    """Double-hoisted BSGS plaintext-matrix x ciphertext product (no rescale).
      1. ModUp(c1) once; R_0 = (P c0, P c1); R_b = hoisted rotation by sign b in PQ.
      2. X_g = sum_b pt_{g,b} * R_b over PQ; x_g = ModDown(X_g).
      3. acc = P x_0 + sum_{g>=1} [rotation of x_g by sign n1 g, kept in PQ];
         z = ModDown(acc)  (z = x_0 when there is one giant step).
      4. Fold: per stage (s, r), z = ModDown(P z + sum_{t=1}^{r-1} rot_PQ(z, t s))."""
    lv = plan.level
    PQ = prm.PQ(lv)
    if pts is None:
        pts = plan_residues(prm, plan)
    babies = plan.baby_steps()
    d = modup(prm, ct[1], lv)
    R = {}
    for b in babies:
        if b == 0:
            R[0] = lift_P(prm, ct, lv)
        else:
            g = galois_for_step(plan.sign * b, prm)
            R[b] = key_inner_product(prm, d, ct[0], lv, keys.swk[g], g)
    xs = {}
    for g in plan.giant_steps():
        X = np.zeros((2, len(PQ), prm.N), dtype=np.uint64)
        for b in babies:
            if (g, b) not in pts:
                continue
            for c in range(2):
                X[c] = add(X[c], mul(pts[(g, b)], R[b][c], PQ), PQ)
        xs[g] = moddown(prm, X, lv)
    giants = plan.giant_steps()
    if giants == [0]:
        z = xs[0]
    else:
        acc = np.zeros((2, len(PQ), prm.N), dtype=np.uint64)
        for g in giants:
            if g == 0:
                Y = lift_P(prm, xs[0], lv)
            else:
                gal = galois_for_step(plan.sign * plan.n1 * g, prm)
                dg = modup(prm, xs[g][1], lv)
                Y = key_inner_product(prm, dg, xs[g][0], lv, keys.swk[gal], gal)
            for c in range(2):
                acc[c] = add(acc[c], Y[c], PQ)
        z = moddown(prm, acc, lv)
    for s, r in plan.stages:
        dz = modup(prm, z[1], lv)
        acc = lift_P(prm, z, lv)
        for t in range(1, r):
            gal = galois_for_step(t * s, prm)
            Y = key_inner_product(prm, dz, z[0], lv, keys.swk[gal], gal)
            for c in range(2):
                acc[c] = add(acc[c], Y[c], PQ)
        z = moddown(prm, acc, lv)
    return z


def lookup(prm: Params, keys: Keys, plan: Plan, ct: np.ndarray, pts=None) -> np.ndarray:
    """Encrypted lookup: matvec followed by one rescale (consumes one level)."""
    return rescale(prm, matvec(prm, keys, plan, ct, pts), plan.level)


# ------------------------------------------------------------------ small DLRM (Sec. II-B, Sec. V-C)

@dataclass
class SmallDLRM:
    """Dense features and uncompressed embedding tables (Sec. II-B): a bottom
    MLP on the dense features, the embedding rows of every table, and a top MLP
    on the concatenation [embedding rows; bottom output].  Every hidden layer is
    followed by the square activation (the degree-2 polynomial the paper uses
    for its small model, Sec. V-C); the last top layer gives the logit."""
    tables: List[TableSpec]
    bottom: List[Tuple[np.ndarray, np.ndarray]]     # (W, b) per layer
    top: List[Tuple[np.ndarray, np.ndarray]]
    n_dense: int

    @property
    def emb_dim(self) -> int:
        return sum(t.d for t in self.tables)

    def input_slots(self, dense: np.ndarray, idx: Sequence[int]) -> np.ndarray:
        """Packed input: dense features in slots [0, n_dense), then the one-hots."""
        return np.concatenate([np.asarray(dense, dtype=float), pack_selector(self.tables, idx)])


def dlrm_cleartext(model: SmallDLRM, dense: np.ndarray, idx: Sequence[int]) -> np.ndarray:
    """fp64 forward pass: the reference the decrypted logit is compared with."""
    h = np.asarray(dense, dtype=float)
    for W, b in model.bottom:
        h = (W @ h + b) ** 2
    e = np.concatenate([t.lookup(i) for t, i in zip(model.tables, idx)])
    z = np.concatenate([e, h])
    for k, (W, b) in enumerate(model.top):
        z = W @ z + b
        if k + 1 < len(model.top):
            z = z ** 2
    return z


@dataclass
class DLRMLayout:
    """The model's layers as matrices over slot vectors.  The embedding matrix
    reads the one-hot slots and writes rows [0, E); the last bottom layer is
    padded to write rows [E, E+H); both have E+H rows, so both products are
    exact (zero) in every slot of [0, next_pow2(E+H)) they do not write and
    their sum is the concatenation."""
    emb: np.ndarray
    bottom: List[np.ndarray]
    bias_bottom: List[np.ndarray]
    top: List[np.ndarray]
    bias_top: List[np.ndarray]


def dlrm_layout(model: SmallDLRM) -> DLRMLayout:
    E = model.emb_dim
    H = model.bottom[-1][0].shape[0]
    width = model.n_dense + sum(t.width for t in model.tables)
    emb = np.zeros((E + H, width))
    emb[:E, model.n_dense:] = pack_tables(model.tables)
    bottom, bb = [], []
    for k, (W, b) in enumerate(model.bottom):
        if k + 1 < len(model.bottom):
            bottom.append(np.array(W, dtype=float))
            bb.append(np.array(b, dtype=float))
        else:
            M = np.zeros((E + H, W.shape[1]))
            M[E:] = W
            bv = np.zeros(E + H)
            bv[E:] = b
            bottom.append(M)
            bb.append(bv)
    return DLRMLayout(emb=emb, bottom=bottom, bias_bottom=bb,
                      top=[np.array(W, dtype=float) for W, _ in model.top],
                      bias_top=[np.array(b, dtype=float) for _, b in model.top])


@dataclass
class DLRMSchedule:
    """Plans, bias plaintexts and levels of the encrypted forward pass.  Every
    matvec's plaintexts are encoded at scale S_out q_l / S_in, so its output
    after the rescale is at S_out (Delta, except the embedding product, whose
    output is put at the scale of the bottom output so the two can be added).
    A square multiplies the scale S into S^2 / q_l."""
    level0: int
    emb: Plan
    bottom: List[Plan]
    bias_bottom: List[np.ndarray]
    top: List[Plan]
    bias_top: List[np.ndarray]
    concat_level: int
    concat_scale: float
    out_level: int

    def plans(self) -> List[Plan]:
        return [self.emb] + self.bottom + self.top

    def rotation_steps(self) -> List[int]:
        return sorted({k for p in self.plans() for k in p.rotation_steps()})


def dlrm_schedule(prm: Params, model: SmallDLRM, level0: int, n1: int = 16, radix: int = 8,
                  sign: int = -1) -> DLRMSchedule:
    lay = dlrm_layout(model)
    delta = float(prm.delta)
    lv, S = level0, delta

    def plan_for(M, level, s_in, s_out):
        m = next_pow2(M.shape[0])
        return make_plan(prm, M, level, min(n1, m), radix, sign, scale=s_out * prm.q[level] / s_in)

    bottom, bb = [], []
    for M, bv in zip(lay.bottom, lay.bias_bottom):
        bottom.append(plan_for(M, lv, S, delta))
        lv -= 1
        S = delta
        bb.append(plain_residues(prm, bv, S, lv))
        S = S * S / prm.q[lv]          # square, then rescale by q_lv
        lv -= 1
    concat_level, concat_scale = lv, S
    emb = plan_for(lay.emb, level0, delta, concat_scale)
    top, bt = [], []
    for k, (M, bv) in enumerate(zip(lay.top, lay.bias_top)):
        top.append(plan_for(M, lv, S, delta))
        lv -= 1
        S = delta
        bt.append(plain_residues(prm, bv, S, lv))
        if k + 1 < len(lay.top):
            S = S * S / prm.q[lv]
            lv -= 1
    return DLRMSchedule(level0=level0, emb=emb, bottom=bottom, bias_bottom=bb, top=top, bias_top=bt,
                        concat_level=concat_level, concat_scale=concat_scale, out_level=lv)


def dlrm_forward(prm: Params, keys: Keys, sch: DLRMSchedule, ct: np.ndarray) -> np.ndarray:
    """Encrypted forward pass of one packed input ciphertext at sch.level0;
    returns the logit ciphertext at sch.out_level (slot 0, scale Delta)."""
    x = ct
    for plan, b in zip(sch.bottom, sch.bias_bottom):
        lv = plan.level - 1
        x = add_plain(prm, lookup(prm, keys, plan, x), b, lv)
        x = rescale(prm, mul_relin(prm, keys, x, x, lv), lv)
    e = mod_drop(lookup(prm, keys, sch.emb, ct), sch.concat_level)
    z = add_ct(prm, e, x, sch.concat_level)
    for k, (plan, b) in enumerate(zip(sch.top, sch.bias_top)):
        lv = plan.level - 1
        z = add_plain(prm, lookup(prm, keys, plan, z), b, lv)
        if k + 1 < len(sch.top):
            z = rescale(prm, mul_relin(prm, keys, z, z, lv), lv)
    return z


# ------------------------------------------------------------------ selectors over several ciphertexts (Sec. III-C)

def split_columns(M: np.ndarray, n: int) -> List[np.ndarray]:
    """Column blocks of at most n columns: block c multiplies ciphertext c,
    which holds selector slots [c n, (c+1) n)."""
    return [M[:, c:c + n] for c in range(0, M.shape[1], n)]


def split_selector(s: np.ndarray, n: int) -> List[np.ndarray]:
    return [s[c:c + n] for c in range(0, len(s), n)]


def make_multi_plan(prm: Params, M: np.ndarray, level: int, n1: int, radix: int = 2, sign: int = 1) -> List[Plan]:
    """One plan per column block, all with the same m, n1, n2 and fold (the
    widest block's span), so their products can be summed before the fold."""
    blocks = split_columns(M, prm.n)
    span = max(fold_span(B, prm.n, sign) for B in blocks)
    plans = []
    for B in blocks:
        p = make_plan(prm, B, level, n1, radix, sign)
        p.span = span
        p.stages = fold_stages(span, p.m, radix)
        plans.append(p)
    return plans


def matvec_multi(prm: Params, keys: Keys, plans: List[Plan], cts: List[np.ndarray]) -> np.ndarray:
    """sum_c M_c s_c for one ciphertext per column block: every block's
    baby-step products are summed into the same giant-step accumulators
    X_g = sum_c sum_b pt_{c,g,b} * R_{c,b} over PQ, then ModDown, the giant
    steps and the fold run once (no rescale)."""
    p0 = plans[0]
    lv = p0.level
    PQ = prm.PQ(lv)
    X = {}
    for plan, ct in zip(plans, cts):
        pts = plan_residues(prm, plan)
        d = modup(prm, ct[1], lv)
        for b in plan.baby_steps():
            if b == 0:
                R = lift_P(prm, ct, lv)
            else:
                gal = galois_for_step(plan.sign * b, prm)
                R = key_inner_product(prm, d, ct[0], lv, keys.swk[gal], gal)
            for g in plan.giant_steps():
                if (g, b) not in pts:
                    continue
                acc = X.setdefault(g, np.zeros((2, len(PQ), prm.N), dtype=np.uint64))
                for c in range(2):
                    acc[c] = add(acc[c], mul(pts[(g, b)], R[c], PQ), PQ)
    giants = sorted(X)
    xs = {g: moddown(prm, X[g], lv) for g in giants}
    if giants == [0]:
        z = xs[0]
    else:
        acc = np.zeros((2, len(PQ), prm.N), dtype=np.uint64)
        for g in giants:
            if g == 0:
                Y = lift_P(prm, xs[0], lv)
            else:
                gal = galois_for_step(p0.sign * p0.n1 * g, prm)
                Y = key_inner_product(prm, modup(prm, xs[g][1], lv), xs[g][0], lv, keys.swk[gal], gal)
            for c in range(2):
                acc[c] = add(acc[c], Y[c], PQ)
        z = moddown(prm, acc, lv)
    for s, r in p0.stages:
        dz = modup(prm, z[1], lv)
        acc = lift_P(prm, z, lv)
        for t in range(1, r):
            gal = galois_for_step(t * s, prm)
            Y = key_inner_product(prm, dz, z[0], lv, keys.swk[gal], gal)
            for c in range(2):
                acc[c] = add(acc[c], Y[c], PQ)
        z = moddown(prm, acc, lv)
    return z


def lookup_multi(prm: Params, keys: Keys, plans: List[Plan], cts: List[np.ndarray]) -> np.ndarray:
    return rescale(prm, matvec_multi(prm, keys, plans, cts), plans[0].level)
