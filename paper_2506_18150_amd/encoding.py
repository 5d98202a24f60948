"""CKKS encoding and decoding (Appendix A "Encoding").

Slot j of a plaintext m(X) in Z[X]/(X^N+1) is m(zeta^(5^j mod 2N)),
zeta = exp(i pi / N).  Encoding inverts the canonical embedding, scales by
Delta and rounds each coefficient half away from zero.  Both directions use a
length-N FFT: with e = 2t + 1 odd, zeta^(e c) = zeta^c * omega^(t c) for
omega = zeta^2, so the N odd-power evaluations are a twisted length-N DFT.
"""
from __future__ import annotations

import numpy as np

_cache = {}


def _tables(N: int):
    if N not in _cache:
        n = N // 2
        e = np.empty(n, dtype=np.int64)
        x = 1
        for j in range(n):
            e[j] = x
            x = x * 5 % (2 * N)
        t_pos = (e - 1) // 2                  # t of zeta^(5^j)
        t_neg = (2 * N - e - 1) // 2          # t of zeta^(-5^j)
        twist = np.exp(1j * np.pi * np.arange(N) / N)   # zeta^c
        _cache[N] = (t_pos, t_neg, twist)
    return _cache[N]


def encode(z, scale: float, N: int) -> np.ndarray:
    """Real or complex slot vector (zero-padded to N/2) -> int64 coefficients."""
    t_pos, t_neg, twist = _tables(N)
    v = np.zeros(N // 2, dtype=np.complex128)
    zz = np.asarray(z, dtype=np.complex128).ravel()
    v[: len(zz)] = zz
    Z = np.zeros(N, dtype=np.complex128)
    Z[t_pos] = scale * v
    Z[t_neg] = np.conj(scale * v)
    m = (np.fft.fft(Z) / twist).real / N
    return (np.sign(m) * np.floor(np.abs(m) + 0.5)).astype(np.int64)


def decode(coeffs, scale: float, N: int) -> np.ndarray:
    t_pos, _, twist = _tables(N)
    m = np.asarray(coeffs, dtype=np.float64)
    Z = np.fft.ifft(m * twist) * N
    return Z[t_pos] / scale
