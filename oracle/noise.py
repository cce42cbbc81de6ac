"""Additive white Gaussian noise at a chosen signal-to-noise ratio (test infrastructure).

Section 3.2 allows Gaussian white noise of a given SNR to be added to the simulated
signal. Readings where the paper is silent:
  * SNR is the ratio of the mean signal power per complex sample of one echo cube,
    mean |H|^2 over its O x N x M elements, to the noise power per complex sample
    sigma^2; each of the real and imaginary parts gets variance sigma^2 / 2.
  * The noise is added to the echo H (the beat signal conj(H) then carries its
    conjugate, which has the same distribution).
  * Random numbers: the counter-based generator Philox4x32 with 10 rounds (Salmon,
    Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).
    Element i (flat index in [O][N][M] order) of cube c uses counter
    (i mod 2^32, i div 2^32, c, 0) and key (seed mod 2^32, seed div 2^32); the first
    two output words give uniforms u = (x + 1/2) 2^-32 in (0, 1), and the Box-Muller
    transform r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2) gives two independent
    standard normals.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57  # round multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85  # key increments (Weyl sequence)
_MASK = 0xFFFFFFFF


def philox4x32(counter, key, rounds: int = 10):
    """Philox4x32-R on arrays: counter = (c0, c1, c2, c3), key = (k0, k1), each an
    integer array (uint64 holding 32-bit values). Returns four uint64 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in counter)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & _MASK for k in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = np.uint64(_M0) * c0  # exact: a 64-bit product of two 32-bit values
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
    return c0, c1, c2, c3


def standard_normal_pairs(n: int, stream: int, seed: int):
    """(re, im) standard normals for elements 0 .. n-1 of stream (cube) `stream`."""
    i = np.arange(n, dtype=np.uint64)
    x0, x1, _, _ = philox4x32((i & _MASK, i >> np.uint64(32),
                               np.full(n, stream, np.uint64), np.zeros(n, np.uint64)),
                              (np.uint64(seed & _MASK), np.uint64((seed >> 32) & _MASK)))
    u1 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def add_awgn(H: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """H[..., O, N, M] (leading axes = cubes) plus complex white Gaussian noise with
    mean |H|^2 / sigma^2 = 10^(snr_db / 10) per cube."""
    H = np.asarray(H, dtype=np.complex128)
    cubes = H.reshape((-1,) + H.shape[-3:])
    out = np.empty_like(cubes)
    for c in range(cubes.shape[0]):
        x = cubes[c]
        sigma2 = np.mean(np.abs(x) ** 2) / 10.0 ** (snr_db / 10.0)
        re, im = standard_normal_pairs(x.size, c, seed)
        s = np.sqrt(0.5 * sigma2)
        out[c] = x + (s * (re + 1j * im)).reshape(x.shape)
    return out.reshape(H.shape)
