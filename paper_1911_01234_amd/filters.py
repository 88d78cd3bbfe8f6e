"""Orthonormal wavelet filters: inputs that choose Psi (Algorithm 1 needs only some
orthogonal wavelet transform).

This module builds the filter, never the reconstruction; it holds none of the method's
arithmetic and is shared by the tests, the benchmark and the CPU oracle's callers.

A filter is the lowpass h[0..L) of a two-channel orthonormal filter bank: sum h = sqrt 2,
sum_t h[t] h[t + 2j] = delta_j.  The highpass is g[t] = (-1)^t h[L - 1 - t].  Haar is
h = (1, 1) / sqrt 2.

Daubechies' compactly supported wavelets with N vanishing moments (length 2N) follow
from the spectral factorisation of Daubechies (1988): |H(w)|^2 = 2 cos^(2N)(w/2)
P(sin^2(w/2)) with P(y) = sum_{k<N} C(N-1+k, k) y^k.  Each root y_k of P gives the pair
z, 1/z of z^2 - (2 - 4 y_k) z + 1 = 0 (from y = (2 - z - 1/z) / 4); keeping the root
inside the unit circle of every pair gives the minimum-phase filter
H(z) = c (1 + z)^N prod_k (z - z_k), scaled so that sum h = sqrt 2.
"""
from __future__ import annotations

from math import comb

import numpy as np


def haar() -> np.ndarray:
    return np.array([1.0, 1.0]) / np.sqrt(2.0)


def daubechies(n_moments: int) -> np.ndarray:
    """Minimum-phase Daubechies lowpass filter with n_moments vanishing moments
    (length 2 n_moments), largest-magnitude taps first; daubechies(1) is Haar."""
    N = int(n_moments)
    if N < 1 or N > 10:
        raise ValueError("n_moments must be in 1..10")
    if N == 1:
        return haar()
    # P(y) = sum_{k<N} C(N-1+k, k) y^k; numpy.roots wants the highest power first
    P = [comb(N - 1 + k, k) for k in range(N)][::-1]
    zs = []
    for yk in np.roots(P):
        b = 2.0 - 4.0 * yk
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zs.append(z1 if abs(z1) < 1.0 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(N):
        poly = np.convolve(poly, [1.0, 1.0])
    for z in zs:
        poly = np.convolve(poly, [1.0, -z])
    h = np.real(poly)
    h = h * (np.sqrt(2.0) / h.sum())
    # orientation: the minimum-phase factor has its energy at the start
    if abs(h[0]) < abs(h[-1]):
        h = h[::-1].copy()
    return h


def highpass(h: np.ndarray) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    L = len(h)
    return np.array([(-1.0) ** t * h[L - 1 - t] for t in range(L)])


def orthonormality_error(h: np.ndarray) -> float:
    """max over j of |sum_t h[t] h[t + 2j] - delta_j| and |sum h - sqrt 2|."""
    h = np.asarray(h, dtype=np.float64)
    L = len(h)
    err = abs(h.sum() - np.sqrt(2.0))
    for j in range(0, (L + 1) // 2):
        acc = float(np.dot(h[: L - 2 * j], h[2 * j:]))
        err = max(err, abs(acc - (1.0 if j == 0 else 0.0)))
    return err
