"""Peano-Hilbert keys for integer lattice points.

Skilling (2004), "Programming the Hilbert curve" (AIP Conf. Proc. 707, 381):
the "axes to transpose" form of the curve, followed by interleaving the
transposed bits into one integer key.  Vectorised over numpy arrays of
lattice indices.  Pure integer arithmetic, so the order is exact.
"""
from __future__ import annotations

import numpy as np


def _axes_to_transpose(X: list[np.ndarray], bits: int) -> list[np.ndarray]:
    n = len(X)
    X = [x.astype(np.int64).copy() for x in X]
    top = 1 << (bits - 1)
    # Undo the excess work of the inverse transform, from the top bit down.
    q = top
    while q > 1:
        p = q - 1
        for i in range(n):
            hit = (X[i] & q) != 0
            # inversion of the low bits of X[0] where bit q of X[i] is set
            X[0] = np.where(hit, X[0] ^ p, X[0])
            # exchange of the low bits of X[0] and X[i] elsewhere
            t = (X[0] ^ X[i]) & p
            t = np.where(hit, 0, t)
            X[0] = X[0] ^ t
            X[i] = X[i] ^ t
        q >>= 1
    # Gray encode.
    for i in range(1, n):
        X[i] = X[i] ^ X[i - 1]
    t = np.zeros_like(X[0])
    q = top
    while q > 1:
        t = np.where((X[n - 1] & q) != 0, t ^ (q - 1), t)
        q >>= 1
    return [x ^ t for x in X]


def hilbert_key(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray, bits: int) -> np.ndarray:
    """Hilbert index of lattice points (ix, iy, iz), each in [0, 2**bits)."""
    ix, iy, iz = (np.asarray(a, dtype=np.int64) for a in (ix, iy, iz))
    lim = 1 << bits
    for a in (ix, iy, iz):
        if a.size and (a.min() < 0 or a.max() >= lim):
            raise ValueError("lattice index outside [0, 2**bits)")
    X = _axes_to_transpose([ix, iy, iz], bits)
    key = np.zeros_like(ix)
    for b in range(bits - 1, -1, -1):
        for i in range(3):
            key = (key << 1) | ((X[i] >> b) & 1)
    return key


def bits_for(n: int) -> int:
    """Smallest number of bits b with 2**b >= n (at least 1)."""
    b = 1
    while (1 << b) < n:
        b += 1
    return b
