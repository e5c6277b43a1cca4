"""Seeded draw of the sampled sketches (fiber indices and Gaussian Omega)
from one counter-based stream, the definition the device-side draw of the
library reproduces (test infrastructure, like the rest of this package).

The sampling step of Algorithm 1 (Section 3.1) takes s_k columns of the mode-k
unfolding uniformly without repetition and a Gaussian Omega_k.  Here both come
from Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011), keyed by (seed, unit), where the unit is the
sketch's number (mode or tree node):

* indices: Floyd's algorithm (Bentley and Floyd, "Programming pearls: a
  sample of brilliance", CACM 1987).  Step i = 0..s-1 considers j = N - s + i,
  draws t uniform on [0, j] as the high 64 bits of w * (j + 1), w the first
  word of the block at counter (i, 0, 0, 0), and takes t if it is new, else
  j.  Every s-subset is equally likely (up to the (j+1)/2^64 granularity of
  the multiply-shift draw); the set is returned sorted.
* Omega[t][e] (t < s, e < ell): the block at counter (t ell + e, 1, 0, 0)
  gives u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1] and u2 = (w1 >> 11) 2^-53 in
  [0, 1); Box-Muller: sqrt(-2 ln u1) cos(2 pi u2).
"""
from __future__ import annotations

import numpy as np

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """(high, low) 64-bit words of the 128-bit product a * b, elementwise,
    from 32-bit halves in uint64 arithmetic."""
    b = b.astype(np.uint64)
    a_lo, a_hi = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (ll & _LO32) | ((mid & _LO32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x64 with 10 rounds: ctr (n, 4) uint64 counters, key (k0, k1);
    returns the (n, 4) uint64 output blocks."""
    c = [np.asarray(ctr[:, i], dtype=np.uint64).copy() for i in range(4)]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(_M0, c[0])
            hi1, lo1 = _mulhilo(_M1, c[2])
            c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return np.stack(c, axis=1)


def draw_indices(ncols: int, s: int, seed: int, unit: int) -> np.ndarray:
    """s distinct column indices of [0, ncols), uniform without repetition
    (Floyd's algorithm on the stream keyed by (seed, unit)), sorted."""
    if not 0 <= s <= ncols:
        raise ValueError("need 0 <= s <= ncols")
    ctr = np.zeros((s, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(s, dtype=np.uint64)
    w = philox4x64_10(ctr, (seed, unit))[:, 0]
    chosen = set()
    for i in range(s):
        j = ncols - s + i
        t = (int(w[i]) * (j + 1)) >> 64   # uniform on [0, j]
        chosen.add(j if t in chosen else t)
    return np.array(sorted(chosen), dtype=np.int64)


def draw_omega(s: int, ell: int, seed: int, unit: int) -> np.ndarray:
    """The s x ell Gaussian test matrix (Box-Muller on the stream keyed by
    (seed, unit)), FP64."""
    n = s * ell
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n, dtype=np.uint64)
    ctr[:, 1] = 1
    w = philox4x64_10(ctr, (seed, unit))
    return box_muller(w[:, 0], w[:, 1]).reshape(s, ell)


def box_muller(w0: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """One standard normal from two 64-bit words: u1 = ((w0 >> 11) + 1) 2^-53
    in (0, 1], u2 = (w1 >> 11) 2^-53 in [0, 1), sqrt(-2 ln u1) cos(2 pi u2)."""
    u1 = ((np.asarray(w0, dtype=np.uint64) >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (np.asarray(w1, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
