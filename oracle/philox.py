"""Philox4x64-10 counter-based generator and Gaussian variates (oracle).
TEST INFRASTRUCTURE ONLY.

The constrained realization draws white-noise vectors omega_1 (per band
pixel) and omega_2 (per component coefficient) (Sect. 2.3).  The paper is
silent on the generator; both sides implement Philox4x64 with 10 rounds
from its published definition (Salmon, Moraes, Dror, Shaw, SC'11), so the
raw 64-bit words match bit for bit:

    round:  (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2   (128-bit products)
            c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
    key schedule between rounds: k0 += W0, k1 += W1.

Variate i of stream (seed, stream, rhs) is word i % 4 of the block with
counter (i // 4, rhs, 0, 0) and key (seed, stream).  Words become uniforms
u = ((w >> 11) + 0.5) 2^-53 in (0, 1), and consecutive pairs (u0, u1),
(u2, u3) become two normals each by Box-Muller:
    n0 = sqrt(-2 ln u0) cos(2 pi u1),  n1 = sqrt(-2 ln u0) sin(2 pi u1).
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 on arrays of counters; returns four uint64 arrays."""
    with np.errstate(over="ignore"):
        c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for rnd in range(10):
            if rnd:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(M0, c[0])
            hi1, lo1 = _mulhilo(M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def raw_words(seed, stream, rhs, n):
    """First n 64-bit words of the stream (seed, stream, rhs)."""
    nblk = (n + 3) // 4
    blk = np.arange(nblk, dtype=np.uint64)
    zero = np.zeros(nblk, dtype=np.uint64)
    w = philox4x64_10(blk, zero + np.uint64(rhs), zero, zero,
                      np.uint64(seed), np.uint64(stream))
    return np.stack(w, axis=1).reshape(-1)[:n]


def uniforms(words):
    """64-bit words -> uniforms ((w >> 11) + 0.5) 2^-53, strictly inside (0, 1)."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def box_muller(u):
    """Uniforms [nblk, 4] -> normals [nblk, 4]: pairs (u0, u1) and (u2, u3);
    the first of a pair sets the radius sqrt(-2 ln u), the second the angle
    2 pi u, and the pair's outputs are radius * (cos, sin) of that angle."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    for a, b in ((0, 1), (2, 3)):
        rad = np.sqrt(-2.0 * np.log(u[:, a]))
        ang = 2.0 * np.pi * u[:, b]
        out[:, a] = rad * np.cos(ang)
        out[:, b] = rad * np.sin(ang)
    return out


def normals(seed, stream, rhs, n):
    """n standard normal variates of stream (seed, stream, rhs)."""
    nblk = (n + 3) // 4
    w = raw_words(seed, stream, rhs, 4 * nblk)
    return box_muller(uniforms(w).reshape(nblk, 4)).reshape(-1)[:n]


# Stream identifiers used by the constrained-realization right-hand side.
STREAM_OMEGA1_BASE = 0x100  # + band index
STREAM_OMEGA2 = 0x200
