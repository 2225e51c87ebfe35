"""Philox4x64-10 and the random draws of the method (test infrastructure only).

The projection's resets (paper section 2.3.1, step 2) and the target
realisations of rank-order matching (section 2.3.2, step 2) are random draws.
To make them reproducible across implementations each draw is a pure function
of a counter: Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11),
written here from its published definition.

Counter words (c0, c1, c2, c3) = (j, sub, stream, event), key = (seed, 0).
Uniforms: u = ((w >> 11) + 0.5) 2^-53 from output words w0, w1.
Normal: sqrt(-2 ln u0) cos(2 pi u1) (Box-Muller, first branch).
Rayleigh with E[a^2] = 1: sqrt(-ln u0).

Streams: 1 = projection reset (sub = line-search trial, event = iteration),
2 = real-space ROM targets, 3 = Fourier-space ROM targets (sub = k bin),
4 = fresh modes of the white-noise upsampling, 5 = Fourier-space ROM targets
of the real/imaginary-part reading (sub = k bin).
"""
import numpy as np

__all__ = ["philox4x64", "uniform_pair", "normal", "rayleigh",
           "STREAM_RESET", "STREAM_ROM_REAL", "STREAM_ROM_FOURIER", "STREAM_UPSAMPLE",
           "STREAM_ROM_FOURIER_REIM"]

STREAM_RESET = 1
STREAM_ROM_REAL = 2
STREAM_ROM_FOURIER = 3
STREAM_UPSAMPLE = 4
STREAM_ROM_FOURIER_REIM = 5

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays: (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll, lh, hl, hh = a_lo * b_lo, a_lo * b_hi, a_hi * b_lo, a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1=0, rounds=10):
    """Philox4x64-R block function on broadcastable uint64 counter words."""
    with np.errstate(over="ignore"):
        x = [np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3)]
        x = list(np.broadcast_arrays(*x))
        x = [v.copy() for v in x]
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for r in range(rounds):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, x[0])
            hi1, lo1 = _mulhilo(_M1, x[2])
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return x


def uniform_pair(j, sub, stream, event, seed):
    """Two uniforms in (0, 1) per counter, from output words 0 and 1."""
    w = philox4x64(np.asarray(j, dtype=np.uint64), sub, stream, event, seed)
    scale = 2.0 ** -53
    u0 = ((w[0] >> np.uint64(11)).astype(np.float64) + 0.5) * scale
    u1 = ((w[1] >> np.uint64(11)).astype(np.float64) + 0.5) * scale
    return u0, u1


def normal(j, sub, stream, event, seed):
    """Standard normal draw for each counter index j."""
    u0, u1 = uniform_pair(j, sub, stream, event, seed)
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def rayleigh(j, sub, stream, event, seed):
    """Rayleigh draw with unit mean square for each counter index j."""
    u0, _ = uniform_pair(j, sub, stream, event, seed)
    return np.sqrt(-np.log(u0))
