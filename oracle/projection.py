"""Projection P onto the Gaussian feasible set (test infrastructure only).

Paper section 2.3.1: the projection is a z-score normalisation (subtract the
mean, divide by the standard deviation) followed by resetting every value
whose magnitude exceeds s_th = 10 to a fresh N(0, 1) draw, so that the
parameters stay in the set {mean 0, std 1, no extreme values}.  Readings:
the standard deviation is the population one (ddof = 0) computed after
removing the mean; resets change the moments, so the two steps repeat until
a pass resets nothing, which makes the output lie in the set and P
idempotent on it (after MAX_PASSES passes with resets, a last z-score keeps
the moments exact); reset draws come from the counter-based
generator (stream RESET, sub = trial + 1024 pass, event = iteration, counter
index = flat element index).
"""
import numpy as np

from . import philox

__all__ = ["project", "MAX_PASSES"]

MAX_PASSES = 32


def project(s, s_th, seed, event, trial):
    """Return (P(s), number of resets over all passes)."""
    s = np.asarray(s, dtype=np.float64)
    x = s.reshape(-1)
    n = x.size
    total = 0
    for pas in range(MAX_PASSES):
        mean = np.sum(x) / n
        dev = x - mean
        std = np.sqrt(np.sum(dev * dev) / n)
        with np.errstate(invalid="ignore", divide="ignore"):
            z = dev / std  # a constant input has no z-score: NaN, rejected by the line search
        bad = np.nonzero(np.abs(z) > s_th)[0]
        if bad.size == 0:
            return z.reshape(s.shape), total
        z[bad] = philox.normal(bad.astype(np.uint64), trial + 1024 * pas,
                               philox.STREAM_RESET, event, seed)
        total += int(bad.size)
        x = z
    mean = np.sum(x) / n
    dev = x - mean
    return (dev / np.sqrt(np.sum(dev * dev) / n)).reshape(s.shape), total
