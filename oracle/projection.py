"""Projection P onto the Gaussian feasible set (test infrastructure only).

Paper section 2.3.1: the projection is a z-score normalisation (subtract the
mean, divide by the standard deviation) followed by resetting every value
whose magnitude exceeds s_th = 10 to a fresh N(0, 1) draw.  Readings: the
standard deviation is the population one (ddof = 0) computed after removing
the mean; there is no renormalisation after the resets; the reset draws come
from the counter-based generator (stream RESET, sub = line-search trial,
event = iteration, counter index = flat element index).
"""
import numpy as np

from . import philox

__all__ = ["project"]


def project(s, s_th, seed, event, trial):
    """Return (P(s), number of resets) for a flat or shaped array s."""
    s = np.asarray(s, dtype=np.float64)
    flat = s.reshape(-1)
    n = flat.size
    mean = np.sum(flat) / n
    dev = flat - mean
    std = np.sqrt(np.sum(dev * dev) / n)
    with np.errstate(invalid="ignore", divide="ignore"):
        z = dev / std  # a constant input has no z-score: NaN, rejected by the line search
    bad = np.nonzero(np.abs(z) > s_th)[0]
    out = z.copy()
    if bad.size:
        out[bad] = philox.normal(bad.astype(np.uint64), trial, philox.STREAM_RESET,
                                 event, seed)
    return out.reshape(s.shape), int(bad.size)
