"""White-noise upsampling for the annealing schedule (test infrastructure only).

The paper runs the method at 4 Mpc/h first and starts the full-resolution run
from its result (section 3, the annealing strategy) without saying how the
white noise goes to the finer grid.  Reading: the field keeps its large-scale
modes and gets fresh small-scale ones.  For unit-variance white noise on N^3
cells the unnormalised DFT has E|s^(k)|^2 = N^3, and the same linear field
sampled on a finer grid of N_h^3 cells has s^_h(k) = (N_h / N_l)^{3/2}
s^_l(k) on the coarse grid's modes (whitening w(k) scales as dq^{-3/2}).  So
the fine field is a fresh N(0,1) field (Philox stream 4, counter (j, 0, 4,
event), j the fine lattice index) whose modes with every wave index inside
(-N_l/2, N_l/2) are replaced by those of the coarse field times
(N_h / N_l)^{3/2}; the coarse Nyquist modes are not carried over."""
import numpy as np

from . import fourier, philox

__all__ = ["STREAM_UPSAMPLE", "coarse_index", "upsample"]

STREAM_UPSAMPLE = 4


def coarse_index(n_low, n_high):
    """Fine-grid indices (full axes) and coarse-grid indices of the carried
    wave numbers -(n_low/2 - 1) .. n_low/2 - 1, in the same order."""
    h = n_low // 2
    fine = np.r_[0:h, n_high - h + 1:n_high]
    coarse = np.r_[0:h, n_low - h + 1:n_low]
    return fine, coarse


def upsample(s_low, n_high, seed, event):
    """Fine-grid white noise carrying the large-scale modes of s_low."""
    s_low = np.asarray(s_low, dtype=np.float64)
    n_low = s_low.shape[0]
    fresh = philox.normal(np.arange(n_high ** 3, dtype=np.uint64), 0, STREAM_UPSAMPLE, event,
                          seed).reshape(n_high, n_high, n_high)
    z = fourier.rfft3(fresh)
    zl = fourier.rfft3(s_low)
    fine, coarse = coarse_index(n_low, n_high)
    kz = np.arange(n_low // 2)
    z[np.ix_(fine, fine, kz)] = (n_high / n_low) ** 1.5 * zl[np.ix_(coarse, coarse, kz)]
    return fourier.irfft3(z, n_high)
