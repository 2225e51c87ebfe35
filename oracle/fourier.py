"""Fourier conventions and k-space multiplier operators (test infrastructure only).

Arrays are C ordered [x][y][z].  The forward transform is the unnormalised
real DFT over all three axes with the half spectrum along z (numpy ``rfftn``
layout, shape (N, N, N/2+1)); the inverse applies 1/N^3.  Index j on a full
axis has wavenumber kappa(j) = (2 pi / L) (j if j < N/2 else j - N); on the
half axis kappa = 2 pi j / L.  The derivative wavenumber kappa~ equals kappa
except that it is 0 at the Nyquist index j = N/2, which keeps every derivative
multiplier Hermitian (the paper is silent on Nyquist handling; this is the
reading used throughout).  |k|^2 uses the true kappa.

A multiplier operator Op_m[x] = irfftn(m(k) rfftn(x)) maps real fields to real
fields when m(-k) = conj(m(k)); its adjoint is Op_conj(m).  The operators used
by the forward model (paper section 2.2.1, items 1-2, and the particle-mesh
force) are

* whitening  w(k) = sqrt(P(k) / dq^3), w(0) = 0   (delta_L = Op_w[s]);
* gradient   g_j(k) = i kappa~_j / k^2            (Op_g[delta] = -grad lap^-1 delta);
* Hessian    h_ij(k) = kappa~_i kappa~_j / k^2    (Op_h[delta] = d_i d_j lap^-1 delta);

all zero at k = 0.
"""
import numpy as np
from scipy import fft as sfft

__all__ = ["rfft3", "irfft3", "dft_modes", "wave_axes", "kgrid", "multiplier", "apply",
           "apply_sum"]

_WORKERS = None


def _workers():
    global _WORKERS
    if _WORKERS is None:
        import os
        try:
            _WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
        except AttributeError:  # pragma: no cover
            _WORKERS = 1
    return _WORKERS


def rfft3(x):
    """Unnormalised forward real 3D DFT, half spectrum along the last axis."""
    return sfft.rfftn(np.asarray(x, dtype=np.float64), workers=_workers())


def irfft3(xk, n):
    """Inverse of rfft3 (applies 1/N^3); n is the real grid side."""
    return sfft.irfftn(xk, s=(n, n, n), workers=_workers())


def dft_modes(x, modes, rows=1 << 16):
    """Selected coefficients X(kx, ky, kz) of the unnormalised forward DFT,
    X(k) = sum_r x(r) exp(-2 pi i k.r / N), summed straight from that
    definition one axis at a time (z for all requested kz together, then y,
    then x).  Costs O(N^3 * #kz) instead of a whole transform, for spot checks
    of grids whose full FP64 transform is too large to hold.  Phases use the
    exact integer product k r mod N."""
    x = np.asarray(x)
    n = x.shape[0]
    r = np.arange(n, dtype=np.int64)
    kzs = sorted({int(m[2]) for m in modes})
    ph = 2.0 * np.pi * (np.outer(r, kzs) % n) / n           # (n, #kz)
    cz, sz = np.cos(ph), np.sin(ph)
    flat = x.reshape(n * n, n)
    tz = np.empty((n * n, len(kzs)), dtype=np.complex128)
    for i0 in range(0, n * n, rows):
        blk = flat[i0:i0 + rows].astype(np.float64)
        tz[i0:i0 + rows] = blk @ cz - 1j * (blk @ sz)
    tz = tz.reshape(n, n, len(kzs))
    out = np.empty(len(modes), dtype=np.complex128)
    for i, (kx, ky, kz) in enumerate(modes):
        ex = np.exp(-2j * np.pi * ((int(kx) * r) % n) / n)
        ey = np.exp(-2j * np.pi * ((int(ky) * r) % n) / n)
        out[i] = ex @ tz[:, :, kzs.index(int(kz))] @ ey
    return out


def wave_axes(n, box):
    """Integer-index wavenumbers for the three axes of a half spectrum.

    Returns (kx, ky, kz, dkx, dky, dkz): true kappa and derivative kappa~ on
    each axis, broadcastable to (n, n, n//2+1)."""
    kf = 2.0 * np.pi / box
    j = np.arange(n)
    full = kf * np.where(j < n // 2, j, j - n).astype(np.float64)
    dfull = full.copy()
    dfull[n // 2] = 0.0
    half = kf * np.arange(n // 2 + 1, dtype=np.float64)
    dhalf = half.copy()
    dhalf[n // 2] = 0.0
    return (full[:, None, None], full[None, :, None], half[None, None, :],
            dfull[:, None, None], dfull[None, :, None], dhalf[None, None, :])


def kgrid(n, box):
    """|k| on the half spectrum."""
    kx, ky, kz, *_ = wave_axes(n, box)
    return np.sqrt(kx * kx + ky * ky + kz * kz)


def multiplier(kind, n, box, axis=None, pk=None):
    """k-space multiplier of the given kind on the (n, n, n/2+1) half spectrum.

    kind: 'white' (needs pk, a callable P(k)), 'grad' (axis j), 'hess' (axis
    pair (i, j)).  All vanish at k = 0."""
    kx, ky, kz, dkx, dky, dkz = wave_axes(n, box)
    shape = (n, n, n // 2 + 1)
    k2 = np.broadcast_to(kx * kx + ky * ky + kz * kz, shape)
    inv_k2 = np.zeros(shape)
    nz = k2 > 0
    inv_k2[nz] = 1.0 / k2[nz]
    dk = (np.broadcast_to(dkx, shape), np.broadcast_to(dky, shape),
          np.broadcast_to(dkz, shape))
    if kind == "white":
        dq3 = (box / n) ** 3
        m = np.zeros(shape)
        m[nz] = np.sqrt(pk(np.sqrt(k2[nz])) / dq3)
        return m.astype(np.complex128)
    if kind == "grad":
        return 1j * dk[axis] * inv_k2
    if kind == "hess":
        i, j = axis
        return (dk[i] * dk[j] * inv_k2).astype(np.complex128)
    raise ValueError(kind)


def apply(m, x):
    """Op_m[x] = irfftn(m * rfftn(x)) for a real cubic field x."""
    n = x.shape[0]
    return irfft3(m * rfft3(x), n)


def apply_sum(pairs):
    """sum_i Op_{m_i}[x_i] for a list of (m_i, x_i) pairs."""
    acc = None
    for m, x in pairs:
        t = apply(m, x)
        acc = t if acc is None else acc + t
    return acc
