"""Rank-order matching R[x] (test infrastructure only).

Paper section 2.3.2: (1) find the descending rank of every element, (2) draw
a realisation of the target distribution of the same length and sort it in
descending order, (3) give each element the draw of its rank.  The method
applies it to the white noise in real space on the cells with tracers and
per k bin to the Fourier modes (100 equal-width bins in |k|, modes with
k < 0.1 h/Mpc untouched).

Readings taken where the paper is silent:

* ties in the ranking keep the canonical index order (stable sort); -0 and +0
  are equal; NaN is an error;
* real space: the set is {n : R(n) >= r_min} in flat index order and the
  target is N(0, 1) (the white noise's own distribution);
* Fourier space: z = rfftn(s) / N^(3/2) so that a white-noise mode has
  E|z|^2 = 1.  The independent modes are all half-spectrum modes with
  0 < kz < N/2 plus, in the kz = 0 and kz = N/2 planes, the member of each
  conjugate pair with the smaller flat index (self-conjugate modes are left
  alone).  Modes with |k| >= k_min = 0.1 fall into bin
  b = min(99, floor((|k| - k_min) / dk)), dk = (sqrt(3) pi N / L - k_min)/100.
  The amplitudes |z| are matched to Rayleigh draws (E a^2 = 1), the phases
  are kept, and the conjugate partners are mirrored before the inverse FFT.
* Fourier space, second reading (rom_fourier_reim): the paper's "matching
  the Fourier modes" may also mean the real and imaginary parts, which for
  white noise are independent N(0, 1/2) samples.  Per bin the 2n values
  Re z_f, Im z_f of its n modes form one set whose canonical order is the
  element index 2 f + c (c = 0 for Re, 1 for Im, f the flat half-spectrum
  index), matched to 2n draws of N(0, 1/2); the conjugate partners are
  mirrored as above.
"""
import numpy as np

from . import fourier, philox

__all__ = ["descending_order", "match", "rom_real", "fourier_mode_sets",
           "rom_fourier", "rom_fourier_reim"]


def descending_order(values):
    """Stable descending argsort: o[j] = index of the j-th largest value."""
    v = np.asarray(values, dtype=np.float64)
    if np.isnan(v).any():
        raise ValueError("NaN in rank-order matching input")
    return np.argsort(-(v + 0.0), kind="stable")


def match(values, targets):
    """R[x]: out[o_j] = tau_j with tau the targets sorted descending."""
    o = descending_order(values)
    tau = np.sort(np.asarray(targets, dtype=np.float64))[::-1]
    out = np.empty(len(o))
    out[o] = tau
    return out, o


def rom_real(s, response, r_min, seed, event):
    """Real-space ROM of the white noise on cells with R >= r_min."""
    s = np.asarray(s, dtype=np.float64)
    flat = s.reshape(-1).copy()
    sel = np.nonzero(np.asarray(response).reshape(-1) >= r_min)[0]
    targets = philox.normal(np.arange(sel.size, dtype=np.uint64), 0,
                            philox.STREAM_ROM_REAL, event, seed)
    matched, o = match(flat[sel], targets)
    flat[sel] = matched
    return flat.reshape(s.shape), dict(n=int(sel.size), order=o, keys=s.reshape(-1)[sel])


def fourier_mode_sets(n, box, k_min=0.1, n_bins=100):
    """Flat half-spectrum indices of the matched modes and their bins, in
    flat index order, plus the flat index of each mode's conjugate partner
    inside the half spectrum (or -1 when it is not stored separately)."""
    nh = n // 2 + 1
    kx, ky, kz = np.meshgrid(np.arange(n), np.arange(n), np.arange(nh), indexing="ij")
    flat = (kx * n + ky) * nh + kz
    cx, cy = (-kx) % n, (-ky) % n
    conj_flat = (cx * n + cy) * nh + kz
    edge = (kz == 0) | (kz == n // 2)
    independent = np.where(edge, flat < conj_flat, True)
    k = fourier.kgrid(n, box)
    dk = (np.sqrt(3.0) * np.pi * n / box - k_min) / n_bins
    chosen = independent & (k >= k_min)
    idx = flat[chosen]
    bins = np.minimum(n_bins - 1, np.floor((k[chosen] - k_min) / dk)).astype(np.int64)
    partner = np.where(edge[chosen], conj_flat[chosen], -1)
    return idx, bins, partner


def rom_fourier(s, box, seed, event, k_min=0.1, n_bins=100):
    """Fourier-space ROM of the amplitudes, phases kept."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[0]
    norm = n ** 1.5
    z = (fourier.rfft3(s) / norm).reshape(-1)
    idx, bins, partner = fourier_mode_sets(n, box, k_min, n_bins)
    orders, keys = {}, {}
    for b in range(n_bins):
        sel = np.nonzero(bins == b)[0]
        if sel.size == 0:
            continue
        amp = np.abs(z[idx[sel]])
        targets = philox.rayleigh(np.arange(sel.size, dtype=np.uint64), b,
                                  philox.STREAM_ROM_FOURIER, event, seed)
        new_amp, o = match(amp, targets)
        zz = z[idx[sel]]
        phase = np.where(amp > 0, zz / np.where(amp > 0, amp, 1.0), 1.0)
        z[idx[sel]] = new_amp * phase
        orders[b], keys[b] = o, amp
    mirror = partner >= 0
    z[partner[mirror]] = np.conj(z[idx[mirror]])
    out = fourier.irfft3(z.reshape(n, n, n // 2 + 1), n) * norm
    return out, dict(orders=orders, keys=keys)


def rom_fourier_reim(s, box, seed, event, k_min=0.1, n_bins=100):
    """Fourier-space ROM of the real and imaginary parts (second reading).

    Per k bin: the 2n values (Re z_f, Im z_f) of its n matched modes, in the
    canonical element order 2 f + c, are rank-matched to 2n draws of
    N(0, 1/2) (Philox stream STREAM_ROM_FOURIER_REIM, sub = bin, j = 0..2n-1,
    each a standard normal times sqrt(1/2)); conjugate partners mirrored."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[0]
    norm = n ** 1.5
    z = (fourier.rfft3(s) / norm).reshape(-1)
    idx, bins, partner = fourier_mode_sets(n, box, k_min, n_bins)
    orders, keys, elements = {}, {}, {}
    for b in range(n_bins):
        sel = np.nonzero(bins == b)[0]
        if sel.size == 0:
            continue
        zz = z[idx[sel]]
        v = np.empty(2 * sel.size)
        v[0::2], v[1::2] = zz.real, zz.imag
        targets = philox.normal(np.arange(2 * sel.size, dtype=np.uint64), b,
                                philox.STREAM_ROM_FOURIER_REIM, event, seed) * np.sqrt(0.5)
        new, o = match(v, targets)
        z[idx[sel]] = new[0::2] + 1j * new[1::2]
        e = np.empty(2 * sel.size, dtype=np.int64)
        e[0::2], e[1::2] = 2 * idx[sel], 2 * idx[sel] + 1
        orders[b], keys[b], elements[b] = o, v, e
    mirror = partner >= 0
    z[partner[mirror]] = np.conj(z[idx[mirror]])
    out = fourier.irfft3(z.reshape(n, n, n // 2 + 1), n) * norm
    return out, dict(orders=orders, keys=keys, elements=elements)
