"""Pins of the oracle's white-noise upsampling (CPU only): every mode of the
fine field, on the full (not half) spectrum from a brute-force DFT, is the
coarse field's mode times (N_h/N_l)^{3/2} where all three wave numbers lie
strictly inside the coarse band and the fresh field's mode elsewhere; the
coarse field comes back exactly from the fine one; white-noise statistics."""
import numpy as np

from oracle import philox, upsample


def brute_dft(x):
    """Full-spectrum DFT straight from the definition (O(N^6))."""
    n = x.shape[0]
    j = np.arange(n)
    e = np.exp(-2j * np.pi * np.outer(j, j) / n)          # e[k, r]
    return np.einsum("ka,lb,mc,abc->klm", e, e, e, x)


def test_modes_of_the_fine_field():
    nl, nh, seed, event = 4, 8, 7, 3
    s = np.random.default_rng(1).standard_normal((nl, nl, nl))
    out = upsample.upsample(s, nh, seed, event)
    fresh = philox.normal(np.arange(nh ** 3, dtype=np.uint64), 0, upsample.STREAM_UPSAMPLE,
                          event, seed).reshape(nh, nh, nh)
    Zo, Zf, Zl = brute_dft(out), brute_dft(fresh), brute_dft(s)
    scale = (nh / nl) ** 1.5
    wave = lambda i, n: i if i < n // 2 else i - n
    for a in range(nh):
        for b in range(nh):
            for c in range(nh):
                k = (wave(a, nh), wave(b, nh), wave(c, nh))
                if all(abs(q) < nl // 2 for q in k):
                    ref = scale * Zl[k[0] % nl, k[1] % nl, k[2] % nl]
                else:
                    ref = Zf[a, b, c]
                assert abs(Zo[a, b, c] - ref) <= 1e-12 * nh ** 1.5, (a, b, c)


def test_coarse_field_comes_back():
    nl, nh = 16, 32
    s = np.random.default_rng(2).standard_normal((nl, nl, nl))
    out = upsample.upsample(s, nh, 9, 1)
    z = np.fft.rfftn(out)
    fine, coarse = upsample.coarse_index(nl, nh)
    zl = np.zeros((nl, nl, nl // 2 + 1), dtype=np.complex128)
    kz = np.arange(nl // 2)
    zl[np.ix_(coarse, coarse, kz)] = (nl / nh) ** 1.5 * z[np.ix_(fine, fine, kz)]
    back = np.fft.irfftn(zl, s=(nl, nl, nl), axes=(0, 1, 2))
    # the coarse Nyquist modes are not carried: compare with s without them
    zs = np.fft.rfftn(s)
    keep = np.zeros_like(zs)
    keep[np.ix_(coarse, coarse, kz)] = zs[np.ix_(coarse, coarse, kz)]
    assert np.max(np.abs(back - np.fft.irfftn(keep, s=(nl, nl, nl), axes=(0, 1, 2)))) <= 1e-12


def test_white_noise_statistics():
    s = np.random.default_rng(3).standard_normal((32, 32, 32))
    out = upsample.upsample(s, 64, 11, 2)
    assert abs(out.mean()) < 0.01 and abs(out.std() - 1.0) < 0.01
