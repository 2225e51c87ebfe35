"""Pins of the oracle's counter generator, projection, rank-order matching and
projected L-BFGS (CPU only)."""
import numpy as np
import pytest

from oracle import fourier, lbfgs, philox, projection, rom


# ----------------------------------------------------------------- Philox
@pytest.mark.parametrize("ctr", [0, 7, 2 ** 40 + 3])
def test_philox_matches_numpy_bit_generator(ctr):
    """numpy's Philox4x64-10 advances its counter before the first block."""
    key = 0x1234ABCD
    bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64),
                          counter=np.array([ctr, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(8)
    ours = [philox.philox4x64(ctr + 1 + b, 0, 0, 0, key) for b in range(2)]
    ours = np.array([int(w) for blk in ours for w in blk], dtype=np.uint64)
    assert np.array_equal(raw, ours)


def test_philox_high_counter_words():
    """Counter words 1..3 as numpy sees them after a carry."""
    key = 99
    c = np.array([2 ** 64 - 1, 5, 6, 7], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64), counter=c)
    raw = bg.random_raw(4)
    ours = philox.philox4x64(0, 6, 6, 7, key)
    assert np.array_equal(raw, np.array([int(w) for w in ours], dtype=np.uint64))


def test_draw_distributions():
    j = np.arange(200000, dtype=np.uint64)
    z = philox.normal(j, 0, 2, 5, 77)
    a = philox.rayleigh(j, 3, 3, 5, 77)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert abs(np.mean(a * a) - 1) < 0.01
    u0, u1 = philox.uniform_pair(j, 0, 1, 0, 77)
    assert u0.min() > 0 and u0.max() < 1 and u1.min() > 0 and u1.max() < 1


# ------------------------------------------------------------- projection
def test_projection_zscore_without_resets():
    s = np.random.default_rng(20).normal(0.3, 2.0, size=(16, 16, 16))
    out, nres = projection.project(s, 10.0, 1, 0, 0)
    assert nres == 0
    assert abs(out.mean()) <= 1e-15
    assert abs(out.std() - 1.0) <= 1e-15


def test_projection_resets_planted_values():
    rng = np.random.default_rng(21)
    s = rng.standard_normal(4096)
    planted = [5, 77, 1000]
    s[planted] = [15.0, -12.0, 20.0]
    out, nres = projection.project(s, 10.0, 9, 3, 2)
    assert nres == 3
    # first pass: z-score, reset the three planted values with the pass-0 draws
    mu = s.mean()
    sd = np.sqrt(np.mean((s - mu) ** 2))
    z = (s - mu) / sd
    z[planted] = philox.normal(np.array(planted, dtype=np.uint64), 2, philox.STREAM_RESET, 3, 9)
    # second pass resets nothing: the output is z re-standardised
    mu2 = z.mean()
    sd2 = np.sqrt(np.mean((z - mu2) ** 2))
    assert np.allclose(out, (z - mu2) / sd2, rtol=0, atol=1e-14)
    assert abs(out.mean()) <= 1e-15 and abs(out.std() - 1) <= 1e-14


def test_projection_output_is_feasible_and_idempotent():
    rng = np.random.default_rng(28)
    s = rng.standard_normal(20000)
    s[rng.integers(0, 20000, 300)] *= 400.0   # many extremes: several passes
    out, nres = projection.project(s, 10.0, 4, 1, 0)
    assert nres >= 300
    assert abs(out.mean()) <= 1e-14 and abs(out.std() - 1) <= 1e-14
    assert np.max(np.abs(out)) <= 10.0
    again, n2 = projection.project(out, 10.0, 4, 2, 0)
    assert n2 == 0 and np.max(np.abs(again - out)) <= 1e-14


def test_projection_is_almost_identity_on_gaussian_samples():
    """Section 2.3.1: P(s) = s + O(1/d) for Gaussian s; the mean-square shift
    per element falls as 1/d."""
    ds, ms = [], []
    for d in [1000, 4000, 16000, 64000]:
        acc = []
        for t in range(40):
            s = np.random.default_rng(1000 * d + t).standard_normal(d)
            out, _ = projection.project(s, 10.0, 0, 0, 0)
            acc.append(np.mean((out - s) ** 2))
        ds.append(d)
        ms.append(np.mean(acc))
    slope = np.polyfit(np.log(ds), np.log(ms), 1)[0]
    assert abs(slope + 1.0) <= 0.1


# -------------------------------------------------------------------- ROM
def brute_ranks(x):
    """rank_i = number of elements strictly greater, plus equal ones before."""
    n = len(x)
    r = [0] * n
    for i in range(n):
        for j in range(n):
            if x[j] > x[i] or (x[j] == x[i] and j < i):
                r[i] += 1
    return r


def test_descending_order_matches_brute_force_with_ties_and_signed_zero():
    x = np.array([0.5, -0.0, 2.0, 0.0, 0.5, -1.0, 2.0, 0.0, -0.0, 3.0])
    o = rom.descending_order(x)
    ranks = np.empty(len(x), dtype=int)
    ranks[o] = np.arange(len(x))
    assert list(ranks) == brute_ranks(list(x))
    with pytest.raises(ValueError):
        rom.descending_order(np.array([1.0, np.nan]))


def test_match_properties():
    rng = np.random.default_rng(22)
    x = rng.standard_normal(500)
    t = rng.standard_normal(500)
    out, o = rom.match(x, t)
    assert np.array_equal(np.sort(out), np.sort(t))           # multiset, bitwise
    assert np.array_equal(np.argsort(-out, kind="stable"), o)  # ranks preserved
    same, _ = rom.match(x, x)
    assert np.array_equal(same, x)                             # identity


def test_match_error_scales_as_inverse_sqrt_n():
    """Section 2.3.2: on an input that already follows p(x) the matching
    moves each value by O(1/sqrt(N))."""
    ns, errs = [], []
    for n in [1000, 4000, 16000, 64000]:
        acc = []
        for t in range(20):
            rng = np.random.default_rng(n + t)
            x = rng.standard_normal(n)
            out, _ = rom.match(x, rng.standard_normal(n))
            acc.append(np.sqrt(np.mean((out - x) ** 2)))
        ns.append(n)
        errs.append(np.mean(acc))
    slope = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert abs(slope + 0.5) <= 0.1


def test_rom_real_only_touches_masked_cells():
    rng = np.random.default_rng(23)
    s = rng.standard_normal((8, 8, 8))
    R = (rng.uniform(size=(8, 8, 8)) > 0.5).astype(float)
    out, info = rom.rom_real(s, R, 1e-3, 5, 1)
    m = R >= 1e-3
    assert np.array_equal(out[~m], s[~m])
    t = philox.normal(np.arange(m.sum(), dtype=np.uint64), 0, philox.STREAM_ROM_REAL, 1, 5)
    assert np.array_equal(np.sort(out[m]), np.sort(t))


def test_rom_fourier_properties():
    n, L = 16, 128.0
    s = np.random.default_rng(24).standard_normal((n, n, n))
    out, info = rom.rom_fourier(s, L, 7, 2)
    z0 = fourier.rfft3(s) / n ** 1.5
    z1 = fourier.rfft3(out) / n ** 1.5
    idx, bins, partner = rom.fourier_mode_sets(n, L)
    touched = np.zeros(z0.size, bool)
    touched[idx] = True
    touched[partner[partner >= 0]] = True
    assert np.max(np.abs(z1.reshape(-1)[~touched] - z0.reshape(-1)[~touched])) <= 1e-12
    for b in range(100):
        sel = np.nonzero(bins == b)[0]
        if sel.size == 0:
            continue
        amp = np.abs(z1.reshape(-1)[idx[sel]])
        t = philox.rayleigh(np.arange(sel.size, dtype=np.uint64), b,
                            philox.STREAM_ROM_FOURIER, 2, 7)
        assert np.allclose(np.sort(amp), np.sort(t), rtol=1e-12, atol=1e-12)
        ph0 = np.angle(z0.reshape(-1)[idx[sel]])
        ph1 = np.angle(z1.reshape(-1)[idx[sel]])
        assert np.max(np.abs(np.angle(np.exp(1j * (ph1 - ph0))))) <= 1e-10
    # the modes below k_min and the self-conjugate modes are untouched
    k = fourier.kgrid(n, L).reshape(-1)
    assert not touched[k < 0.1].any()


def test_fourier_mode_sets_cover_each_conjugate_pair_once():
    n, L = 8, 8.0  # k_min below the fundamental: every non-DC mode qualifies
    idx, bins, partner = rom.fourier_mode_sets(n, L)
    nh = n // 2 + 1
    # count real degrees of freedom: 2 per independent complex mode
    selfconj = 8  # kx, ky, kz each in {0, N/2}
    dof = 2 * len(idx) + selfconj
    assert dof == n ** 3
    assert len(set(idx.tolist()) & set(partner[partner >= 0].tolist())) == 0


# ----------------------------------------------------------------- L-BFGS
def test_two_loop_equals_explicit_bfgs_matrix():
    rng = np.random.default_rng(25)
    d = 30
    opt = lbfgs.ProjectedLBFGS(m=50)
    A = rng.standard_normal((d, d))
    A = A @ A.T + d * np.eye(d)
    for _ in range(12):
        S = rng.standard_normal(d)
        opt.S.append(S)
        opt.Y.append(A @ S)
    Sl, Yl = opt.S, opt.Y
    gamma = Sl[-1] @ Yl[-1] / (Yl[-1] @ Yl[-1])
    H = gamma * np.eye(d)
    for S, Y in zip(Sl, Yl):
        rho = 1.0 / (S @ Y)
        V = np.eye(d) - rho * np.outer(Y, S)
        H = V.T @ H @ V + rho * np.outer(S, S)
    g = rng.standard_normal(d)
    p = opt.direction(g)
    assert np.allclose(p, -H @ g, rtol=1e-12, atol=1e-12)
    assert np.allclose(H @ Yl[-1], Sl[-1], rtol=1e-12, atol=1e-12)   # secant


def test_projected_lbfgs_monotone_on_quadratic():
    """On a convex quadratic whose minimiser is unaffected by the projection
    scale, every accepted step satisfies the sufficient-decrease test along
    the projection arc and lowers the loss."""
    rng = np.random.default_rng(26)
    d = 4096
    target = rng.standard_normal(d)
    target = (target - target.mean()) / target.std()
    diag = rng.uniform(1.0, 5.0, d)
    fun = lambda s: (0.5 * np.sum(diag * (s - target) ** 2), diag * (s - target))
    opt = lbfgs.ProjectedLBFGS(seed=3)
    s, _ = projection.project(rng.standard_normal(d), 10.0, 3, 0, 0)
    L, g = fun(s)
    for k in range(15):
        s2, g2, L2, info = opt.step(s, g, L, fun, k)
        dec = float(np.dot(g, s2 - s))
        assert dec < 0 and L2 <= L + 1e-4 * dec      # Armijo along the projection arc
        assert L2 < L
        s, g, L = s2, g2, L2
    assert L < 1e-2 * fun(projection.project(rng.standard_normal(d), 10, 3, 0, 0)[0])[0]


def test_line_search_restarts_with_steepest_descent():
    """A quasi-Newton direction along s itself is undone by the projection
    (P(s + eps c s) = s), so its line search cannot decrease the loss; the
    step then resets the history and searches along -g."""
    d = 1000
    rng = np.random.default_rng(27)
    s, _ = projection.project(rng.standard_normal(d), 10.0, 1, 0, 0)
    target, _ = projection.project(rng.standard_normal(d), 10.0, 1, 0, 1)
    fun = lambda x: (0.5 * np.sum((x - target) ** 2), x - target)
    opt = lbfgs.ProjectedLBFGS(seed=1, max_trials=5)
    opt.S.append(np.ones(d))
    opt.Y.append(np.ones(d))
    L, g = fun(s)
    opt.direction = lambda gg: -np.sign(gg @ s) * s
    s2, g2, L2, info = opt.step(s, g, L, fun, 0)
    assert info["restarted"] and L2 < L
    assert info["evaluations"] == info["trials"]  # 5 failed trials, then the -g search


def test_plain_lbfgs_reaches_the_minimiser_of_a_quadratic():
    """Without projected steps the method is plain backtracking L-BFGS: on a
    strictly convex quadratic 1/2 x^T A x - b^T x it reaches the solution of
    A x = b (an independent linear solve)."""
    from oracle import lbfgs
    rng = np.random.default_rng(31)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 30.0, n)) @ Q.T
    b = rng.standard_normal(n)

    def fun(x):
        x = x.reshape(-1)
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    opt = lbfgs.ProjectedLBFGS(project_steps=False)
    x = np.zeros(n)
    L, g = fun(x)
    for it in range(200):
        if np.linalg.norm(g) < 1e-6:   # |x - x*| <= |g| / lambda_min = |g|
            break
        x, g, L, info = opt.step(x, g, L, fun, it)
        assert info["resets"] == 0
    assert np.linalg.norm(g) < 1e-6
    ref = np.linalg.solve(A, b)
    assert np.max(np.abs(x - ref)) <= 1e-6


def test_rom_fourier_reim_properties():
    """Second reading of the Fourier-space matching (section 2.3.2): per k bin
    the real and imaginary parts of the matched modes are one set of 2n
    values matched to 2n draws of N(0, 1/2).  Pins: after the inverse and a
    fresh forward transform each bin's Re/Im multiset is the sorted draws,
    their ranks are the input's ranks (brute-force O(n^2) ranks on every
    bin), modes outside the matched set and their partners are untouched, and
    the draws have the variance 1/2 of a white-noise mode's parts."""
    n, L = 16, 128.0
    s = np.random.default_rng(26).standard_normal((n, n, n))
    out, info = rom.rom_fourier_reim(s, L, 7, 2)
    assert out.dtype == np.float64 and out.shape == s.shape
    z0 = (fourier.rfft3(s) / n ** 1.5).reshape(-1)
    z1 = (fourier.rfft3(out) / n ** 1.5).reshape(-1)
    idx, bins, partner = rom.fourier_mode_sets(n, L)
    touched = np.zeros(z0.size, bool)
    touched[idx] = True
    touched[partner[partner >= 0]] = True
    assert np.max(np.abs(z1[~touched] - z0[~touched])) <= 1e-12
    nb = 0
    for b in range(100):
        sel = np.nonzero(bins == b)[0]
        if sel.size == 0:
            continue
        nb += 1
        old = np.empty(2 * sel.size)
        old[0::2], old[1::2] = z0[idx[sel]].real, z0[idx[sel]].imag
        new = np.empty(2 * sel.size)
        new[0::2], new[1::2] = z1[idx[sel]].real, z1[idx[sel]].imag
        t = philox.normal(np.arange(2 * sel.size, dtype=np.uint64), b,
                          philox.STREAM_ROM_FOURIER_REIM, 2, 7) * np.sqrt(0.5)
        assert np.allclose(np.sort(new), np.sort(t), rtol=0, atol=1e-12)
        ranks = np.array(brute_ranks(list(old)))
        assert np.allclose(new, np.sort(t)[::-1][ranks], rtol=0, atol=1e-12)
        assert np.array_equal(info["elements"][b][0::2], 2 * idx[sel])
    assert nb > 50
    # conjugate partners hold the conjugate of their matched mode
    m = partner >= 0
    assert np.max(np.abs(z1[partner[m]] - np.conj(z1[idx[m]]))) <= 1e-12
    d = philox.normal(np.arange(400000, dtype=np.uint64), 3, philox.STREAM_ROM_FOURIER_REIM,
                      1, 9) * np.sqrt(0.5)
    assert abs(d.mean()) <= 5e-3 and abs(d.var() - 0.5) <= 5e-3
