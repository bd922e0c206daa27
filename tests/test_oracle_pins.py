"""Pins of the FP64 oracle against things other than itself: brute force on
tiny inputs, closed forms, library routines, invariants the paper states and
finite differences.  CPU only."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle.swift_oracle import bilinear_clamped, STATUS_NEAR_TIE, STATUS_DEGENERATE
from datagen import make_pair64

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def ident(cx, cy, tx=0.0, ty=0.0):
    return np.array([cx, cy, 1.0, 0.0, tx, 0.0, 1.0, ty])


# ---------------------------------------------------------------- gather
def test_gather_identity_is_pixel_copy():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, size=(40, 50)).astype(np.uint8)
    n = 16
    a, cl = O.gather(img, ident(20, 17), n)
    assert not cl
    # window pixel (i, j) samples (20 + i - 8, 17 + j - 8)
    np.testing.assert_array_equal(a, img[9:25, 12:28].astype(np.float64))


def test_gather_integer_translation_exact():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(40, 40)).astype(np.uint8)
    a, _ = O.gather(img, ident(20, 20, tx=3.0, ty=-2.0), 8)
    np.testing.assert_array_equal(a, img[14:22, 19:27].astype(np.float64))


def test_bilinear_reproduces_affine_ramps():
    # closed form: bilinear interpolation is exact for f = alpha x + beta y + gamma
    h, w = 30, 37
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    al, be, ga = 0.37, -1.21, 5.5
    img = al * xx + be * yy + ga
    rng = np.random.default_rng(2)
    x = rng.uniform(0, w - 1, 500)
    y = rng.uniform(0, h - 1, 500)
    v, _ = bilinear_clamped(img, x, y)
    np.testing.assert_allclose(v, al * x + be * y + ga, rtol=0, atol=1e-12)


def test_bilinear_matches_scipy_map_coordinates_nearest():
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 255, size=(25, 31))
    x = rng.uniform(-3, 34, 2000)
    y = rng.uniform(-3, 28, 2000)
    v, cl = bilinear_clamped(img, x, y)
    ref = map_coordinates(img, [y, x], order=1, mode="nearest")
    assert cl
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-10)


def test_gather_affine_matches_scipy():
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 255, size=(64, 64))
    th = np.array([31.0, 30.0, 1.01, 0.02, 0.3, -0.015, 0.99, -0.7])
    n = 32
    a, _ = O.gather(img, th, n)
    u = np.arange(n) - n // 2
    uu, vv = np.meshgrid(u, u)
    x = th[0] + th[2] * uu + th[3] * vv + th[4]
    y = th[1] + th[5] * uu + th[6] * vv + th[7]
    ref = map_coordinates(img, [y, x], order=1, mode="nearest")
    np.testing.assert_allclose(a, ref, atol=1e-10)


# ---------------------------------------------------------------- taper / mean
@pytest.mark.parametrize("n", [16, 64, 512])
def test_taper_raised_cosine_properties(n):
    t = O.taper_1d(n, 0.25)
    L = n // 8
    # mirror symmetry, complementarity of the raised cosine, flat middle
    np.testing.assert_allclose(t, t[::-1], atol=0)
    for i in range(L):
        assert abs(t[i] + t[L - 1 - i] - 1.0) < 1e-15
    assert np.all(t[L:n - L] == 1.0)
    assert np.all(np.diff(t[:L]) > 0)
    # half-angle identity: t(0) = sin^2(pi / (4 L))
    assert abs(t[0] - math.sin(math.pi / (4 * L)) ** 2) < 1e-15
    assert np.all(O.taper_1d(n, 0.0) == 1.0)


def test_mean_removal_zero_sum_and_offset_invariance():
    rng = np.random.default_rng(5)
    a = rng.uniform(0, 255, (32, 32))
    T = O.taper_2d(32, 0.25)
    w, m = O.prepare(a, T)
    assert abs(w.sum()) < 1e-9
    w2, _ = O.prepare(a + 17.25, T)
    np.testing.assert_allclose(w, w2, atol=1e-9)


# ---------------------------------------------------------------- FFT conventions
def test_rfft2_matches_bruteforce_dft():
    n = 8
    rng = np.random.default_rng(6)
    x = rng.standard_normal((n, n))
    F = np.zeros((n, n), complex)
    for ky, kx in itertools.product(range(n), range(n)):
        s = 0
        for yy, xx in itertools.product(range(n), range(n)):
            s += x[yy, xx] * np.exp(-2j * np.pi * (ky * yy + kx * xx) / n)
        F[ky, kx] = s
    np.testing.assert_allclose(np.fft.rfft2(x), F[:, : n // 2 + 1], atol=1e-11)


# ---------------------------------------------------------------- p = 0: plain correlation
@pytest.mark.parametrize("n", [16, 32])
def test_p0_equals_bruteforce_circular_correlation(n):
    rng = np.random.default_rng(7 + n)
    wA, _ = O.prepare(rng.standard_normal((n, n)), O.taper_2d(n, 0.25))
    wB, _ = O.prepare(rng.standard_normal((n, n)), O.taper_2d(n, 0.25))
    c = O.whitened_surface(wA, wB, 0.0, 1e-4)
    bf = np.zeros((n, n))
    for sy in range(n):
        for sx in range(n):
            bf[sy, sx] = np.sum(wA * np.roll(wB, (-sy, -sx), axis=(0, 1)))
    np.testing.assert_allclose(c, bf, rtol=0, atol=1e-12 * np.abs(bf).max())


# ---------------------------------------------------------------- p = 1: phase-only delta
def test_p1_delta_closed_form():
    g = GOLD["poc_delta_n64"]
    n = g["n"]
    dx, dy = g["shift_dx_dy"]
    rng = np.random.default_rng(8)
    a = rng.standard_normal((n, n))
    b = np.roll(a, (dy, dx), axis=(0, 1))  # b(x) = a(x - d)
    T = O.taper_2d(n, 0.0)
    wA, _ = O.prepare(a, T)
    wB, _ = O.prepare(b, T)
    c = O.whitened_surface(wA, wB, 1.0, 0.0)
    iy, ix = dy % n, dx % n
    assert abs(c[iy, ix] - g["peak_value"]) < 1e-12
    mask = np.ones_like(c, bool)
    mask[iy, ix] = False
    assert np.max(np.abs(c[mask] - g["off_peak_value"])) < 1e-12
    rec = O.peak_stats(c)
    assert (rec["iy"], rec["ix"]) == (iy, ix)
    assert (rec["sx"], rec["sy"]) == (dx, dy)
    assert abs(rec["snr"] - g["snr"]) < 1e-9
    assert abs(rec["snr"] - math.sqrt(n * n - 1)) < 1e-9


# ---------------------------------------------------------------- integer shift recovery
@pytest.mark.parametrize("p", GOLD["pair64_integer_peak"]["p_values"])
def test_pair64_integer_peak(p):
    g = GOLD["pair64_integer_peak"]
    a, b = make_pair64()
    rec = O.match_pair(a, b, ident(32, 32), ident(32, 32), 64, O.Params(p=p))
    assert [rec["iy"], rec["ix"]] == g["peak_index_iy_ix"]
    assert abs(rec["dx"] - 7) < 0.5 and abs(rec["dy"] + 3) < 0.5


# ---------------------------------------------------------------- whitening before/after the multiply
@pytest.mark.parametrize("p", [0.3, 0.65, 1.0])
def test_whitening_before_equals_after_multiply(p):
    n = 32
    rng = np.random.default_rng(9)
    T = O.taper_2d(n, 0.25)
    wA, _ = O.prepare(rng.standard_normal((n, n)), T)
    wB, _ = O.prepare(rng.standard_normal((n, n)), T)
    c = O.whitened_surface(wA, wB, p, 0.0)
    FA = np.fft.rfft2(wA)
    FB = np.fft.rfft2(wB)
    Cb = np.conj(FA / np.abs(FA) ** p) * (FB / np.abs(FB) ** p)
    Cb[0, 0] = 0
    cb = np.fft.irfft2(Cb, s=(n, n))
    np.testing.assert_allclose(c, cb, atol=1e-12 * np.abs(cb).max())


def test_whitening_changes_amplitudes_only():
    # phases of C equal phases of X wherever X != 0
    n = 16
    rng = np.random.default_rng(10)
    T = O.taper_2d(n, 0.25)
    wA, _ = O.prepare(rng.standard_normal((n, n)), T)
    wB, _ = O.prepare(rng.standard_normal((n, n)), T)
    _, parts = O.whitened_surface(wA, wB, 0.7, 1e-4, return_parts=True)
    X, C = parts["X"], parts["C"]
    nz = np.abs(X) > 1e-9
    nz[0, 0] = False
    np.testing.assert_allclose(np.angle(C[nz]), np.angle(X[nz]), atol=1e-12)


# ---------------------------------------------------------------- SNR
@pytest.mark.parametrize("p", [0.0, 0.65, 1.0])
def test_snr_invariant_to_intensity_affine(p):
    a, b = (v.astype(np.float64) for v in make_pair64())
    par = O.Params(p=p, eps_rel=1e-4)
    r0 = O.match_pair(a, b, ident(32, 32), ident(32, 32), 64, par)
    r1 = O.match_pair(3.5 * a + 11.0, 0.25 * b - 40.0, ident(32, 32), ident(32, 32), 64, par)
    assert abs(r0["snr"] - r1["snr"]) < 1e-9 * r0["snr"]
    assert (r0["ix"], r0["iy"]) == (r1["ix"], r1["iy"])


def test_snr_bound_and_parseval():
    rng = np.random.default_rng(11)
    n = 32
    T = O.taper_2d(n, 0.25)
    for p in (0.0, 0.5, 1.0):
        wA, _ = O.prepare(rng.standard_normal((n, n)), T)
        wB, _ = O.prepare(rng.standard_normal((n, n)), T)
        c, parts = O.whitened_surface(wA, wB, p, 1e-4, return_parts=True)
        rec = O.peak_stats(c)
        assert rec["snr"] <= math.sqrt(n * n - 1) + 1e-9
        # surface mean is zero (DC bin removed) and its variance follows from
        # the half spectrum by Parseval (multiplicity 2 off the kx = 0, N/2 columns)
        C = parts["C"]
        mult = np.full(C.shape, 2.0)
        mult[:, 0] = 1.0
        mult[:, n // 2] = 1.0
        var = np.sum(mult * np.abs(C) ** 2) / float(n) ** 4
        assert abs(rec["mean"]) < 1e-14 * np.abs(c).max()
        assert abs(rec["std"] - math.sqrt(var)) < 1e-12 * rec["std"]


@pytest.mark.parametrize("value", [100.0, 37.0, 211.5])
@pytest.mark.parametrize("taper", [0.25, 0.0, 1.0])
@pytest.mark.parametrize("n", [64, 256])
def test_degenerate_constant_window(value, taper, n):
    """A constant window is exactly zero after the taper-weighted mean removal
    (w = (a - m_T) T with m_T = a), so its surface is zero, sigma = 0 and the
    match is degenerate, whatever the taper and the constant."""
    a = np.full((n, n), value)
    b = np.random.default_rng(3).normal(128.0, 30.0, (n, n))
    w, m = O.prepare(a, O.taper_2d(n, taper))
    assert m == value and not w.any()
    rec = O.match_pair(a, b, ident(n / 2, n / 2), ident(n / 2, n / 2), n, O.Params(p=0.65, taper_frac=taper))
    assert rec["snr"] == 0.0 and rec["status"] & STATUS_DEGENERATE


def _taper_sums(n, taper):
    t = O.taper_1d(n, taper)
    T = np.outer(t, t)
    return T, float(T.sum()), float((T * T).sum())


def test_prepare_is_the_weighted_mean_removal_about_any_offset():
    """w = (a - m_T) T with m_T = sum(aT)/sum(T), whatever offset the sums are
    taken about (written out directly here, not through the offset form)."""
    rng = np.random.default_rng(21)
    n = 32
    T, sT, _ = _taper_sums(n, 0.25)
    a = rng.uniform(0, 255, (n, n))
    mT = float((a * T).sum()) / sT
    direct = (a - mT) * T
    for o in (0.0, 128.0, float(a[n // 2, n // 2]), 1e4):
        w, m = O.prepare(a, T, o)
        np.testing.assert_allclose(w, direct, atol=1e-9 * np.abs(direct).max())
        assert abs(m - mT) < 1e-9 * abs(mT)


@pytest.mark.parametrize("n", [64, 512])
def test_near_constant_window_is_scored(n):
    """A window of 200 with one pixel at 201 is not degenerate: about the
    centre pixel o = 200, d is one unit impulse at p, and ||w||^2 / sum (dT)^2
    = 1 - 2 T_p / sum T + sum T^2 / (sum T)^2 (closed form, near 1)."""
    T, sT, sT2 = _taper_sums(n, 0.25)
    py, px = n // 3, n // 5
    a = np.full((n, n), 200.0)
    a[py, px] = 201.0
    w, _ = O.prepare(a, T, 200.0)
    Tp = T[py, px]
    ratio = 1 - 2 * Tp / sT + sT2 / sT ** 2
    assert abs(float((w * w).sum()) - Tp * Tp * ratio) < 1e-12 * Tp * Tp
    rng = np.random.default_rng(2)
    img = np.full((n + 8, n + 8), 200.0)
    img[4 + py, 4 + px] = 201.0
    th = ident(4 + n / 2, 4 + n / 2)
    assert O.centre_pixel(img, th) == 200.0
    b = img + 0.0
    rec = O.match_pair(img, b, th, th, n, O.Params(p=0.65))
    assert not rec["status"] & STATUS_DEGENERATE and rec["snr"] > 1.0
    assert (rec["sx"], rec["sy"]) == (0, 0)
    del rng


@pytest.mark.parametrize("below", [True, False])
def test_degeneracy_threshold_closed_form(below):
    """d = a - o = K + delta [i = p]: ||w||^2 = delta^2 T_p^2 rho (rho as in
    the impulse case, K drops out with the mean) while sum (dT)^2 = K^2 sum T^2
    + 2 K delta T_p^2 + delta^2 T_p^2.  The window is degenerate exactly when
    their ratio is at most 1e-6."""
    n = 64
    T, sT, sT2 = _taper_sums(n, 0.25)
    py, px = 20, 41
    Tp = T[py, px]
    rho = 1 - 2 * Tp / sT + sT2 / sT ** 2
    delta = 1.0
    target = 0.5e-6 if below else 2e-6
    # solve K^2 sT2 + 2 K delta Tp^2 + delta^2 Tp^2 = delta^2 Tp^2 rho / target for K > 0
    qa, qb, qc = sT2, 2 * delta * Tp * Tp, delta * delta * Tp * Tp * (1 - rho / target)
    K = (-qb + math.sqrt(qb * qb - 4 * qa * qc)) / (2 * qa)
    a = np.full((n, n), 50.0 + K)
    a[py, px] += delta
    w, _ = O.prepare(a, T, 50.0)
    ratio = float((w * w).sum()) / float((((a - 50.0) * T) ** 2).sum())
    if below:
        assert not w.any()
    else:
        assert w.any() and abs(ratio / target - 1) < 1e-6


def test_constant_window_off_the_offset_is_degenerate():
    """Columns alternate 0 and 2; at half a pixel of x translation every
    bilinear sample is exactly 1 while the centre pixel is 0 or 2, so the
    samples are constant but not equal to the offset: still degenerate."""
    n = 64
    img = np.zeros((n + 8, n + 8))
    img[:, 1::2] = 2.0
    th = ident(4 + n / 2, 4 + n / 2, tx=0.5)
    a, _ = O.gather(img, th, n)
    assert np.all(a == 1.0) and O.centre_pixel(img, th) in (0.0, 2.0)
    rng = np.random.default_rng(4)
    imgb = rng.uniform(0, 255, img.shape)
    rec = O.match_pair(img, imgb, th, ident(4 + n / 2, 4 + n / 2), n, O.Params(p=0.65))
    assert rec["status"] & STATUS_DEGENERATE and rec["snr"] == 0.0


def test_centre_pixel_rounds_half_up_and_clamps():
    img = np.arange(20 * 30, dtype=np.float64).reshape(20, 30)
    assert O.centre_pixel(img, ident(10.0, 5.0, tx=0.5, ty=0.49)) == img[5, 11]
    assert O.centre_pixel(img, ident(10.0, 5.0, tx=0.49, ty=0.5)) == img[6, 10]
    assert O.centre_pixel(img, ident(-3.0, 5.0)) == img[5, 0]
    assert O.centre_pixel(img, ident(10.0, 40.0)) == img[19, 10]


def test_snr_background_exclusion_closed_form():
    """Checkerboard surface (-1)^(x+y) on 8 x 8 with a 3 x 3 box of 5 around a
    peak of 10 at (iy, ix) = (2, 3).  Without the box the background is the
    55 checkerboard entries outside it: the box covers five entries of sign
    -1 and four of +1, so they sum to +1 and their squares to 55: mean 1/55,
    population variance 1 - 1/55^2.  The whole-surface statistics count the
    box as well."""
    n = 8
    y, x = np.mgrid[0:n, 0:n]
    c = np.where((x + y) % 2 == 0, 1.0, -1.0)
    c[1:4, 2:5] = 5.0
    c[2, 3] = 10.0
    rec = O.peak_stats(c, exclude_r=1)
    assert (rec["iy"], rec["ix"]) == (2, 3)
    mu = 1.0 / 55.0
    sd = math.sqrt(1.0 - mu * mu)
    assert abs(rec["mean"] - mu) < 1e-15 and abs(rec["std"] - sd) < 1e-15
    assert abs(rec["snr"] - (10.0 - mu) / sd) < 1e-13
    full = O.peak_stats(c)
    mf = (1.0 + 8 * 5.0 + 10.0) / 64.0
    assert abs(full["mean"] - mf) < 1e-15
    # the box wraps around the surface edge
    c2 = np.roll(np.roll(c, -2, axis=0), -3, axis=1)
    rec2 = O.peak_stats(c2, exclude_r=1)
    assert (rec2["iy"], rec2["ix"]) == (0, 0)
    assert abs(rec2["mean"] - mu) < 1e-15 and abs(rec2["std"] - sd) < 1e-15


# ---------------------------------------------------------------- peak / centroid
def test_centroid_closed_forms_and_wrap():
    n = 16
    c = np.zeros((n, n))
    c[3, 5] = 1.0
    c[3, 6] = 0.5
    rec = O.peak_stats(c)
    mu = 1.5 / (n * n)
    assert (rec["ix"], rec["iy"]) == (5, 3)
    assert abs(rec["dx"] - (5 + (0.5 - mu) / (1.5 - 2 * mu))) < 1e-14
    assert rec["dy"] == 3
    # symmetric neighbourhood -> integer centroid; wrap of indices >= N/2
    c = np.zeros((n, n))
    c[8, 15] = 2.0
    c[8, 14] = c[8, 0] = 0.7
    c[7, 15] = c[9, 15] = 0.4
    rec = O.peak_stats(c)
    assert (rec["sx"], rec["sy"]) == (-1, -8)
    assert abs(rec["dx"] + 1) < 1e-14 and abs(rec["dy"] + 8) < 1e-14


def test_argmax_first_occurrence_and_near_tie():
    c = np.zeros((8, 8))
    c[2, 3] = 1.0
    c[5, 1] = 1.0
    rec = O.peak_stats(c)
    assert (rec["iy"], rec["ix"]) == (2, 3)
    assert rec["status"] & STATUS_NEAR_TIE


def test_search_window_brute_force_and_decoy():
    # the windowed peak is the first row-major maximum among the entries with
    # wrapped |sx|, |sy| <= r (brute force over the window), the background
    # stays the whole surface, and a stronger decoy outside the window loses
    rng = np.random.default_rng(17)
    n, r = 32, 5
    c = rng.normal(0, 1, (n, n))
    c[3, n - 2] = 9.0    # inside: shift (-2, 3)
    c[12, 20] = 15.0     # outside
    full = O.peak_stats(c)
    assert (full["iy"], full["ix"]) == (12, 20)
    win = O.peak_stats(c, max_shift=r)
    best, arg = -np.inf, None
    for iy in range(n):
        for ix in range(n):
            sy = iy - n if iy >= n // 2 else iy
            sx = ix - n if ix >= n // 2 else ix
            if abs(sx) <= r and abs(sy) <= r and c[iy, ix] > best:
                best, arg = c[iy, ix], (iy, ix)
    assert (win["iy"], win["ix"]) == arg == (3, n - 2)
    assert (win["sx"], win["sy"]) == (-2, 3)
    assert win["mean"] == full["mean"] and win["std"] == full["std"]
    assert win["snr"] == (9.0 - full["mean"]) / full["std"]
    # the near-tie test compares within the window only
    c2 = c.copy()
    c2[n - 1, 1] = 9.0
    assert O.peak_stats(c2, max_shift=r)["status"] & STATUS_NEAR_TIE
    assert not (O.peak_stats(c2)["status"] & STATUS_NEAR_TIE)
    # radius 0 and radii of half the surface or more search everything
    for rr in (0, n // 2, n):
        assert (O.peak_stats(c, max_shift=rr)["iy"], O.peak_stats(c, max_shift=rr)["ix"]) == (12, 20)
    # a window of radius r holds (2r + 1)^2 entries
    assert O.swift_oracle.search_mask(n, r).sum() == (2 * r + 1) ** 2


# ---------------------------------------------------------------- qualitative claim (Fig. 2)
def test_mid_whitening_beats_extremes_on_distorted_pair():
    """Section III / Fig. 2: an intermediate exponent gives a higher SNR than
    both plain correlation and phase-only correlation on distorted content."""
    import torch
    from datagen import make_section, warp_affine
    a = make_section(320, 320, seed=21).float()
    m = np.array([[math.cos(0.03), -math.sin(0.03)], [math.sin(0.03), math.cos(0.03)]]) * 1.01
    cen = np.array([159.5, 159.5])
    b = warp_affine(a, m, cen - m @ cen + np.array([3.3, -2.2]))
    g = torch.Generator().manual_seed(5)
    b = (b + 10 * torch.randn(b.shape, generator=g)).clamp(0, 255).numpy()
    a = a.numpy()
    th = ident(160, 160)
    snr = {p: O.match_pair(a, b, th, th, 256, O.Params(p=p))["snr"] for p in (0.0, 0.65, 1.0)}
    assert snr[0.65] > snr[0.0] and snr[0.65] > snr[1.0], snr


# ---------------------------------------------------------------- projection / pyramid
def _proj_bruteforce(stack, s, k, exclude):
    S = stack.shape[0]
    out = np.zeros(stack.shape[1:], np.uint8)
    for y in range(stack.shape[1]):
        for x in range(stack.shape[2]):
            vals = [int(stack[j, y, x]) for j in range(S)
                    if 1 <= abs(j - s) <= k and not exclude[j]]
            q = Fraction(sum(vals), len(vals))
            out[y, x] = math.floor(q + Fraction(1, 2))
    return out


def test_projection_bit_exact_vs_bruteforce():
    rng = np.random.default_rng(12)
    st = rng.integers(0, 256, size=(9, 6, 7)).astype(np.uint8)
    excl = np.zeros(9, bool)
    excl[5] = True
    for s in range(9):
        for k in (1, 3):
            np.testing.assert_array_equal(O.project(st, s, k, excl), _proj_bruteforce(st, s, k, excl))


def test_projection_noise_reduction_inv_sqrt_n():
    # Section III: averaging n sections reduces independent noise as 1/sqrt(n)
    rng = np.random.default_rng(13)
    st = np.clip(rng.normal(128, 20, size=(7, 256, 256)), 0, 255).round().astype(np.uint8)
    r = O.project(st, 3, 3).astype(np.float64)
    ratio = r.std() / st[3].astype(np.float64).std()
    assert abs(ratio - 1 / math.sqrt(6)) < 0.03


def test_pyramid_bit_exact_vs_bruteforce():
    rng = np.random.default_rng(14)
    img = rng.integers(0, 256, size=(9, 11)).astype(np.uint8)
    p = O.pyramid(img)
    assert p.shape == (4, 5)
    for y in range(4):
        for x in range(5):
            s = sum(int(img[2 * y + a, 2 * x + b]) for a in (0, 1) for b in (0, 1))
            assert p[y, x] == math.floor(Fraction(s, 4) + Fraction(1, 2))


# ---------------------------------------------------------------- affine LSQ
def test_fit_affine_recovers_exact_affine():
    rng = np.random.default_rng(15)
    A = np.array([[1.01, 0.02, 3.0], [-0.01, 0.99, -4.0]])
    src = rng.uniform(0, 1000, (64, 2))
    dst = src @ A[:, :2].T + A[:, 2]
    np.testing.assert_allclose(O.fit_affine(src, dst, rng.uniform(1, 5, 64)), A, atol=1e-9)


# ---------------------------------------------------------------- adjoint vs finite differences
def _smooth_img(h, w, seed):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    return gaussian_filter(rng.uniform(0, 255, (h, w)), 1.5) * 3 - 200


@pytest.mark.parametrize("p,eps", [(0.65, 1e-2), (0.0, 1e-4), (1.0, 1e-2), (0.4, 0.0)])
def test_adjoint_matches_central_fd(p, eps):
    n = 16
    img = _smooth_img(48, 48, 16)
    imgB = np.roll(img, (1, -2), axis=(0, 1)) + _smooth_img(48, 48, 17) * 0.05
    thA = np.array([24.0, 23.0, 1.0013, 0.0021, 0.3, -0.0017, 0.9988, 0.27])
    thB = np.array([24.0, 23.0, 0.9991, -0.0012, 0.61, 0.0008, 1.0011, 0.58])
    par = O.Params(p=p, eps_rel=eps, taper_frac=0.5)
    for gp, gs in ((0.0, 1.0), (1.0, 0.0), (0.3, -0.7)):
        rec, gA, gB = O.match_grad(img, imgB, thA, thB, n, par, g_peak=gp, g_snr=gs)
        idx = [2, 3, 4, 5, 6, 7]
        h = 1e-6
        for which, th, g in (("A", thA, gA), ("B", thB, gB)):
            fd = np.zeros(6)
            for q in range(6):
                tp = th.copy()
                tm = th.copy()
                tp[idx[q]] += h
                tm[idx[q]] -= h
                if which == "A":
                    rp = O.match_pair(img, imgB, tp, thB, n, par, return_surface=True)
                    rm = O.match_pair(img, imgB, tm, thB, n, par, return_surface=True)
                else:
                    rp = O.match_pair(img, imgB, thA, tp, n, par, return_surface=True)
                    rm = O.match_pair(img, imgB, thA, tm, n, par, return_surface=True)
                # hold the argmax fixed: evaluate the objective at rec's s*
                def J(r):
                    cc = r["surface"]
                    pk = cc[rec["iy"], rec["ix"]]
                    return gp * pk + gs * (pk - cc.mean()) / cc.std()
                fd[q] = (J(rp) - J(rm)) / (2 * h)
            err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
            assert err < 1e-5, (which, p, eps, gp, gs, err, g, fd)


# ---------------------------------------------------------------- curvature and refinement steps
def test_peak_curvature_exact_on_quadratic():
    # second differences are exact for a quadratic surface around the peak
    n = 16
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    X, Y = xx - 5, yy - 7
    c = 10 - (0.8 * X * X + 0.3 * X * Y + 0.5 * Y * Y)
    rec = O.peak_stats(c)
    assert (rec["ix"], rec["iy"]) == (5, 7)
    assert abs(rec["hxx"] + 1.6) < 1e-12 and abs(rec["hyy"] + 1.0) < 1e-12 and abs(rec["hxy"] + 0.3) < 1e-12


def test_newton_step_is_exact_for_linear_centroid():
    # d(t) = J (t - t*): one Newton step from anywhere lands on t*
    J = np.array([[0.29, -0.02], [0.03, 0.31]])
    tstar = np.array([0.23, -0.31])
    t0 = np.array([-0.1, 0.15])
    d = J @ (t0 - tstar)
    rec = dict(dx=d[0], dy=d[1], sx=0, sy=0, status=0)
    jac = np.zeros((2, 6))
    jac[:, 2] = J[:, 0]
    jac[:, 5] = J[:, 1]
    th = np.array([10, 10, 1, 0, t0[0], 0, 1, t0[1]])
    th2, ln = O.refine_step(rec, th, "newton", jac=jac, max_step=5.0)
    np.testing.assert_allclose(th2[[4, 7]], tstar, atol=1e-12)
    assert abs(ln - np.hypot(*(tstar - t0))) < 1e-12
    # a singular Jacobian falls back to the centroid step
    th3, _ = O.refine_step(rec, th, "newton", jac=np.zeros((2, 6)), max_step=5.0)
    np.testing.assert_allclose(th3[[4, 7]], t0 - d, atol=1e-15)
    # the integer peak one cell off: d = s + J (t - t* - s) within that cell,
    # and the step s + J^-1 (d - s) lands on t* even with max_step below |s|
    t1 = np.array([0.8, -0.6])
    s_ = np.array([1.0, -1.0])
    d1 = s_ + J @ (t1 - s_)  # t1 is the offset t - t*
    rec1 = dict(dx=d1[0], dy=d1[1], sx=1, sy=-1, status=0)
    th1 = np.array([10, 10, 1, 0, t1[0] + tstar[0], 0, 1, t1[1] + tstar[1]])
    th4, _ = O.refine_step(rec1, th1, "newton", jac=jac, max_step=0.5)
    np.testing.assert_allclose(th4[[4, 7]], tstar + 0.0, atol=1e-12)
    # two cells off: the centroid step, clamped
    th5, ln5 = O.refine_step(dict(rec1, sx=2, dx=2.1), th1, "newton", jac=jac, max_step=0.5)
    assert abs(ln5 - 0.5) < 1e-12


def test_centroid_step_and_clamp():
    rec = dict(dx=0.3, dy=-0.4, sx=0, sy=0, status=0, hxx=-1, hyy=-1, hxy=0)
    th = np.zeros(8)
    th2, ln = O.refine_step(rec, th, "centroid")
    assert (th2[4], th2[7], ln) == (-0.3, 0.4, 0.5)
    th3, ln = O.refine_step(dict(rec, dx=3.0, dy=4.0), th, "centroid", max_step=1.0)
    np.testing.assert_allclose([th3[4], th3[7], ln], [-0.6, -0.8, 1.0])
    # a peak away from the origin takes the centroid (integer) step even in Newton mode
    th4, _ = O.refine_step(dict(rec, sx=2, dx=2.1), th, "newton", jac=np.eye(2, 6, 2), max_step=5.0)
    assert th4[4] == -2.1


def test_surface_hessian_of_trigonometric_surface():
    # closed form: second derivatives of a sum of plane waves
    n = 32
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    w1 = 2 * np.pi * np.array([3, 2]) / n      # (x, y) frequencies
    w2 = 2 * np.pi * np.array([-5, 1]) / n
    c = np.cos(w1[0] * xx + w1[1] * yy) + 0.5 * np.sin(w2[0] * xx + w2[1] * yy)
    x0, y0 = 7, 11
    p1 = w1[0] * x0 + w1[1] * y0
    p2 = w2[0] * x0 + w2[1] * y0
    hxx = -w1[0] ** 2 * np.cos(p1) - 0.5 * w2[0] ** 2 * np.sin(p2)
    hyy = -w1[1] ** 2 * np.cos(p1) - 0.5 * w2[1] ** 2 * np.sin(p2)
    hxy = -w1[0] * w1[1] * np.cos(p1) - 0.5 * w2[0] * w2[1] * np.sin(p2)
    got = O.surface_hessian(c, y0, x0)
    np.testing.assert_allclose(got, [hxx, hyy, hxy], atol=1e-12)


def test_centroid_jacobian_matches_central_fd():
    # d(dx, dy)/d theta_A with the integer peak and the positive-weight set
    # held fixed, against central differences of the oracle's own centroid
    n = 16
    img = _smooth_img(48, 48, 16)
    imgB = np.roll(img, (1, -2), axis=(0, 1)) + _smooth_img(48, 48, 17) * 0.05
    thA = np.array([24.0, 23.0, 1.0013, 0.0021, 0.3, -0.0017, 0.9988, 0.27])
    thB = np.array([24.0, 23.0, 0.9991, -0.0012, 0.61, 0.0008, 1.0011, 0.58])
    for p in (0.65, 0.0, 1.0):
        par = O.Params(p=p, eps_rel=1e-2, taper_frac=0.5)
        rec, jac = O.centroid_jacobian(img, imgB, thA, thB, n, par)
        idx = [2, 3, 4, 5, 6, 7]
        h = 1e-6
        fd = np.zeros((2, 6))
        for q in range(6):
            tp, tm = thA.copy(), thA.copy()
            tp[idx[q]] += h
            tm[idx[q]] -= h
            rp = O.match_pair(img, imgB, tp, thB, n, par)
            rm = O.match_pair(img, imgB, tm, thB, n, par)
            assert (rp["ix"], rp["iy"]) == (rm["ix"], rm["iy"]) == (rec["ix"], rec["iy"])
            fd[0, q] = (rp["dx"] - rm["dx"]) / (2 * h)
            fd[1, q] = (rp["dy"] - rm["dy"]) / (2 * h)
        err = np.linalg.norm(jac - fd) / np.linalg.norm(fd)
        assert err < 1e-5, (p, err, jac, fd)
        # the translation block is far from zero (the Newton system is well posed)
        assert abs(np.linalg.det(jac[:, [2, 5]])) > 1e-3


# ---------------------------------------------------------------- stack loop: levels, render, windows, fit
def test_level_coordinates_match_the_pyramid_of_a_ramp():
    # the 2 x 2 box mean of a linear ramp is the ramp at the block centre, so the
    # x2 pyramid of an integer ramp is the ramp at level_to_base, rounded half up
    yy, xx = np.mgrid[0:64, 0:96].astype(np.int64)
    ramp = (xx + 2 * yy + 7).astype(np.uint8)  # stays below 256
    lvl = ramp
    for level in (1, 2):
        lvl = O.pyramid(lvl)
        h, w = lvl.shape
        y1, x1 = np.mgrid[0:h, 0:w].astype(np.float64)
        exact = O.level_to_base(x1, level) + 2 * O.level_to_base(y1, level) + 7
        np.testing.assert_array_equal(lvl, np.floor(exact + 0.5).astype(np.uint8))
    np.testing.assert_allclose(O.base_to_level(O.level_to_base(np.arange(5.0), 3), 3), np.arange(5.0))


def test_render_identity_and_integer_translation():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (40, 56)).astype(np.uint8)
    out = O.render(img, [1, 0, 0, 0, 1, 0], 0, 40, 56)
    np.testing.assert_array_equal(out, img)
    # q = p + (3, -2): out[y][x] = img[clamp(y - 2)][clamp(x + 3)]
    out = O.render(img, [1, 0, 3, 0, 1, -2], 0, 40, 56)
    yy, xx = np.mgrid[0:40, 0:56]
    np.testing.assert_array_equal(out, img[np.clip(yy - 2, 0, 39), np.clip(xx + 3, 0, 55)])
    # at level 2 a level-0 translation of (8, -4) moves level-2 pixels by (2, -1)
    out = O.render(img, [1, 0, 8, 0, 1, -4], 2, 40, 56)
    np.testing.assert_array_equal(out, img[np.clip(yy - 1, 0, 39), np.clip(xx + 2, 0, 55)])


def test_render_reproduces_an_affine_ramp():
    # bilinear interpolation is exact on a linear ramp, so rendering a ramp by
    # any affine gives the ramp at the mapped points (rounded half up)
    yy, xx = np.mgrid[0:80, 0:80].astype(np.float64)
    img = (40 + xx + 1.0 * yy).astype(np.uint8)
    aff = [0.999, 0.012, 3.37, -0.011, 1.002, 2.71]
    out = O.render(img, aff, 0, 60, 60).astype(np.int64)
    y1, x1 = np.mgrid[0:60, 0:60].astype(np.float64)
    qx, qy = O.apply_affine(aff, x1, y1)
    exact = 40 + qx + qy
    ref = np.floor(exact + 0.5)
    safe = np.abs(exact - np.floor(exact) - 0.5) > 1e-6
    np.testing.assert_array_equal(out[safe], ref[safe])


def test_render_matches_scipy_map_coordinates():
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (50, 70)).astype(np.float64)
    aff = [1.01, -0.02, 1.3, 0.015, 0.99, -2.2]
    for level in (0, 1):
        out = O.render(img.astype(np.uint8), aff, level, 45, 66)
        y1, x1 = np.mgrid[0:45, 0:66].astype(np.float64)
        qx, qy = O.apply_affine(aff, O.level_to_base(x1, level), O.level_to_base(y1, level))
        v = map_coordinates(img, [O.base_to_level(qy, level), O.base_to_level(qx, level)], order=1, mode="nearest")
        np.testing.assert_array_equal(out, np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8))


def test_stack_windows_and_correspondence():
    ta, tb = O.stack_windows([1, 0, 0, 0, 1, 0], 1, 64, 4, 256, 256)
    np.testing.assert_array_equal(ta, tb)
    assert tuple(tb[5, :2]) == (96, 96)
    # a level-0 translation (8, -6) shifts level-1 raw centres by (4, -3)
    ta, tb = O.stack_windows([1, 0, 8, 0, 1, -6], 1, 64, 4, 256, 256)
    np.testing.assert_allclose(ta[:, 0] + ta[:, 4] - tb[:, 0], 4.0)
    np.testing.assert_allclose(ta[:, 1] + ta[:, 7] - tb[:, 1], -3.0)
    # fractional centres: rounded part plus remainder
    ta, _ = O.stack_windows([1.001, 0, 0.3, 0, 1, 0.2], 0, 64, 4, 256, 256)
    assert np.all(np.abs(ta[:, 4]) <= 0.5) and np.all(ta[:, 0] == np.rint(ta[:, 0]))
    # correspondence at level 1: model centre p, raw point = A's centre - L d
    p, q = O.correspondence([100, 50, 1, 0, 0.25, 0, 1, -0.5], [96, 52, 1, 0, 0, 0, 1, 0], 1.0, 2.0, 1)
    np.testing.assert_allclose(p, (2 * 96 + 0.5, 2 * 52 + 0.5))
    np.testing.assert_allclose(q, (2 * (100.25 - 1.0) + 0.5, 2 * (49.5 - 2.0) + 0.5))


def test_fit_section_exact_and_singular():
    rng = np.random.default_rng(21)
    A = np.array([1.002, -0.003, 4.5, 0.001, 0.998, -7.25])
    p = rng.uniform(0, 4096, (64, 2))
    q = np.stack(O.apply_affine(A, p[:, 0], p[:, 1]), 1)
    w = rng.uniform(5, 40, 64)
    aff, st = O.fit_section(p, q, w, np.zeros(6))
    assert st == 0
    np.testing.assert_allclose(aff, A, rtol=0, atol=1e-9)
    # two weighted points, and collinear points, keep the previous affine
    prev = np.array([1, 0, 1, 0, 1, 2.0])
    w2 = np.zeros(64)
    w2[:2] = 1
    assert O.fit_section(p, q, w2, prev)[1] == O.swift_oracle.STACK_FIT_SINGULAR
    pl = np.stack([np.linspace(0, 100, 64), np.linspace(0, 50, 64)], 1)
    aff, st = O.fit_section(pl, pl, np.ones(64), prev)
    assert st == O.swift_oracle.STACK_FIT_SINGULAR and np.array_equal(aff, prev)
    assert O.match_weight(20.0, 0, 6.0) == 20.0 and O.match_weight(5.0, 0, 6.0) == 0.0
    assert O.match_weight(20.0, O.swift_oracle.STATUS_DEGENERATE, 6.0) == 0.0


# --------------------------------------------------------------------------- local-affine mesh
def _orient(a, b, c):
    """Twice the signed area of triangle (a, b, c), exact on integers."""
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def test_mesh_triangles_tile_the_hull():
    grid, h, w = 6, 47, 61
    nodes = O.mesh_node_xy(grid, h, w)
    tris = O.mesh_triangles(grid)
    sx, sy = w // grid, h // grid
    areas = np.array([_orient(*nodes[t]) for t in tris])
    # every triangle is half a cell, all with one orientation, and they add up to the hull
    assert np.all(areas == areas[0]) and abs(int(areas[0])) == sx * sy
    hull = (nodes[:, 0].max() - nodes[:, 0].min()) * (nodes[:, 1].max() - nodes[:, 1].min())
    assert abs(int(areas.sum())) == 2 * hull


def test_mesh_triangle_of_matches_orientation_tests():
    # the integer rule against containment by orientation signs: every pixel in
    # the hull lies in its triangle, and a pixel strictly inside one triangle
    # lies in no other; outside the hull, the clamped cell and the side of its
    # diagonal decide
    grid, h, w = 5, 47, 61
    nodes = O.mesh_node_xy(grid, h, w)
    tris = O.mesh_triangles(grid)
    yy, xx = np.mgrid[0:h, 0:w]
    t = O.mesh_triangle_of(xx, yy, grid, h, w)
    sgn = np.sign(_orient(*nodes[tris[0]]))
    sx, sy = w // grid, h // grid
    for y in range(h):
        for x in range(w):
            p = (x, y)
            o = [sgn * _orient(nodes[tris[t[y, x]]][a], nodes[tris[t[y, x]]][(a + 1) % 3], p) for a in range(3)]
            in_hull = nodes[0, 0] <= x <= nodes[-1, 0] and nodes[0, 1] <= y <= nodes[-1, 1]
            if in_hull:
                assert min(o) >= 0, (x, y)
                if min(o) > 0:
                    others = [k for k, tri in enumerate(tris)
                              if k != t[y, x] and min(sgn * _orient(nodes[tri][a], nodes[tri][(a + 1) % 3], p)
                                                      for a in range(3)) >= 0]
                    assert others == [], (x, y, others)
            ci = min(max((x - sx // 2) // sx, 0), grid - 2)
            cj = min(max((y - sy // 2) // sy, 0), grid - 2)
            assert t[y, x] // 2 == cj * (grid - 1) + ci
            k00 = cj * grid + ci
            d0, d1 = nodes[k00 + 1], nodes[k00 + grid]
            first = np.sign(_orient(d0, d1, p)) in (0, np.sign(_orient(d0, d1, nodes[k00])))
            assert t[y, x] % 2 == (0 if first else 1), (x, y)


def test_mesh_band_is_the_vertex_one_ring():
    # the band is the set of vertices of every triangle touching t (brute force)
    grid = 6
    tris = O.mesh_triangles(grid)
    for t in range(len(tris)):
        touch = [tri for tri in tris if set(tri) & set(tris[t])]
        ref = sorted(set(int(v) for tri in touch for v in tri))
        assert O.mesh_band(grid, t).tolist() == ref
    # interior triangles see twelve points, the corner triangle at the origin six
    assert len(O.mesh_band(grid, 2 * (2 * (grid - 1) + 2))) == 12
    assert len(O.mesh_band(grid, 2 * (2 * (grid - 1) + 2) + 1)) == 12
    assert len(O.mesh_band(grid, 0)) == 6


def test_fit_mesh_exact_on_piecewise_affine_points():
    # nodes in columns i <= 2 follow A1, columns i >= 3 follow A2.  A triangle of
    # cell ci reaches columns ci-1 .. ci+2 through its band, so cell 0 fits A1
    # exactly, cells >= 4 fit A2 exactly, and the cells between mix the two.
    grid, h, w, level = 7, 700, 840, 0
    nodes = O.mesh_node_xy(grid, h, w).astype(np.float64)
    A1 = np.array([1.001, -0.002, 3.5, 0.0015, 0.999, -2.25])
    A2 = np.array([0.997, 0.003, -4.0, -0.001, 1.002, 6.5])
    col = np.arange(grid * grid) % grid
    q = np.where((col <= 2)[:, None], np.stack(O.apply_affine(A1, nodes[:, 0], nodes[:, 1]), 1),
                 np.stack(O.apply_affine(A2, nodes[:, 0], nodes[:, 1]), 1))
    rng = np.random.default_rng(4)
    wts = rng.uniform(6, 40, grid * grid)
    # an outlier of weight 0 changes nothing
    q[3 * grid + 5] += 50.0
    wts[3 * grid + 5] = 0.0
    sec = np.array([1, 0, 0, 0, 1, 0.0])
    tri, st = O.fit_mesh(nodes, q, wts, grid, sec)
    assert np.all(st == 0)
    for t in range(len(tri)):
        ci = (t // 2) % (grid - 1)
        if ci == 0:
            np.testing.assert_allclose(tri[t], A1, rtol=0, atol=1e-9)
        elif ci >= 4:
            np.testing.assert_allclose(tri[t], A2, rtol=0, atol=1e-9)
        else:
            assert not np.allclose(tri[t], A1, atol=1e-6) and not np.allclose(tri[t], A2, atol=1e-6)
    # no weighted points in the top-left corner: those triangles keep the section's affine
    w0 = wts.copy()
    for j in range(3):
        for i in range(3):
            w0[j * grid + i] = 0.0
    tri, st = O.fit_mesh(nodes, q, w0, grid, sec)
    assert st[0] == O.swift_oracle.MESH_FIT_SINGULAR and np.array_equal(tri[0], sec)
    assert np.all(st[2 * (grid - 1) * 4:] == 0)


@pytest.mark.parametrize("level", [0, 1])
def test_render_mesh_reduces_to_render(level):
    rng = np.random.default_rng(12 + level)
    img = rng.integers(0, 256, (70, 90)).astype(np.uint8)
    A = [1.004, -0.01, 2.6, 0.008, 0.995, -1.7]
    grid = 4
    T = 2 * (grid - 1) ** 2
    out = O.render_mesh(img, np.tile(A, (T, 1)), level, grid, 64, 88)
    np.testing.assert_array_equal(out, O.render(img, A, level, 64, 88))
    # distinct affines: each pixel is the plain render by its own triangle's affine
    tri = np.tile(A, (T, 1)) + rng.uniform(-0.5, 0.5, (T, 6)) * [0.01, 0.01, 3, 0.01, 0.01, 3]
    out = O.render_mesh(img, tri, level, grid, 64, 88)
    yy, xx = np.mgrid[0:64, 0:88]
    t = O.mesh_triangle_of(xx, yy, grid, 64, 88)
    for k in range(T):
        ref = O.render(img, tri[k], level, 64, 88)
        np.testing.assert_array_equal(out[t == k], ref[t == k])


def test_mesh_windows_reduce_to_stack_windows():
    grid, level, h, w = 4, 1, 256, 320
    A = np.array([1.002, 0.001, 8.3, -0.002, 0.999, -5.6])
    T = 2 * (grid - 1) ** 2
    ta, tb = O.mesh_windows(np.tile(A, (T, 1)), level, 64, grid, h, w)
    ra, rb = O.stack_windows(A, level, 64, grid, h, w)
    np.testing.assert_array_equal(ta, ra)
    np.testing.assert_array_equal(tb, rb)
    # distinct affines: node (i, j) reads through the first triangle of its
    # cell, the last row and column through the cells before them
    rng = np.random.default_rng(2)
    tri = np.tile(A, (T, 1)) + rng.uniform(-1, 1, (T, 6)) * [0.001, 0.001, 2, 0.001, 0.001, 2]
    ta, _ = O.mesh_windows(tri, level, 64, grid, h, w)
    for j in range(grid):
        for i in range(grid):
            ci, cj = min(i, grid - 2), min(j, grid - 2)
            t = 2 * (cj * (grid - 1) + ci) + (1 if (i == grid - 1 and j == grid - 1) else 0)
            k = j * grid + i
            np.testing.assert_array_equal(ta[k, [2, 3, 5, 6]], tri[t, [0, 1, 3, 4]])


# --------------------------------------------------------------------------- Pearson-normalised correlation
def test_pearson_matches_numpy_corrcoef():
    rng = np.random.default_rng(41)
    for n in (16, 32):
        a = rng.normal(0, 1, (n, n))
        f = rng.normal(0, 1, (n, n))
        g, st = O.pearson_surface(a, f)
        m, c0, R = n // 2, n // 4, n // 4
        t = a[c0:c0 + m, c0:c0 + m].ravel()
        for sy in range(-R, R + 1):
            for sx in range(-R, R + 1):
                p = f[c0 + sy:c0 + sy + m, c0 + sx:c0 + sx + m].ravel()
                assert abs(g[sy + R, sx + R] - np.corrcoef(t, p)[0, 1]) < 1e-12
        assert abs(st - np.sum((t - t.mean()) ** 2)) < 1e-9


def test_pearson_equals_fft_correlation_with_cumulative_area_correction():
    # Section II: an FFT correlation becomes the Pearson coefficient after a
    # cumulative-area correction.  Numerator: circular correlation of the
    # zero-padded, mean-free template with the window; denominator: the
    # patch energies from summed-area tables of f and f^2.
    rng = np.random.default_rng(42)
    n = 32
    m, c0, R = n // 2, n // 4, n // 4
    a = rng.integers(0, 256, (n, n)).astype(np.float64)
    f = rng.integers(0, 256, (n, n)).astype(np.float64)
    g, _ = O.pearson_surface(a, f)
    tz = np.zeros((n, n))
    t = a[c0:c0 + m, c0:c0 + m]
    tz[c0:c0 + m, c0:c0 + m] = t - t.mean()
    c = np.real(np.fft.ifft2(np.conj(np.fft.fft2(tz)) * np.fft.fft2(f)))
    sat1 = np.zeros((n + 1, n + 1))
    sat2 = np.zeros((n + 1, n + 1))
    sat1[1:, 1:] = np.cumsum(np.cumsum(f, 0), 1)
    sat2[1:, 1:] = np.cumsum(np.cumsum(f * f, 0), 1)

    def box(S, y, x):
        return S[y + m, x + m] - S[y, x + m] - S[y + m, x] + S[y, x]

    st = np.sum(tz * tz)
    for sy in range(-R, R + 1):
        for sx in range(-R, R + 1):
            y, x = c0 + sy, c0 + sx
            e1, e2 = box(sat1, y, x), box(sat2, y, x)
            v = e2 - e1 * e1 / (m * m)
            ref = c[sy % n, sx % n] / np.sqrt(st * v)
            assert abs(g[sy + R, sx + R] - ref) < 1e-9


def test_pearson_exact_shift_sign_and_invariance():
    rng = np.random.default_rng(43)
    img = rng.integers(0, 256, (200, 200)).astype(np.float64)
    n = 64
    thA = np.array([100, 100, 1, 0, 0, 0, 1, 0], np.float64)
    # window B sits 5 px right and 3 px up: its content is A's moved by d = (-5, 3)
    thB = np.array([105, 97, 1, 0, 0, 0, 1, 0], np.float64)
    r = O.pearson_pair(img, img, thA, thB, n, return_surface=True)
    assert (r["sx"], r["sy"]) == (-5, 3) and abs(r["peak"] - 1.0) < 1e-12
    assert abs(r["dx"] + 5) < 0.5 and abs(r["dy"] - 3) < 0.5 and r["snr"] > 10
    g = r["surface"]
    assert np.all(np.abs(g) <= 1 + 1e-12)
    # an affine intensity map of either image leaves every coefficient unchanged,
    # a negative one flips the sign
    r2 = O.pearson_pair(img, 3.5 * img - 40, thA, thB, n, return_surface=True)
    np.testing.assert_allclose(r2["surface"], g, atol=1e-12)
    r3 = O.pearson_pair(img, 255 - img, thA, thB, n, return_surface=True)
    np.testing.assert_allclose(r3["surface"], -g, atol=1e-12)
    assert abs(r3["surface"][3 + n // 4, -5 + n // 4] + 1.0) < 1e-12
    # a constant window is degenerate
    r4 = O.pearson_pair(np.full((200, 200), 9.0), img, thA, thB, n)
    assert r4["status"] & STATUS_DEGENERATE and r4["snr"] == 0.0


# --------------------------------------------------------------------------- jump repair
def test_pearson_peak_record_closed_form():
    """Hand-built 5 x 5 placement grid (n = 8, range R = n/4 = 2): peak 1 at
    the range corner (sy, sx) = (2, 2), 0.5 at (1, 2) and (2, 1), 0.25 at
    (1, 1), and 0.8 at (-2, -2), the entry a wrapped neighbour (sy or sx = 3)
    would read.  Over the 25 placements: mean 3.05 / 25 = 0.122, population
    variance sum g^2 / 25 - mean^2 = 2.2025 / 25 - 0.122^2 (ddof 0, not 1),
    SNR (1 - mean) / sigma.  The 3 x 3 centroid uses only the four
    neighbours inside the range, weights g - mean."""
    n, R = 8, 2
    g = np.zeros((2 * R + 1, 2 * R + 1))

    def put(sy, sx, v):
        g[sy + R, sx + R] = v

    put(2, 2, 1.0)
    put(1, 2, 0.5)
    put(2, 1, 0.5)
    put(1, 1, 0.25)
    put(-2, -2, 0.8)
    rec = O.pearson_peak(g, n, st=1.0)
    mu = 3.05 / 25.0
    var = 2.2025 / 25.0 - mu * mu
    assert (rec["ix"], rec["iy"], rec["sx"], rec["sy"]) == (2, 2, 2, 2)
    assert abs(rec["mean"] - mu) < 1e-15
    assert abs(rec["std"] - math.sqrt(var)) < 1e-15
    assert abs(rec["snr"] - (1.0 - mu) / math.sqrt(var)) < 1e-13
    w11, w12, w21, w22 = 0.25 - mu, 0.5 - mu, 0.5 - mu, 1.0 - mu
    sw = w11 + w12 + w21 + w22
    assert abs(rec["dx"] - (2 + (-w11 - w21) / sw)) < 1e-15
    assert abs(rec["dy"] - (2 + (-w11 - w12) / sw)) < 1e-15
    assert rec["status"] == 0


def test_pearson_peak_tie_order_and_degenerate():
    """Equal best coefficients at sy = -1 and sy = +1 (sx = 0): the wrapped
    row of sy = -1 is n - 1, so the row-major first maximum is sy = +1 and the
    near-tie bit is set.  A zero template energy is degenerate."""
    n, R = 16, 4
    g = np.full((2 * R + 1, 2 * R + 1), 0.1)
    g[-1 + R, R] = 0.9
    g[1 + R, R] = 0.9
    rec = O.pearson_peak(g, n, st=2.0)
    assert (rec["sx"], rec["sy"], rec["iy"]) == (0, 1, 1)
    assert rec["status"] & STATUS_NEAR_TIE
    deg = O.pearson_peak(g, n, st=0.0)
    assert deg["status"] & STATUS_DEGENERATE and deg["snr"] == 0.0
    flat = O.pearson_peak(np.full((2 * R + 1, 2 * R + 1), 0.3), n, st=2.0)
    assert flat["status"] & STATUS_DEGENERATE and flat["std"] == 0.0


def test_one_sided_models_brute_force():
    rng = np.random.default_rng(51)
    st = rng.integers(0, 256, (9, 5, 7)).astype(np.uint8)
    excl = np.zeros(9, bool)
    excl[3] = True
    for s in range(9):
        for side in (-1, 1):
            J = [j for j in range(9) if (0 < (s - j) <= 3 if side < 0 else 0 < (j - s) <= 3) and not excl[j]]
            got = O.project_side(st, s, 3, side, excl)
            if not J:
                assert not got.any()
                continue
            mean = st[J].astype(np.float64).mean(0)
            np.testing.assert_array_equal(got, np.floor(mean + 0.5).astype(np.uint8))
        # the two sides together hold the two-sided model's neighbours
        left = [j for j in range(max(0, s - 3), s) if not excl[j]]
        right = [j for j in range(s + 1, min(9, s + 4)) if not excl[j]]
        if left or right:
            both = np.floor(st[left + right].astype(np.float64).mean(0) + 0.5).astype(np.uint8)
            np.testing.assert_array_equal(O.project(st, s, 3, excl), both)


def test_span_blend_is_the_cubic_bezier():
    def casteljau(t, c):
        c = list(c)
        while len(c) > 1:
            c = [(1 - t) * c[i] + t * c[i + 1] for i in range(len(c) - 1)]
        return c[0]
    for a, b in ((4, 4), (2, 5), (0, 9)):
        for s in range(a, b + 1):
            t = (s - a + 1) / (b - a + 2)
            assert abs(O.span_weight(s, a, b) - casteljau(t, (0, 0, 1, 1))) < 1e-15
    # symmetric about the middle of the span, zero slope at its ends
    assert abs(O.span_weight(2, 2, 4) + O.span_weight(4, 2, 4) - 1) < 1e-15
    h = 1e-6
    w = lambda t: 3 * t * t - 2 * t ** 3  # noqa: E731
    assert abs((w(h) - w(0)) / h) < 1e-5 and abs((w(1) - w(1 - h)) / h) < 1e-5
    L = np.tile([1, 0, 2, 0, 1, -1.0], (10, 1))
    R = np.tile([1.01, 0, -3, 0, 0.99, 4.0], (10, 1))
    out = O.blend_span(L, R, 3, 5)
    assert out.shape == (3, 6)
    # entries move monotonically from the left fit toward the right fit
    assert np.all(np.diff(out[:, 2]) < 0) and np.all(np.diff(out[:, 5]) > 0)
    np.testing.assert_allclose(out[1], 0.5 * (L[4] + R[4]), atol=1e-15)


def test_failed_spans_runs():
    snr = [30, 31, 29, 8, 7, 30, 32, 10, 31]
    assert O.failed_spans(snr, 0.5) == [(3, 4), (7, 7)]
    assert O.failed_spans([20] * 5, 0.5) == []
    # an even count: the median is the midpoint of the two middle values (25,
    # threshold 12.5), not the lower one (20, threshold 10)
    assert O.failed_spans([10, 20, 30, 40], 0.5) == [(0, 0)]


def test_break_score_closed_forms():
    rng = np.random.default_rng(62)
    c = rng.uniform(0, 4096, (64, 2))
    aff = np.array([1.001, -0.002, 3.0, 0.0015, 0.999, -4.0])
    # a fit that only translates: every centre moves by (dx, dy)
    fit = aff + np.array([0, 0, 1.5, 0, 0, -2.0])
    assert abs(O.break_score(aff, fit, c) - 2.5) < 1e-12
    assert O.break_score(aff, aff, c) == 0.0
    # every entry scaled by (1 + e): centre c moves by e A(c), so the score is e RMS|A(c)|
    e = 1e-3
    fit2 = aff * np.array([1 + e, 1 + e, 1 + e, 1 + e, 1 + e, 1 + e])
    pa = np.stack(O.apply_affine(aff, c[:, 0], c[:, 1]), 1)
    assert abs(O.break_score(aff, fit2, c) - e * np.sqrt(np.mean(np.sum(pa ** 2, 1)))) < 1e-9


def test_join_break_closed_forms():
    rng = np.random.default_rng(61)
    S, j = 7, 3
    aff = np.array([[1 + rng.uniform(-1e-3, 1e-3), rng.uniform(-1e-3, 1e-3), rng.uniform(-5, 5),
                     rng.uniform(-1e-3, 1e-3), 1 + rng.uniform(-1e-3, 1e-3), rng.uniform(-5, 5)] for _ in range(S)])
    left = aff.copy()
    left[j] = [1.02, 0.001, -30.0, -0.002, 1.019, 42.0]
    out = O.join_break(aff, left, j)
    # sections before the break are untouched, section j becomes its left fit
    np.testing.assert_array_equal(out[:j], aff[:j])
    np.testing.assert_allclose(out[j], left[j], rtol=0, atol=1e-12)
    # every later section moves by the same aligned-frame correction: mapping
    # its new affine back through its old one gives that correction
    p = rng.uniform(0, 4096, (20, 2))
    def app(a, q):
        return np.stack(O.apply_affine(a, q[:, 0], q[:, 1]), 1)
    def inv(a):
        m = np.array([[a[0], a[1]], [a[3], a[4]]])
        mi = np.linalg.inv(m)
        t = -mi @ np.array([a[2], a[5]])
        return [mi[0, 0], mi[0, 1], t[0], mi[1, 0], mi[1, 1], t[1]]
    d_j = app(inv(aff[j]), app(out[j], p))
    for s in range(j + 1, S):
        np.testing.assert_allclose(app(inv(aff[s]), app(out[s], p)), d_j, rtol=0, atol=1e-8)


def test_search_select_stops_at_the_threshold():
    # the first candidate at or above the threshold ends the search (even if a
    # later one would be better); otherwise every candidate runs and the first
    # best is kept
    assert O.search_select([3.0, 20.0, 40.0], 15.0) == (1, 2)
    assert O.search_select([15.0, 2.0], 15.0) == (0, 1)
    assert O.search_select([3.0, 9.0, 9.0, 4.0], 15.0) == (1, 4)
    assert O.search_select([], 15.0) == (-1, 0)
    # with no threshold the search is exhaustive and keeps the best
    assert O.search_select([3.0, 20.0, 40.0, 1.0], np.inf) == (2, 4)
