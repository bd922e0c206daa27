"""CPU FP32 baseline of the whitened match (test and benchmark infrastructure).

The same computation as `swift_oracle.match_pair` (Section III: taper and
weighted mean, forward transforms, cross power with the amplitudes raised to
-p, inverse transform, Z-score of the first maximum, 3 x 3 centroid), but in
single precision over a batch of window pairs at once, with SciPy's
multithreaded pocketfft.  It is the fast CPU implementation the GPU path is
set against in the benchmark, not the parity oracle: the FP64 definition in
swift_oracle is.  Only tests and the benchmark's CPU leg use it.

Windows are sampled as in the oracle (bilinear, clamp-to-edge, affine
theta = (cx, cy, a11, a12, tx, a21, a22, ty)); the spectra are normalised by
the window norms before the cross power so FP32 cannot overflow.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .swift_oracle import DEGENERATE_REL, taper_1d


def gather_batch(img, thetas, n):
    """Windows [B, n, n] (float32) of img at the affines thetas [B, 8]
    (bilinear, clamp-to-edge), and the clamp flags [B]."""
    img = np.asarray(img)
    h, w = img.shape
    th = np.asarray(thetas, np.float64)
    u = (np.arange(n) - n // 2).astype(np.float64)
    # x[b, j, i] = cx + a11 u_i + a12 v_j + tx
    x = (th[:, 0] + th[:, 4])[:, None, None] + th[:, 2, None, None] * u[None, None, :] + \
        th[:, 3, None, None] * u[None, :, None]
    y = (th[:, 1] + th[:, 7])[:, None, None] + th[:, 5, None, None] * u[None, None, :] + \
        th[:, 6, None, None] * u[None, :, None]
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = (x - x0).astype(np.float32)
    fy = (y - y0).astype(np.float32)
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    clamped = ((x0 < 0) | (x0 > w - 2) | (y0 < 0) | (y0 > h - 2)).any(axis=(1, 2))
    cx0, cx1 = np.clip(x0, 0, w - 1), np.clip(x0 + 1, 0, w - 1)
    cy0, cy1 = np.clip(y0, 0, h - 1), np.clip(y0 + 1, 0, h - 1)
    src = img.astype(np.float32, copy=False)
    i00, i10 = src[cy0, cx0], src[cy0, cx1]
    i01, i11 = src[cy1, cx0], src[cy1, cx1]
    top = i00 + fx * (i10 - i00)
    bot = i01 + fx * (i11 - i01)
    return (top + fy * (bot - top)).astype(np.float32), clamped


def _centre_pixels(img, thetas):
    img = np.asarray(img)
    h, w = img.shape
    th = np.asarray(thetas, np.float64)
    xi = np.clip(np.floor(th[:, 0] + th[:, 4] + 0.5), 0, w - 1).astype(np.int64)
    yi = np.clip(np.floor(th[:, 1] + th[:, 7] + 0.5), 0, h - 1).astype(np.int64)
    return img[yi, xi].astype(np.float32)


def match_batch(imgA, imgB, thA, thB, n, p=0.65, eps_rel=1e-4, taper_frac=0.25, workers=1):
    """Records of a batch of pairs: dict of arrays ix, iy, dx, dy, peak, mean,
    std, snr (float64 statistics of the FP32 surface)."""
    a, _ = gather_batch(imgA, thA, n)
    b, _ = gather_batch(imgB, thB, n)
    t = taper_1d(n, taper_frac).astype(np.float32)
    T = np.outer(t, t)
    sT = float(T.sum(dtype=np.float64))

    def prep(win, o):
        d = win - o[:, None, None]
        dT = d * T
        m = (dT.sum(axis=(1, 2), dtype=np.float64) / sT).astype(np.float32)
        wv = (d - m[:, None, None]) * T
        e = (wv.astype(np.float64) ** 2).sum(axis=(1, 2))
        e0 = (dT.astype(np.float64) ** 2).sum(axis=(1, 2))
        return wv, e, ~(e > DEGENERATE_REL * e0)

    wA, eA, degA = prep(a, _centre_pixels(imgA, thA))
    wB, eB, degB = prep(b, _centre_pixels(imgB, thB))
    FA = sfft.rfft2(wA, axes=(1, 2), workers=workers)
    FB = sfft.rfft2(wB, axes=(1, 2), workers=workers)
    ok = ~(degA | degB)
    sA = np.where(ok, 1.0 / np.sqrt(np.where(ok, eA, 1.0)), 0.0).astype(np.float32)
    sB = np.where(ok, 1.0 / np.sqrt(np.where(ok, eB, 1.0)), 0.0).astype(np.float32)
    # normalised cross power X^ = X / (||w_A|| ||w_B||); C = X^ (|X^|^2 + eps_rel^2)^(-p/2) kw
    X = np.conj(FA * sA[:, None, None]) * (FB * sB[:, None, None])
    d = (X.real * X.real + X.imag * X.imag) + np.float32(eps_rel * eps_rel)
    C = X * (d ** np.float32(-0.5 * p)) if p != 0 else X
    kw = np.where(ok, np.exp(0.5 * (1.0 - p) * (np.log(np.where(ok, eA, 1.0)) + np.log(np.where(ok, eB, 1.0)))),
                  0.0).astype(np.float32)
    C = C * kw[:, None, None]
    C[:, 0, 0] = 0
    c = sfft.irfft2(C, s=(n, n), axes=(1, 2), workers=workers).astype(np.float32)
    B = c.shape[0]
    flat = c.reshape(B, -1).argmax(axis=1)
    iy, ix = flat // n, flat % n
    peak = c.reshape(B, -1)[np.arange(B), flat].astype(np.float64)
    mu = c.mean(axis=(1, 2), dtype=np.float64)
    sd = np.sqrt(np.maximum((c.astype(np.float64) ** 2).mean(axis=(1, 2)) - mu * mu, 0.0))
    snr = np.where(sd > 0, (peak - mu) / np.where(sd > 0, sd, 1.0), 0.0)
    sw = np.zeros(B)
    swx = np.zeros(B)
    swy = np.zeros(B)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            v = c[np.arange(B), (iy + dy) % n, (ix + dx) % n].astype(np.float64)
            wv = np.maximum(v - mu, 0.0)
            sw += wv
            swx += wv * dx
            swy += wv * dy
    sx = np.where(ix >= n // 2, ix - n, ix)
    sy = np.where(iy >= n // 2, iy - n, iy)
    safe = np.where(sw > 0, sw, 1.0)
    return dict(ix=ix, iy=iy, dx=sx + np.where(sw > 0, swx / safe, 0.0), dy=sy + np.where(sw > 0, swy / safe, 0.0),
                peak=peak, mean=mu, std=sd, snr=snr)
