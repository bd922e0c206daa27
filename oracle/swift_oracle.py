"""Plain FP64 CPU oracle for signal-whitened FFT window matching.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  Never imported by the product package.

Source: Wetzel et al., "Registering large volume serial-section electron
microscopy image sets for neural circuit reconstruction using FFT signal
whitening" (arXiv 1612.04787).  The paper states the method in prose only
(Section III); every formula below is the plain definition of what that prose
describes, with the readings of unstated details listed in the repository's
design notes (taper shape and width, the epsilon floor, the correlation sign,
the SNR background, the centroid, the projection rounding).

Conventions
  * Images are row-major [y][x].  A window of edge N has pixel (i, j) = (x, y)
    index; its window-centred coordinates are u = i - N/2, v = j - N/2.
  * theta (8 values): cx, cy, a11, a12, tx, a21, a22, ty.  The window samples
    the image at x = cx + a11 u + a12 v + tx, y = cy + a21 u + a22 v + ty.
  * Forward DFT unnormalised, inverse DFT scaled by 1/N^2.
  * Correlation sign: X = conj(F_A) F_B, so if B(x) = A(x - d) the peak is at +d.

Every function is FP64 throughout; library FFTs (NumPy pocketfft) and a few
array primitives are used as steps, with no blocking, fusion or reordering.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

STATUS_NEAR_TIE = 1
STATUS_DEGENERATE = 2
STATUS_CLAMPED = 4
NEAR_TIE_REL = 2e-4


@dataclass
class Params:
    """Matching parameters.

    p          whitening exponent in [0, 1]: 0 is plain correlation (NCC-like),
               1 is phase-only correlation (Section III, whitening paragraph).
    eps_rel    relative floor of the whitening denominator (design reading).
    taper_frac fraction of the window edge covered by the cosine taper, both
               edges together (apodization paragraph of Section III).
    centroid_r half-width of the sub-pixel centroid box.
    max_shift  radius r of the expected-shift neighbourhood: r > 0 (and below
               N/2) restricts the integer peak to wrapped shifts |sx|, |sy| <= r
               (the pruned inverse transform, a speed-up the paper names in
               Section V); 0 searches the whole surface.  The SNR background
               is the whole surface either way.
    snr_exclude_r  R >= 0: the SNR background (mean and population std) leaves
               out the (2R+1)^2 surface entries around the integer peak
               (wrapped); 0 takes the whole surface (Section III, Z-score
               paragraph: the peak is scored against the background
               distribution of the surface).
    """
    p: float = 0.65
    eps_rel: float = 1e-4
    taper_frac: float = 0.25
    centroid_r: int = 1
    max_shift: int = 0
    snr_exclude_r: int = 0


# ---------------------------------------------------------------------------
# Window gather (tiled local patches, Section III)
# ---------------------------------------------------------------------------
def bilinear_clamped(img, x, y):
    """Bilinear sample of img at real coordinates (x, y), clamp-to-edge reads.
    Returns (values, clamped_any)."""
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    x1 = x0 + 1
    y1 = y0 + 1
    clamped = bool(np.any((x0 < 0) | (y0 < 0) | (x1 > w - 1) | (y1 > h - 1)))

    def rd(xx, yy):
        return img[np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)]

    v = (1 - fy) * ((1 - fx) * rd(x0, y0) + fx * rd(x1, y0)) \
        + fy * ((1 - fx) * rd(x0, y1) + fx * rd(x1, y1))
    return v, clamped


def window_coords(theta, n):
    """Sample coordinates (x, y) of an n x n window, each of shape (n, n) [j][i]."""
    cx, cy, a11, a12, tx, a21, a22, ty = [float(t) for t in theta]
    u = np.arange(n, dtype=np.float64) - n // 2
    uu, vv = np.meshgrid(u, u)  # uu[j][i] = u_i, vv[j][i] = v_j
    x = cx + a11 * uu + a12 * vv + tx
    y = cy + a21 * uu + a22 * vv + ty
    return x, y, uu, vv


def gather(img, theta, n):
    """Window of edge n sampled from img at the affine theta (bilinear,
    clamp-to-edge).  Returns (a [n][n] float64, clamped flag)."""
    x, y, _, _ = window_coords(theta, n)
    return bilinear_clamped(img, x, y)


# ---------------------------------------------------------------------------
# Apodization: cosine taper (Section III) and mean removal
# ---------------------------------------------------------------------------
def taper_1d(n, taper_frac):
    """Raised-cosine edge taper with L = round(taper_frac * n / 2) samples per
    edge: t(i) = (1 - cos(pi (i + 1/2) / L)) / 2 for i < L, mirrored at the far
    edge, 1 in between.  taper_frac = 0 gives all ones."""
    L = int(np.floor(taper_frac * n / 2.0 + 0.5))
    t = np.ones(n, dtype=np.float64)
    for i in range(min(L, n // 2)):
        t[i] = 0.5 * (1.0 - np.cos(np.pi * (i + 0.5) / L))
        t[n - 1 - i] = t[i]
    return t


def taper_2d(n, taper_frac):
    t = taper_1d(n, taper_frac)
    return np.outer(t, t)


DEGENERATE_REL = 1e-6


def centre_pixel(img, theta):
    """Value of the source pixel nearest the window centre (u = v = 0), i.e.
    img[clamp(floor(y + 1/2))][clamp(floor(x + 1/2))] at x = cx + tx,
    y = cy + ty.  It is the offset o about which a window's sums are taken
    (prepare)."""
    img = np.asarray(img)
    h, w = img.shape
    x = float(theta[0]) + float(theta[4])
    y = float(theta[1]) + float(theta[7])
    xi = int(np.clip(np.floor(x + 0.5), 0, w - 1))
    yi = int(np.clip(np.floor(y + 0.5), 0, h - 1))
    return float(img[yi, xi])


def prepare(a, T, o=None):
    """Subtract the taper-weighted mean, then taper: w = (a - m_T) T with
    m_T = sum(a T) / sum(T).  Returns (w, m_T).

    The sums are taken about an offset o (default: the centre sample): with
    d = a - o and m' = sum(d T) / sum(T), w = (d - m') T and m_T = o + m',
    the same w in exact arithmetic.  A window is degenerate (no signal to
    match) when ||w||^2 <= 1e-6 sum((d T)^2): its samples are equal up to
    rounding relative to their spread about o.  Its w is returned as exactly
    zero, so its surface is zero and its record degenerate.  A window whose
    samples all equal o has d = 0 and is degenerate exactly."""
    a = np.asarray(a, dtype=np.float64)
    if o is None:
        o = float(a[a.shape[0] // 2, a.shape[1] // 2])
    d = a - o
    dT = d * T
    m1 = float(np.sum(dT) / np.sum(T))
    w = (d - m1) * T
    if float(np.sum(w * w)) <= DEGENERATE_REL * float(np.sum(dT * dT)):
        return np.zeros_like(w), o + m1
    return w, o + m1


# ---------------------------------------------------------------------------
# Whitened correlation surface (Section III: power scaling of Fourier
# amplitudes, exponent 0..1; equivalently before or after the multiply)
# ---------------------------------------------------------------------------
def whitened_surface(wA, wB, p, eps_rel, return_parts=False):
    """c = IDFT2( X (|X|^2 + eps^2)^(-p/2) ), X = conj(DFT2 wA) DFT2 wB,
    eps^2 = eps_rel^2 sum(wA^2) sum(wB^2), DC bin forced to 0."""
    n = wA.shape[0]
    FA = np.fft.rfft2(wA)
    FB = np.fft.rfft2(wB)
    X = np.conj(FA) * FB
    r = (X * np.conj(X)).real
    eps2 = eps_rel ** 2 * float(np.sum(wA * wA)) * float(np.sum(wB * wB))
    d = r + eps2
    if p == 0:
        C = X.copy()
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            C = np.where(d > 0, X * np.power(d, -0.5 * p), 0.0)
    C[0, 0] = 0.0
    c = np.fft.irfft2(C, s=(n, n))
    if return_parts:
        return c, dict(FA=FA, FB=FB, X=X, C=C, eps2=eps2)
    return c


def _wrap(i, n):
    return i - n if i >= n // 2 else i


def search_mask(n, max_shift):
    """Surface entries the integer peak may take: all of them for max_shift
    0 (or >= n/2), else those whose wrapped shifts satisfy |sx|, |sy| <=
    max_shift."""
    if max_shift <= 0 or max_shift >= n // 2:
        return np.ones((n, n), dtype=bool)
    s = np.array([abs(_wrap(i, n)) <= max_shift for i in range(n)])
    return s[:, None] & s[None, :]


def background_mask(n, iy, ix, exclude_r):
    """Surface entries of the SNR background: all of them for exclude_r 0,
    else all but the (2R+1)^2 box around (iy, ix), wrapped."""
    bg = np.ones((n, n), dtype=bool)
    for dyy in range(-exclude_r, exclude_r + 1):
        for dxx in range(-exclude_r, exclude_r + 1):
            bg[(iy + dyy) % n, (ix + dxx) % n] = False
    return bg


def peak_stats(c, centroid_r=1, max_shift=0, exclude_r=0):
    """Integer peak (first maximum in row-major order among the entries of
    search_mask), Z-score SNR against the background (population std; the
    whole surface, or the surface without the (2R+1)^2 box around the peak
    for exclude_r = R > 0), and a (2r+1)^2 centroid with weights
    max(c - mean, 0), shifts wrapped to [-N/2, N/2)."""
    n = c.shape[0]
    cand = np.where(search_mask(n, max_shift), c, -np.inf).ravel()
    flat = int(np.argmax(cand))
    iy, ix = divmod(flat, n)
    peak = float(c[iy, ix])
    bgv = c[background_mask(n, iy, ix, int(exclude_r))] if exclude_r > 0 else c
    mu = float(np.mean(bgv))
    sd = float(np.sqrt(np.mean((bgv - mu) ** 2)))
    status = 0
    if sd > 0:
        snr = (peak - mu) / sd
    else:
        snr = 0.0
        status |= STATUS_DEGENERATE
    rest = np.delete(cand, flat)
    second = float(np.max(rest)) if rest.size else -np.inf
    if peak - second <= NEAR_TIE_REL * abs(peak):
        status |= STATUS_NEAR_TIE
    sx, sy = _wrap(ix, n), _wrap(iy, n)
    r = int(centroid_r)
    sw = swx = swy = 0.0
    for dyy in range(-r, r + 1):
        for dxx in range(-r, r + 1):
            wv = max(float(c[(iy + dyy) % n, (ix + dxx) % n]) - mu, 0.0)
            sw += wv
            swx += wv * dxx
            swy += wv * dyy
    dx = sx + (swx / sw if sw > 0 else 0.0)
    dy = sy + (swy / sw if sw > 0 else 0.0)

    def cv(ddx, ddy):
        return float(c[(iy + ddy) % n, (ix + ddx) % n])

    # curvature of the surface at the integer peak (central second differences)
    hxx = cv(1, 0) - 2 * peak + cv(-1, 0)
    hyy = cv(0, 1) - 2 * peak + cv(0, -1)
    hxy = 0.25 * (cv(1, 1) - cv(1, -1) - cv(-1, 1) + cv(-1, -1))
    return dict(ix=ix, iy=iy, sx=sx, sy=sy, dx=dx, dy=dy, peak=peak, mean=mu,
                std=sd, snr=snr, status=status, second=second, hxx=hxx, hyy=hyy, hxy=hxy)


def surface_hessian(c, iy, ix):
    """Hessian (d2/dx2, d2/dy2, d2/dxdy) at (ix, iy) of the trigonometric
    interpolant of the n x n surface c, from its spectrum over signed
    frequencies; the Nyquist frequency counts in the pure terms with (n/2)^2 and
    not in the mixed term."""
    n = c.shape[0]
    C = np.fft.fft2(c)
    f = np.arange(n, dtype=np.float64)
    f = np.where(f < n // 2, f, f - n)
    fm = f.copy()
    fm[n // 2] = 0.0
    f2 = f * f
    f2[n // 2] = (n // 2) ** 2
    ky, kx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    e = np.exp(2j * np.pi * (ky * iy + kx * ix) / n)
    sc = -(2 * np.pi / n) ** 2 / (n * n)
    hxx = sc * float(np.sum((C * e).real * f2[None, :]))
    hyy = sc * float(np.sum((C * e).real * f2[:, None]))
    hxy = sc * float(np.sum((C * e).real * fm[:, None] * fm[None, :]))
    return hxx, hyy, hxy


# ---------------------------------------------------------------------------
# Iterative refinement (Section IV: match, update, repeat until the scores
# stabilise).  One step on the translation (tx, ty) of window A.
# ---------------------------------------------------------------------------
def refine_step(rec, theta, mode="centroid", jac=None, max_step=0.5):
    """Returns (new theta, step length).

    centroid: t <- t - d with d = (dx, dy), the centroid shift of the peak.
    Steps longer than max_step are scaled to max_step.

    newton: Newton's method on the centroid, with the 2 x 2 Jacobian J =
    d d / d t taken from jac = [d(dx)/d theta_A, d(dy)/d theta_A] (six
    entries each, translations at 2 and 5).  Within the cell of the integer
    peak s the centroid moves as d = s + J (t - t* - s), so
    t <- t - (s + J^-1 (d - s)).  It applies when s is the origin, or one of
    its eight neighbours with J^-1 (d - s) inside [-0.6, 0.6]^2 (the model
    places t in the peak's cell), the window is not degenerate and det J >
    1e-6; otherwise the centroid step.  The Newton step is scaled down to at most
    |s| + max_step, so the whole-pixel part is never cut."""
    theta = np.array(theta, dtype=np.float64)
    d = np.array([rec["dx"], rec["dy"]], dtype=np.float64)
    step = -d
    limit = max_step
    near = abs(rec["sx"]) <= 1 and abs(rec["sy"]) <= 1
    if mode == "newton" and jac is not None and near and not (rec["status"] & STATUS_DEGENERATE):
        jac = np.asarray(jac, dtype=np.float64).reshape(2, 6)
        J = np.array([[jac[0, 2], jac[0, 5]], [jac[1, 2], jac[1, 5]]])
        if np.linalg.det(J) > 1e-6:
            sv = np.array([rec["sx"], rec["sy"]], dtype=np.float64)
            off = np.linalg.solve(J, d - sv)
            if (sv[0] == 0 and sv[1] == 0) or np.all(np.abs(off) <= 0.6):
                step = -(sv + off)
                limit = max_step + float(np.hypot(sv[0], sv[1]))
    ln = float(np.hypot(step[0], step[1]))
    if not ln <= limit:
        step = step * (limit / ln) if ln > 0 else np.zeros(2)
        ln = limit
    theta[4] += step[0]
    theta[7] += step[1]
    return theta, ln


def centroid_jacobian(imgA, imgB, thetaA, thetaB, n, params: Params):
    """Returns (record, [d(dx)/d theta_A, d(dy)/d theta_A]) as a 2 x 6 array,
    with the integer peak held fixed."""
    rec, gx, _ = match_grad(imgA, imgB, thetaA, thetaB, n, params, g_peak=0.0, g_snr=0.0, g_dx=1.0)
    _, gy, _ = match_grad(imgA, imgB, thetaA, thetaB, n, params, g_peak=0.0, g_snr=0.0, g_dy=1.0)
    return rec, np.stack([gx, gy])


def match_pair(imgA, imgB, thetaA, thetaB, n, params: Params, return_surface=False):
    """Full plain method for one window pair: gather, taper + mean, forward
    FFTs, whitened cross-power, inverse FFT, peak + SNR + centroid."""
    a, clA = gather(imgA, thetaA, n)
    b, clB = gather(imgB, thetaB, n)
    T = taper_2d(n, params.taper_frac)
    wA, _ = prepare(a, T, centre_pixel(imgA, thetaA))
    wB, _ = prepare(b, T, centre_pixel(imgB, thetaB))
    c = whitened_surface(wA, wB, params.p, params.eps_rel)
    rec = peak_stats(c, params.centroid_r, params.max_shift, params.snr_exclude_r)
    if clA or clB:
        rec["status"] |= STATUS_CLAMPED
    if return_surface:
        rec["surface"] = c
    return rec


# ---------------------------------------------------------------------------
# Adjoint: gradient of g_peak * c[s*] + g_snr * SNR with respect to the six
# affine entries of each window (argmax s* held fixed).  Not in the paper; it
# differentiates the plain definition above by the chain rule (complex
# gradients G = dJ/dRe + i dJ/dIm over the full N x N spectrum).
# ---------------------------------------------------------------------------
def _bilinear_partials(img, x, y):
    """d(bilinear)/dx and d/dy at (x, y), clamped reads, floor cell."""
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)

    def rd(xx, yy):
        return img[np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)]

    i00, i10 = rd(x0, y0), rd(x0 + 1, y0)
    i01, i11 = rd(x0, y0 + 1), rd(x0 + 1, y0 + 1)
    gx = (1 - fy) * (i10 - i00) + fy * (i11 - i01)
    gy = (1 - fx) * (i01 - i00) + fx * (i11 - i10)
    return gx, gy


def match_grad(imgA, imgB, thetaA, thetaB, n, params: Params, g_peak=0.0, g_snr=1.0, g_dx=0.0, g_dy=0.0):
    """Returns (record, dJ/dthetaA[6], dJ/dthetaB[6]) with J = g_peak c[s*] +
    g_snr SNR + g_dx dx + g_dy dy (dx, dy: the centroid shift); the six
    entries are (a11, a12, tx, a21, a22, ty)."""
    if params.snr_exclude_r:
        raise NotImplementedError("the adjoint takes the whole surface as the SNR background")
    p, eps_rel = params.p, params.eps_rel
    a, _ = gather(imgA, thetaA, n)
    b, _ = gather(imgB, thetaB, n)
    T = taper_2d(n, params.taper_frac)
    wA, _ = prepare(a, T, centre_pixel(imgA, thetaA))
    wB, _ = prepare(b, T, centre_pixel(imgB, thetaB))
    M = n * n
    # forward on the full spectrum
    FA = np.fft.fft2(wA)
    FB = np.fft.fft2(wB)
    X = np.conj(FA) * FB
    r = (X * np.conj(X)).real
    SA = float(np.sum(wA * wA))
    SB = float(np.sum(wB * wB))
    eps2 = eps_rel ** 2 * SA * SB
    d = r + eps2
    with np.errstate(divide="ignore", invalid="ignore"):
        h = np.where(d > 0, np.power(d, -0.5 * p), 0.0) if p != 0 else np.ones_like(d)
        hp = np.where(d > 0, -0.5 * p * np.power(d, -0.5 * p - 1.0), 0.0) if p != 0 else np.zeros_like(d)
    C = X * h
    C[0, 0] = 0.0
    c = np.fft.ifft2(C).real
    rec = peak_stats(c, params.centroid_r, params.max_shift)
    iy, ix = rec["iy"], rec["ix"]
    mu, sd, snr = rec["mean"], rec["std"], rec["snr"]
    # cotangent of the surface
    Gc = np.zeros((n, n))
    Gc[iy, ix] += g_peak
    if sd > 0:
        Gc[iy, ix] += g_snr / sd
        Gc += g_snr * (-1.0 / (M * sd) - snr * (c - mu) / (M * sd * sd))
    # centroid: d = s* + sum w_d delta / sum w_d, w_d = max(c(s* + delta) - mean, 0).
    # d(dx)/dc(s* + delta) = (delta_x - (dx - sx)) / sum w on the positive weights;
    # the mean's share is uniform over the surface and vanishes with the DC bin.
    if g_dx != 0.0 or g_dy != 0.0:
        wsum = 0.0
        cells = []
        for dyy in (-1, 0, 1):
            for dxx in (-1, 0, 1):
                yy, xx = (iy + dyy) % n, (ix + dxx) % n
                wv = c[yy, xx] - mu
                if wv > 0:
                    wsum += wv
                    cells.append((yy, xx, dxx, dyy))
        if wsum > 0:
            fx, fy = rec["dx"] - rec["sx"], rec["dy"] - rec["sy"]
            for (yy, xx, dxx, dyy) in cells:
                Gc[yy, xx] += (g_dx * (dxx - fx) + g_dy * (dyy - fy)) / wsum
    # c = Re(IDFT2 C): G_C = DFT2(Gc) / M
    GC = np.fft.fft2(Gc) / M
    GC[0, 0] = 0.0
    # C = X h(|X|^2 + eps^2)
    GX = GC * (h + r * hp) + np.conj(GC) * X * X * hp
    GX[0, 0] = 0.0
    dJ_deps2 = float(np.sum((np.conj(GC) * X * hp).real))
    # X = conj(FA) FB
    GFA = np.conj(GX) * FB
    GFB = GX * FA
    # F = DFT2(w): G_w = Re(M IDFT2 G_F); plus the eps^2 path
    GwA = (np.fft.ifft2(GFA) * M).real + dJ_deps2 * 2.0 * eps_rel ** 2 * SB * wA
    GwB = (np.fft.ifft2(GFB) * M).real + dJ_deps2 * 2.0 * eps_rel ** 2 * SA * wB
    # w = (a - m) T, m = sum(aT)/sum(T)
    sT = float(np.sum(T))
    GaA = T * GwA - (T / sT) * float(np.sum(T * GwA))
    GaB = T * GwB - (T / sT) * float(np.sum(T * GwB))

    def theta_grad(img, theta, Ga):
        x, y, uu, vv = window_coords(theta, n)
        gx, gy = _bilinear_partials(img, x, y)
        return np.array([np.sum(Ga * gx * uu), np.sum(Ga * gx * vv), np.sum(Ga * gx),
                         np.sum(Ga * gy * uu), np.sum(Ga * gy * vv), np.sum(Ga * gy)])

    return rec, theta_grad(imgA, thetaA, GaA), theta_grad(imgB, thetaB, GaB)


# ---------------------------------------------------------------------------
# Model projection (remod): rounded mean of the z-neighbours, self and
# damaged sections omitted (Section III, model paragraph)
# ---------------------------------------------------------------------------
def project(stack, s, k, exclude=None):
    """R = round-half-up( sum_{j in J} I_j / |J| ), J = {j : 1 <= |j - s| <= k,
    0 <= j < S, not excluded}; integer arithmetic (2 S + n) // (2 n)."""
    S = stack.shape[0]
    J = [j for j in range(max(0, s - k), min(S, s + k + 1))
         if j != s and not (exclude is not None and exclude[j])]
    if not J:
        raise ValueError("projection has no included neighbour")
    acc = np.zeros(stack.shape[1:], dtype=np.int64)
    for j in J:
        acc += stack[j].astype(np.int64)
    nn = len(J)
    return ((2 * acc + nn) // (2 * nn)).astype(np.uint8)


def pyramid(img):
    """One level of the x2 source pyramid (iscale): 2 x 2 box mean rounded half
    up, (a + b + c + d + 2) >> 2; an odd trailing row/column is dropped."""
    img = np.asarray(img).astype(np.int64)
    h, w = img.shape[0] // 2, img.shape[1] // 2
    a = img[0:2 * h:2, 0:2 * w:2]
    b = img[0:2 * h:2, 1:2 * w:2]
    c = img[1:2 * h:2, 0:2 * w:2]
    d = img[1:2 * h:2, 1:2 * w:2]
    return ((a + b + c + d + 2) >> 2).astype(np.uint8)


# ---------------------------------------------------------------------------
# Global affine from correspondence points (mir, least squares; Section III)
# ---------------------------------------------------------------------------
def fit_affine(src, dst, weights=None):
    """Weighted linear least squares for dst ~ A [src; 1] (A is 2 x 3).
    src, dst: [n, 2] points (x, y).  Returns A as a 2 x 3 float64 array."""
    src = np.asarray(src, dtype=np.float64)
    dst = np.asarray(dst, dtype=np.float64)
    wts = np.ones(len(src)) if weights is None else np.asarray(weights, dtype=np.float64)
    D = np.column_stack([src, np.ones(len(src))])
    sw = np.sqrt(wts)[:, None]
    A, *_ = np.linalg.lstsq(D * sw, dst * sw, rcond=None)
    return A.T


# ---------------------------------------------------------------------------
# Stack loop (Sections III-IV): iscale levels, mir rendering by a section
# affine, swim windows through the affine against the remod model, and the
# least-squares affine of the correspondences.
#
# A section affine maps aligned-frame points p to raw-section points q, both in
# level-0 pixels: q = L p + t, stored as (a11, a12, tx, a21, a22, ty).  A level-l
# pyramid pixel x_l covers level-0 pixels 2^l x_l .. 2^l x_l + 2^l - 1, so its
# centre is x_0 = 2^l x_l + (2^l - 1) / 2.
# ---------------------------------------------------------------------------
STACK_FIT_SINGULAR = 1


def level_to_base(x, level):
    s = float(1 << level)
    return np.asarray(x, dtype=np.float64) * s + (s - 1.0) / 2.0


def base_to_level(x0, level):
    s = float(1 << level)
    return (np.asarray(x0, dtype=np.float64) - (s - 1.0) / 2.0) / s


def apply_affine(aff, x, y):
    a11, a12, tx, a21, a22, ty = [float(v) for v in aff]
    return a11 * x + a12 * y + tx, a21 * x + a22 * y + ty


def render(img, aff, level, out_h, out_w):
    """mir, one section: out[y][x] = bilinear value of the level-l image img at
    the raw point of aligned pixel (x, y), rounded half up to uint8:
    q_l = base_to_level(aff(level_to_base(x, y)))."""
    yy, xx = np.meshgrid(np.arange(out_h, dtype=np.float64), np.arange(out_w, dtype=np.float64), indexing="ij")
    qx, qy = apply_affine(aff, level_to_base(xx, level), level_to_base(yy, level))
    v, _ = bilinear_clamped(img, base_to_level(qx, level), base_to_level(qy, level))
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def stack_windows(aff, level, n, grid, h_l, w_l):
    """swim windows of one section at level l: a grid x grid tiling of n x n
    windows of the level-l aligned frame.  Window B reads the model at the
    tile centre p (identity); window A reads the raw section around the raw
    point of p, with the section's linear part.  The raw centre is split into
    a rounded part (cx, cy) and the remainder (tx, ty).  Returns float64
    (theta_a [grid^2, 8], theta_b [grid^2, 8])."""
    a11, a12, _, a21, a22, _ = [float(v) for v in aff]
    sx, sy = w_l // grid, h_l // grid
    ta = np.zeros((grid * grid, 8))
    tb = np.zeros((grid * grid, 8))
    for j in range(grid):
        for i in range(grid):
            k = j * grid + i
            px, py = sx // 2 + i * sx, sy // 2 + j * sy
            qx, qy = apply_affine(aff, level_to_base(px, level), level_to_base(py, level))
            cx, cy = base_to_level(qx, level), base_to_level(qy, level)
            rx, ry = np.rint(cx), np.rint(cy)
            ta[k] = [rx, ry, a11, a12, cx - rx, a21, a22, cy - ry]
            tb[k] = [px, py, 1, 0, 0, 0, 1, 0]
    return ta, tb


def correspondence(theta_a, theta_b, dx, dy, level):
    """Level-0 (p, q) of one match: the model point at the centre of window B,
    and the raw point that window A maps to it.  A window pair whose content
    satisfies B(x) = A(x - d) aligns A's window point -d with B's centre."""
    cxa, cya, a11, a12, txa, a21, a22, tya = [float(v) for v in theta_a]
    cxb, cyb, _, _, txb, _, _, tyb = [float(v) for v in theta_b]
    p = (level_to_base(cxb + txb, level), level_to_base(cyb + tyb, level))
    qx = cxa + txa - a11 * dx - a12 * dy
    qy = cya + tya - a21 * dx - a22 * dy
    return p, (level_to_base(qx, level), level_to_base(qy, level))


def match_weight(snr, status, min_snr):
    """Weight of a correspondence in the section fit: its SNR, or 0 for a
    degenerate window or an SNR below min_snr."""
    if (status & STATUS_DEGENERATE) or not (snr >= min_snr):
        return 0.0
    return float(snr)


def fit_section(p, q, w, prev):
    """mir's least-squares affine of one section from its correspondences (p ->
    q, weights w).  Fewer than three weighted points, or points on one line,
    keep `prev` and report STACK_FIT_SINGULAR.  Returns (aff [6], status)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    if np.count_nonzero(w > 0) < 3:
        return np.asarray(prev, dtype=np.float64).copy(), STACK_FIT_SINGULAR
    pc = p - np.sum(w[:, None] * p, 0) / np.sum(w)
    G = (w[:, None, None] * pc[:, :, None] * pc[:, None, :]).sum(0)
    if np.linalg.det(G) <= 1e-12 * np.trace(G) ** 2:
        return np.asarray(prev, dtype=np.float64).copy(), STACK_FIT_SINGULAR
    A = fit_affine(p, q, w)
    return np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 0], A[1, 1], A[1, 2]]), 0


# ---------------------------------------------------------------------------
# Local-affine triangle mesh (mir at the finest stages, Section IV; texture
# mapping of a triangulated mesh, Section III).  Every triangle carries its own
# affine, the weighted least-squares fit of the swim points in the triangle and
# in the band of triangles around it; every output pixel is rendered by the
# affine of the triangle it falls in.
#
# Mesh of one section (design reading): the nodes are the swim window centres
# of a grid x grid layout of the level-l aligned frame, node (i, j) at
# (sx//2 + i sx, sy//2 + j sy) with sx = w_l // grid, sy = h_l // grid, node
# index k = j grid + i.  Cell (ci, cj), 0 <= ci, cj < grid - 1, spans nodes
# ci..ci+1 by cj..cj+1 and is cut along the diagonal from node (ci+1, cj) to
# node (ci, cj+1).  Triangle 2 c holds nodes (ci, cj), (ci+1, cj), (ci, cj+1);
# triangle 2 c + 1 holds (ci+1, cj), (ci+1, cj+1), (ci, cj+1); c = cj (grid-1)
# + ci.  A pixel outside the hull of the nodes belongs to the nearest cell's
# triangle on its side of that cell's diagonal (the border triangles extend
# to the frame edges).
# ---------------------------------------------------------------------------
MESH_FIT_SINGULAR = 1


def mesh_node_xy(grid, h_l, w_l):
    """Level-l positions of the nodes: [grid^2, 2] int64 (x, y)."""
    sx, sy = w_l // grid, h_l // grid
    jj, ii = np.meshgrid(np.arange(grid), np.arange(grid), indexing="ij")
    return np.stack([sx // 2 + ii.ravel() * sx, sy // 2 + jj.ravel() * sy], 1).astype(np.int64)


def mesh_triangles(grid):
    """Node indices of every triangle, [2 (grid-1)^2, 3]."""
    tris = []
    for cj in range(grid - 1):
        for ci in range(grid - 1):
            k00 = cj * grid + ci
            k10, k01, k11 = k00 + 1, k00 + grid, k00 + grid + 1
            tris.append([k00, k10, k01])
            tris.append([k10, k11, k01])
    return np.array(tris, dtype=np.int64)


def mesh_band(grid, t):
    """The swim points that fit triangle t: its three vertices and every node
    that shares a mesh edge (a side of some triangle) with one of them.  Sorted
    node indices."""
    tris = mesh_triangles(grid)
    verts = set(int(v) for v in tris[t])
    band = set(verts)
    for tri in tris:
        for a in range(3):
            for b in range(3):
                if a != b and int(tri[a]) in verts:
                    band.add(int(tri[b]))
    return np.array(sorted(band), dtype=np.int64)


def mesh_triangle_of(x, y, grid, h_l, w_l):
    """Triangle index of level-l pixel (x, y) (integer arrays): the cell is
    (floor((x - x_0) / sx), floor((y - y_0) / sy)) clamped to the cells, and the
    pixel takes the cell's first triangle when (x - x_c)/sx + (y - y_c)/sy <= 1
    (x_c, y_c its first node), decided exactly in integers."""
    sx, sy = w_l // grid, h_l // grid
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    ci = np.clip(np.floor_divide(x - sx // 2, sx), 0, grid - 2)
    cj = np.clip(np.floor_divide(y - sy // 2, sy), 0, grid - 2)
    dx = x - (sx // 2 + ci * sx)
    dy = y - (sy // 2 + cj * sy)
    second = dx * sy + dy * sx > sx * sy
    return 2 * (cj * (grid - 1) + ci) + second.astype(np.int64)


def fit_mesh(p, q, w, grid, section_aff):
    """mir's affine of every triangle of one section from its grid^2 node
    correspondences (node k: model point p[k], raw point q[k], weight w[k], as
    for fit_section).  A triangle whose band has fewer than three weighted
    points, or collinear ones, takes the section's affine and status
    MESH_FIT_SINGULAR.  Returns (tri_aff [2 (grid-1)^2, 6], status [...])."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    T = 2 * (grid - 1) ** 2
    out = np.zeros((T, 6))
    st = np.zeros(T, dtype=np.int64)
    for t in range(T):
        b = mesh_band(grid, t)
        out[t], s = fit_section(p[b], q[b], w[b], section_aff)
        st[t] = MESH_FIT_SINGULAR if s else 0
    return out, st


def render_mesh_at(img, tri_aff, level, grid, out_h, out_w, x, y):
    """Pixels (x, y) (integer arrays) of render_mesh(img, tri_aff, level, grid,
    out_h, out_w): the bilinear value of the level-l image at the raw point of
    aligned pixel (x, y) under the affine of its triangle in the mesh of the
    out_h x out_w frame, rounded half up to uint8; the arithmetic of render,
    per pixel."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    t = mesh_triangle_of(x, y, grid, out_h, out_w)
    a = np.asarray(tri_aff, dtype=np.float64)[t]
    px = level_to_base(x.astype(np.float64), level)
    py = level_to_base(y.astype(np.float64), level)
    qx = a[..., 0] * px + a[..., 1] * py + a[..., 2]
    qy = a[..., 3] * px + a[..., 4] * py + a[..., 5]
    v, _ = bilinear_clamped(img, base_to_level(qx, level), base_to_level(qy, level))
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def render_mesh(img, tri_aff, level, grid, out_h, out_w):
    """mir texture mapping of one section: every pixel of the out_h x out_w
    aligned frame by render_mesh_at."""
    yy, xx = np.meshgrid(np.arange(out_h), np.arange(out_w), indexing="ij")
    return render_mesh_at(img, tri_aff, level, grid, out_h, out_w, xx, yy)


def mesh_windows(tri_aff, level, n, grid, h_l, w_l):
    """swim windows of one section through its mesh: window k sits at node k of
    the level-l aligned frame exactly as in stack_windows, and window A reads
    the raw section through the affine of the triangle the node's pixel belongs
    to (mesh_triangle_of).  Returns float64 (theta_a, theta_b) [grid^2, 8]."""
    nodes = mesh_node_xy(grid, h_l, w_l)
    t = mesh_triangle_of(nodes[:, 0], nodes[:, 1], grid, h_l, w_l)
    ta = np.zeros((grid * grid, 8))
    tb = np.zeros((grid * grid, 8))
    for k in range(grid * grid):
        aff = np.asarray(tri_aff[t[k]], dtype=np.float64)
        px, py = int(nodes[k, 0]), int(nodes[k, 1])
        qx, qy = apply_affine(aff, level_to_base(px, level), level_to_base(py, level))
        cx, cy = base_to_level(qx, level), base_to_level(qy, level)
        rx, ry = np.rint(cx), np.rint(cy)
        ta[k] = [rx, ry, aff[0], aff[1], cx - rx, aff[3], aff[4], cy - ry]
        tb[k] = [px, py, 1, 0, 0, 0, 1, 0]
    return ta, tb


# ---------------------------------------------------------------------------
# Pearson-normalised correlation (Section II: the NCC of other registration
# codes; an FFT correlation gives it after a cumulative-area correction).
# Design reading: the template is the central m x m part of window A, m = n/2,
# and it is scored against every placement inside window B, shifts |sx|, |sy|
# <= R = n/4 (no placement wraps around), by the Pearson correlation
# coefficient of the two m x m patches.  The peak and its record follow the
# whitened match: first maximum in row-major order of the wrapped n x n index,
# Z score over the (2R+1)^2 placements, 3 x 3 centroid with weights
# max(gamma - mean, 0) (placements outside the search range weigh 0).
# ---------------------------------------------------------------------------
def pearson_surface(a, f):
    """gamma [2R+1, 2R+1] (row sy + R, column sx + R) of the central n/2 x n/2
    template of the n x n window a against window f; a placement whose patch
    (or the template) is constant gets 0.  Returns (gamma, template energy)."""
    n = a.shape[0]
    m, c0, R = n // 2, n // 4, n // 4
    t = np.asarray(a, dtype=np.float64)[c0:c0 + m, c0:c0 + m]
    tc = t - t.mean()
    st = float(np.sum(tc * tc))
    f = np.asarray(f, dtype=np.float64)
    g = np.zeros((2 * R + 1, 2 * R + 1))
    for sy in range(-R, R + 1):
        for sx in range(-R, R + 1):
            p = f[c0 + sy:c0 + sy + m, c0 + sx:c0 + sx + m]
            pc = p - p.mean()
            sp = float(np.sum(pc * pc))
            if st > 0 and sp > 0:
                g[sy + R, sx + R] = float(np.sum(tc * pc)) / np.sqrt(st * sp)
    return g, st


def pearson_peak(g, n, st):
    """Record of a Pearson surface (see pearson_surface): integer peak, Z
    score over the placements, 3 x 3 centroid, near-tie and degenerate bits."""
    R = n // 4
    full = np.full((n, n), -np.inf)
    for sy in range(-R, R + 1):
        for sx in range(-R, R + 1):
            full[sy % n, sx % n] = g[sy + R, sx + R]
    flat = int(np.argmax(full.ravel()))
    iy, ix = divmod(flat, n)
    sx, sy = _wrap(ix, n), _wrap(iy, n)
    peak = float(full[iy, ix])
    mu = float(g.mean())
    sd = float(np.sqrt(np.mean((g - mu) ** 2)))
    status = 0
    snr = (peak - mu) / sd if sd > 0 else 0.0
    if not (st > 0 and sd > 0):
        status |= STATUS_DEGENERATE
        snr = 0.0
    rest = np.delete(full.ravel(), flat)
    second = float(np.max(rest))
    if peak - second <= NEAR_TIE_REL * abs(peak):
        status |= STATUS_NEAR_TIE
    sw = swx = swy = 0.0
    for ddy in (-1, 0, 1):
        for ddx in (-1, 0, 1):
            if abs(sx + ddx) <= R and abs(sy + ddy) <= R:
                wv = max(float(g[sy + ddy + R, sx + ddx + R]) - mu, 0.0)
                sw += wv
                swx += wv * ddx
                swy += wv * ddy
    dx = sx + (swx / sw if sw > 0 else 0.0)
    dy = sy + (swy / sw if sw > 0 else 0.0)
    return dict(ix=ix, iy=iy, sx=sx, sy=sy, dx=dx, dy=dy, peak=peak, mean=mu, std=sd, snr=snr,
                status=status, second=second)


def pearson_pair(imgA, imgB, thetaA, thetaB, n, return_surface=False):
    """Pearson-normalised match of one window pair: gather both windows
    (bilinear, clamp to edge; no taper, no whitening), then pearson_surface
    and pearson_peak."""
    a, clA = gather(imgA, thetaA, n)
    f, clB = gather(imgB, thetaB, n)
    g, st = pearson_surface(a, f)
    rec = pearson_peak(g, n, st)
    if clA or clB:
        rec["status"] |= STATUS_CLAMPED
    if return_surface:
        rec["surface"] = g
    return rec


# ---------------------------------------------------------------------------
# Jump repair (Section III, model paragraphs).  An abrupt change of content
# or magnification can lock a section's match to one side of its two-sided
# model.  The sections involved are then fitted against a left-only and a
# right-only model, and the affines across the failed span follow a smooth
# curve between the two fits.  Design readings: the one-sided models are the rounded means of the
# k sections before (side -1) or after (side +1), offending ones omitted; the
# curve is the cubic Bezier with control values 0, 0, 1, 1 (zero slope at
# both ends) blending, per affine entry, the left-model fit into the
# right-model fit across the span.
# ---------------------------------------------------------------------------
def project_side(stack, s, k, side, exclude=None):
    """One-sided model of section s: round-half-up of the mean of sections
    s-k..s-1 (side -1) or s+1..s+k (side +1) inside the stack and not
    excluded; zeros when there is none.  Integer arithmetic as project."""
    S = stack.shape[0]
    J = range(max(0, s - k), s) if side < 0 else range(s + 1, min(S, s + k + 1))
    J = [j for j in J if not (exclude is not None and exclude[j])]
    if not J:
        return np.zeros(stack.shape[1:], dtype=np.uint8)
    acc = np.zeros(stack.shape[1:], dtype=np.int64)
    for j in J:
        acc += stack[j].astype(np.int64)
    nn = len(J)
    return ((2 * acc + nn) // (2 * nn)).astype(np.uint8)


def span_weight(s, a, b):
    """Weight of the right-model fit for section s of the failed span [a, b]:
    t = (s - a + 1) / (b - a + 2) (the span's good neighbours a - 1 and b + 1
    sit at t = 0 and 1), w = 3 t^2 - 2 t^3."""
    t = (s - a + 1) / (b - a + 2)
    return 3.0 * t * t - 2.0 * t * t * t


def blend_span(aff_left, aff_right, a, b):
    """Repaired affines [b - a + 1, 6] of the span: (1 - w) A_left + w A_right
    entry by entry, with w = span_weight; aff_left, aff_right indexed by
    section."""
    out = []
    for s in range(a, b + 1):
        w = span_weight(s, a, b)
        out.append((1.0 - w) * np.asarray(aff_left[s], dtype=np.float64) + w * np.asarray(aff_right[s], dtype=np.float64))
    return np.array(out)


def failed_spans(section_snr, frac):
    """Maximal runs [a, b] of sections whose SNR is below frac times the
    median over all sections."""
    v = np.asarray(section_snr, dtype=np.float64)
    bad = v < frac * np.median(v)
    spans, s = [], 0
    while s < len(v):
        if bad[s]:
            e = s
            while e + 1 < len(v) and bad[e + 1]:
                e += 1
            spans.append((s, e))
            s = e + 1
        else:
            s += 1
    return spans


def break_score(aff, fit, centres):
    """How far a section's fit against its left one-sided model moves its
    windows: the RMS over the window centres c (level-0 px) of
    |fit(c) - aff(c)|.  A score above the break threshold starts a break
    (design reading of the locked-match paragraph of Section III)."""
    c = np.asarray(centres, dtype=np.float64)
    pa = np.stack(apply_affine(aff, c[:, 0], c[:, 1]), 1)
    pf = np.stack(apply_affine(fit, c[:, 0], c[:, 1]), 1)
    return float(np.sqrt(np.mean(np.sum((pf - pa) ** 2, 1))))


def join_break(aff, aff_left, j):
    """Joins the sections from j on to the frame of the sections before a
    break at j: with A_j the affine of section j and L_j its fit against the
    left one-sided model, the aligned-frame correction D = A_j^-1 L_j is
    composed into every section s >= j (A_s <- A_s D), so that section j
    becomes L_j.  Affines (a11, a12, tx, a21, a22, ty) map aligned to raw
    points."""
    def mat(a):
        a = np.asarray(a, dtype=np.float64)
        return np.array([[a[0], a[1], a[2]], [a[3], a[4], a[5]], [0.0, 0.0, 1.0]])

    D = np.linalg.inv(mat(aff[j])) @ mat(aff_left[j])
    out = np.array(aff, dtype=np.float64).copy()
    for s in range(j, len(out)):
        m = mat(out[s]) @ D
        out[s] = [m[0, 0], m[0, 1], m[0, 2], m[1, 0], m[1, 1], m[1, 2]]
    return out


# ---------------------------------------------------------------------------
# Search with an SNR stop (Section III, SNR paragraph: an SNR above 15 marks
# a correct match, so a search for better matches can stop there).  Design
# reading: a window whose placement is unknown beyond the capture range is
# matched at candidate translations in a fixed order; it keeps its best
# (highest SNR) match so far and leaves the search at the first candidate
# whose SNR reaches the threshold.
# ---------------------------------------------------------------------------
def search_select(snrs, accept):
    """snrs: SNR of each candidate in search order (one window).  Returns
    (index of the kept candidate, candidates matched): the first candidate
    whose SNR reaches accept ends the search; otherwise all are matched and
    the best (first of equals) is kept."""
    best, arg = -np.inf, -1
    for k, v in enumerate(snrs):
        if v > best:
            best, arg = v, k
        if v >= accept:
            return arg, k + 1
    return arg, len(snrs)
