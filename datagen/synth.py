"""Seeded synthetic serial-section data.

The paper's datasets (mouse LGN and zebrafish ssEM, Sections I and IV) are not
available, so every input here is synthetic with their structure: 8-bit
sections of textured background crossed by thin dark curved "membranes",
neighbouring sections that share content and drift slowly in z, and per-section
affine distortions.

Two back ends are used:
  * NumPy/SciPy for the tiny single-pair case (exactly reproducible anywhere);
  * PyTorch (CPU or GPU, seeded torch.Generator) for sections and stacks, so the
    multi-gigapixel workloads can be generated on the GPU in milliseconds.
Warps use library bilinear resampling (torch.nn.functional.grid_sample with
align_corners=True, i.e. integer pixel centres), never code of this project.
"""
from __future__ import annotations

import math

import numpy as np

try:  # torch is needed for sections/stacks only
    import torch
    import torch.nn.functional as F
except Exception:  # pragma: no cover
    torch = None
    F = None


# ----------------------------------------------------------------------------
# Single 64x64 pair (NumPy/SciPy)
# ----------------------------------------------------------------------------
def make_pair64(n: int = 64, shift=(7, -3), noise_var: float = 4.0,
                seed_a: int = 1, seed_b: int = 101, blur: float = 2.0):
    """One pair of fp32 windows: A = blurred white noise scaled to [0, 255];
    B = A circularly shifted by shift=(dx, dy) plus Gaussian noise of variance
    `noise_var`.  B(x, y) = A(x - dx, y - dy), so the content of B sits at +d.
    Returns (A, B) as float32 arrays of shape (n, n), row-major [y][x]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed_a)
    a0 = rng.standard_normal((n, n))
    a = gaussian_filter(a0, blur, mode="wrap")
    a = (a - a.min()) / (a.max() - a.min()) * 255.0
    dx, dy = shift
    b = np.roll(a, (dy, dx), axis=(0, 1))
    rng_b = np.random.default_rng(seed_b)
    b = b + rng_b.normal(0.0, math.sqrt(noise_var), size=(n, n))
    return a.astype(np.float32), b.astype(np.float32)


# ----------------------------------------------------------------------------
# Sections (PyTorch)
# ----------------------------------------------------------------------------
def _gen(seed: int, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _gauss_blur(img, sigma: float):
    """Separable Gaussian blur of a (H, W) float32 tensor, reflect padding."""
    r = max(1, int(math.ceil(3.0 * sigma)))
    xs = torch.arange(-r, r + 1, dtype=torch.float32, device=img.device)
    k = torch.exp(-0.5 * (xs / sigma) ** 2)
    k = k / k.sum()
    x = img[None, None]
    x = F.pad(x, (r, r, 0, 0), mode="reflect")
    x = F.conv2d(x, k.view(1, 1, 1, -1))
    x = F.pad(x, (0, 0, r, r), mode="reflect")
    x = F.conv2d(x, k.view(1, 1, -1, 1))
    return x[0, 0]


def _texture(h: int, w: int, g, device, blur=2.0, mean=128.0, std=30.0):
    noise = torch.randn(h, w, generator=g, device=device, dtype=torch.float32)
    t = _gauss_blur(noise, blur)
    t = (t - t.mean()) / t.std()
    return t * std + mean


def _curve_params(h: int, w: int, n: int, g, device, span: float = 300.0):
    """Control points of n random quadratic Bezier curves (endpoints <= span apart)."""
    p0 = torch.rand(n, 2, generator=g, device=device) * torch.tensor([w, h], device=device)
    ang = torch.rand(n, generator=g, device=device) * (2 * math.pi)
    ln = torch.rand(n, generator=g, device=device) * span
    p2 = p0 + torch.stack([torch.cos(ang), torch.sin(ang)], 1) * ln[:, None]
    bend = (torch.rand(n, generator=g, device=device) - 0.5) * ln
    perp = torch.stack([-torch.sin(ang), torch.cos(ang)], 1)
    p1 = 0.5 * (p0 + p2) + perp * bend[:, None]
    return p0, p1, p2


def _draw_curves(img, p0, p1, p2, value: float):
    """Draw 2-px-wide curves of constant intensity into img (in place)."""
    h, w = img.shape
    n = p0.shape[0]
    if n == 0:
        return img
    steps = 640
    t = torch.linspace(0.0, 1.0, steps, device=img.device)[None, :, None]
    pts = ((1 - t) ** 2) * p0[:, None] + 2 * (1 - t) * t * p1[:, None] + (t ** 2) * p2[:, None]
    pts = pts.reshape(-1, 2).round().long()
    for oy in (0, 1):
        for ox in (0, 1):
            x = pts[:, 0] + ox
            y = pts[:, 1] + oy
            ok = (x >= 0) & (x < w) & (y >= 0) & (y < h)
            img[y[ok], x[ok]] = value
    return img


def _to_u8(img):
    return img.clamp(0, 255).round().to(torch.uint8)


def make_section(h: int, w: int, seed: int, device="cpu", blur=2.0, mean=128.0,
                 std=30.0, n_curves=None, curve_value=40.0):
    """One uint8 section: blurred noise (mean 128, std 30) plus
    ceil(h*w/256^2) dark 2-px-wide quadratic Bezier curves."""
    g = _gen(seed, device)
    img = _texture(h, w, g, device, blur, mean, std)
    if n_curves is None:
        n_curves = int(math.ceil(h * w / 256.0 ** 2))
    p0, p1, p2 = _curve_params(h, w, n_curves, g, device)
    _draw_curves(img, p0, p1, p2, curve_value)
    return _to_u8(img)


def random_affine_about_center(h: int, w: int, seed: int, max_rot_deg=0.5,
                               max_scale=0.002, max_shift=40.0, max_shear=0.0):
    """A seeded affine map q -> M q + b (pixel coordinates, x first), built as a
    rotation/scale/shear about the image centre followed by a shift.
    Returns (M 2x2, b 2) as float64 NumPy arrays."""
    rng = np.random.default_rng(seed)
    th = math.radians(rng.uniform(-max_rot_deg, max_rot_deg))
    s = 1.0 + rng.uniform(-max_scale, max_scale)
    sh = rng.uniform(-max_shear, max_shear) if max_shear > 0 else 0.0
    t = rng.uniform(-max_shift, max_shift, size=2)
    rot = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    m = s * rot @ np.array([[1.0, sh], [0.0, 1.0]])
    c = np.array([(w - 1) / 2.0, (h - 1) / 2.0])
    b = c - m @ c + t
    return m, b


def bend_displacement(bend, x, y):
    """Smooth nonlinear displacement of a bend (ax, ay, phx, phy, period):
    (ax sin(2 pi y / period + phx), ay sin(2 pi x / period + phy))."""
    ax, ay, phx, phy, lam = bend
    k = 2.0 * math.pi / lam
    if isinstance(x, torch.Tensor):
        return ax * torch.sin(k * y + phx), ay * torch.sin(k * x + phy)
    return ax * np.sin(k * np.asarray(y) + phx), ay * np.sin(k * np.asarray(x) + phy)


def warp_affine(img_f32, m, b, out_hw=None, bend=None):
    """out(q) = img(M q + b + D(q)), bilinear, clamp-to-edge, via grid_sample;
    D is the bend displacement (zero when bend is None).
    img_f32: (H, W) float32 tensor. q = (x, y) in pixels of the output grid."""
    h, w = img_f32.shape
    oh, ow = out_hw if out_hw is not None else (h, w)
    dev = img_f32.device
    ys = torch.arange(oh, device=dev, dtype=torch.float64)
    xs = torch.arange(ow, device=dev, dtype=torch.float64)
    yy, xx = torch.meshgrid(ys, xs, indexing="ij")
    sx = m[0][0] * xx + m[0][1] * yy + b[0]
    sy = m[1][0] * xx + m[1][1] * yy + b[1]
    if bend is not None:
        dx, dy = bend_displacement(bend, xx, yy)
        sx = sx + dx
        sy = sy + dy
        del dx, dy
    gx = (2.0 * sx / (w - 1) - 1.0).float()
    gy = (2.0 * sy / (h - 1) - 1.0).float()
    del sx, sy, xx, yy
    grid = torch.stack([gx, gy], dim=-1)[None]
    out = F.grid_sample(img_f32[None, None], grid, mode="bilinear",
                        padding_mode="border", align_corners=True)
    return out[0, 0]


def make_section_pair(h: int, w: int, seed_a: int = 2, seed_b: int = 202,
                      device="cpu", noise_sigma=8.0, max_rot_deg=0.5,
                      max_scale=0.002, max_shift=40.0):
    """Section A plus B = bilinear affine warp of A (about the centre) plus
    Gaussian noise.  B(q) = A(M q + b).  Returns (A u8, B u8, M, b)."""
    a = make_section(h, w, seed_a, device)
    m, bvec = random_affine_about_center(h, w, seed_b, max_rot_deg, max_scale, max_shift)
    g = _gen(seed_b, device)
    bw = warp_affine(a.float(), m, bvec)
    bw = bw + noise_sigma * torch.randn(bw.shape, generator=g, device=device)
    return a, _to_u8(bw), m, bvec


def make_stack(n_sections: int, h: int, w: int, seed: int, device="cpu",
               keyframe_every=8, noise_sigma=8.0, drift_px_per_section=0.3,
               warps=None):
    """A (S, H, W) uint8 stack whose content varies smoothly in z: keyframe
    textures every `keyframe_every` sections blended linearly, membrane control
    points drifting slowly with z, independent noise per section.
    `warps`, if given, is a list of (M, b) or (M, b, bend) per section applied
    to the clean section before noise (observed(q) = clean(M q + b + D(q)), D
    the bend displacement)."""
    g = _gen(seed, device)
    n_key = n_sections // keyframe_every + 2
    keys = [_texture(h, w, g, device) for _ in range(n_key)]
    n_curves = int(math.ceil(h * w / 256.0 ** 2))
    p0, p1, p2 = _curve_params(h, w, n_curves, g, device)
    v0 = (torch.rand(n_curves, 2, generator=g, device=device) - 0.5) * 2 * drift_px_per_section
    v1 = (torch.rand(n_curves, 2, generator=g, device=device) - 0.5) * 2 * drift_px_per_section
    v2 = (torch.rand(n_curves, 2, generator=g, device=device) - 0.5) * 2 * drift_px_per_section
    out = torch.empty((n_sections, h, w), dtype=torch.uint8, device=device)
    for s in range(n_sections):
        k = s // keyframe_every
        al = (s % keyframe_every) / float(keyframe_every)
        tex = (1.0 - al) * keys[k] + al * keys[k + 1]
        _draw_curves(tex, p0 + s * v0, p1 + s * v1, p2 + s * v2, 40.0)
        if warps is not None and warps[s] is not None:
            m, b = warps[s][0], warps[s][1]
            tex = warp_affine(tex, m, b, bend=warps[s][2] if len(warps[s]) > 2 else None)
        tex = tex + noise_sigma * torch.randn(tex.shape, generator=g, device=device)
        out[s] = _to_u8(tex)
        del tex
    return out


def window_grid(h: int, w: int, n: int, grid: int, spacing=None):
    """Centres (cx, cy) of a grid x grid layout of n x n windows, row-major.
    With spacing None the grid tiles the image exactly (spacing = h // grid)."""
    sy = spacing if spacing is not None else h // grid
    sx = spacing if spacing is not None else w // grid
    cs = []
    for j in range(grid):
        for i in range(grid):
            cs.append((sx // 2 + i * sx, sy // 2 + j * sy))
    return np.array(cs, dtype=np.float64)


def config4_thetas(n_windows: int, seed: int = 404, max_shift=0.5, max_lin=1e-3):
    """Per-window affine perturbations: translation U(-0.5, 0.5)^2 px and a
    linear part I + E with |E_ij| <= 1e-3.  Returns [n, 6] float64 in the order
    (a11, a12, tx, a21, a22, ty)."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(-max_lin, max_lin, size=(n_windows, 4))
    t = rng.uniform(-max_shift, max_shift, size=(n_windows, 2))
    th = np.empty((n_windows, 6))
    th[:, 0] = 1.0 + e[:, 0]
    th[:, 1] = e[:, 1]
    th[:, 2] = t[:, 0]
    th[:, 3] = e[:, 2]
    th[:, 4] = 1.0 + e[:, 3]
    th[:, 5] = t[:, 1]
    return th
