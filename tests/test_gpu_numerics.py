"""GPU parity of the numerically delicate cases against the FP64 oracle:
near-constant and low-contrast windows (the degeneracy reading and the
window offset), large fp32 intensities (the normalised cross power), the
SNR background without the box around the peak, and the tune cache."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from datagen import make_section
from parity_util import compare, gpu_record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def _run(ctx, images, n, tha, thb, params, surfaces=True, ia=None, ib=None):
    k = tha.shape[0]
    ia = torch.zeros(k, dtype=torch.int32) if ia is None else ia
    ib = torch.ones(k, dtype=torch.int32) if ib is None else ib
    res = ctx.match_batch([im.to(dev()) for im in images], [n] * k, ia, ib, torch.from_numpy(tha),
                          torch.from_numpy(thb), params, surfaces=surfaces)
    torch.cuda.synchronize()
    return res


def _ident(cx, cy, tx=0.0, ty=0.0):
    return [cx, cy, 1, 0, tx, 0, 1, ty]


def test_near_constant_window_is_scored(ctx):
    """64^2 window of 200 with one pixel at 201 (uint8) matched against a
    shifted window of the same image, at whole and at fractional offsets:
    scored, not degenerate, record and surface as the oracle's; a constant
    window is degenerate on both sides."""
    import paper_1612_04787_amd as sw
    print("case near-constant 64", flush=True)
    n = 64
    img = np.full((96, 96), 200, np.uint8)
    img[40, 37] = 201
    rng = np.random.default_rng(12)
    other = rng.integers(0, 256, (96, 96)).astype(np.uint8)
    const = np.full((96, 96), 200, np.uint8)
    tha = np.array([_ident(48, 48), _ident(48, 48, 0.25, -0.5), _ident(48, 48)], np.float32)
    thb = np.array([_ident(48, 48, 1.0, 2.0), _ident(48, 48, -2.0, 1.5), _ident(48, 48)], np.float32)
    imgs = [torch.from_numpy(img), torch.from_numpy(other), torch.from_numpy(const)]
    ia = torch.tensor([0, 0, 2], dtype=torch.int32)
    ib = torch.tensor([0, 0, 1], dtype=torch.int32)
    res = _run(ctx, imgs, n, tha, thb, sw.make_params(p=0.65), ia=ia, ib=ib)
    surf = res["surfaces"].view(3, n, n).cpu().numpy()
    srcs = [img, other, const]
    for i in range(3):
        r = O.match_pair(srcs[int(ia[i])].astype(np.float64), srcs[int(ib[i])].astype(np.float64),
                         tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                         return_surface=True)
        g = gpu_record(res, i)
        e = compare(g, r, n, surf[i], "near-constant %d" % i)
        print("  ", i, g["snr"], r["snr"], g["status"], e, flush=True)
        if i < 2:
            assert not g["status"] & sw.ST_DEGENERATE and g["snr"] > 1.0
        else:
            assert g["status"] & sw.ST_DEGENERATE and g["snr"] == 0.0


def _low_contrast_pair(seed, size, mean, sigma, shift):
    """uint8 (or fp32 if mean does not fit a byte) texture of the given mean
    and std; B is A moved by `shift` plus a little noise."""
    g = torch.Generator().manual_seed(seed)
    base = torch.randn((size, size), generator=g)
    base = torch.nn.functional.avg_pool2d(base[None, None], 5, 1, 2)[0, 0]
    base = (base - base.mean()) / base.std()
    a = mean + sigma * base
    b = torch.roll(a, shifts=(shift[1], shift[0]), dims=(0, 1)) + 0.1 * sigma * torch.randn((size, size), generator=g)
    if mean + 6 * sigma < 255:
        return a.round().clamp(0, 255).to(torch.uint8), b.round().clamp(0, 255).to(torch.uint8)
    return a.float(), b.float()


@pytest.mark.parametrize("case", ["bright_u8_512", "dark_u8_512", "offset_f32_256"])
def test_low_contrast_windows(ctx, case):
    """Bright (mean 240, std 2) and dark (mean 12, std 2) uint8 texture at
    512^2, and fp32 texture of mean 1e4 and std 5 at 256^2 (std / mean =
    5e-4): scored, and records as the oracle's."""
    import paper_1612_04787_amd as sw
    print("case low contrast %s" % case, flush=True)
    mean, sigma, n = {"bright_u8_512": (240.0, 2.0, 512), "dark_u8_512": (12.0, 2.0, 512),
                      "offset_f32_256": (1e4, 5.0, 256)}[case]
    size = n + 96
    a, b = _low_contrast_pair(31, size, mean, sigma, (5, -3))
    c = size / 2
    tha = np.array([_ident(c, c), _ident(c, c, 0.375, -0.25)], np.float32)
    thb = np.array([_ident(c, c), _ident(c, c, 1.5, 0.75)], np.float32)
    res = _run(ctx, [a, b], n, tha, thb, sw.make_params(p=0.65))
    surf = res["surfaces"].view(2, n, n).cpu().numpy()
    an, bn = a.numpy().astype(np.float64), b.numpy().astype(np.float64)
    for i in range(2):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                         return_surface=True)
        g = gpu_record(res, i)
        e = compare(g, r, n, surf[i], "%s %d" % (case, i))
        print("  ", i, g["dx"], g["dy"], g["snr"], r["snr"], e, flush=True)
        assert not g["status"] & sw.ST_DEGENERATE and r["snr"] > 5.0


@pytest.mark.parametrize("p", [0.65, 1.0, 0.0])
def test_fp32_scale_invariance_1024(ctx, p):
    """An fp32 source at 1024^2 and the same source times 1e3 (values up to
    2.55e5): the integer peak, the sub-pixel shift and the SNR agree (the
    SNR is invariant to intensity scale), the peak value scales by
    1e3^(2 - 2p), and the scaled record matches the oracle's."""
    import paper_1612_04787_amd as sw
    print("case fp32 scale p=%g" % p, flush=True)
    n = 1024
    a = make_section(1200, 1200, 61).float()
    b = torch.roll(a, shifts=(-3, 5), dims=(0, 1)) + 4.0 * torch.randn((1200, 1200),
                                                                        generator=torch.Generator().manual_seed(3))
    tha = np.array([_ident(600, 600, 0.25, -0.125)], np.float32)
    thb = np.array([_ident(600, 600)], np.float32)
    params = sw.make_params(p=p)
    r1 = _run(ctx, [a, b], n, tha, thb, params, surfaces=False)
    rs = _run(ctx, [a * 1e3, b * 1e3], n, tha, thb, params, surfaces=True)
    g1, gs = gpu_record(r1, 0), gpu_record(rs, 0)
    print("  x1", g1, "\n  x1e3", gs, flush=True)
    assert (g1["ix"], g1["iy"]) == (gs["ix"], gs["iy"])
    assert abs(g1["dx"] - gs["dx"]) <= 1e-3 and abs(g1["dy"] - gs["dy"]) <= 1e-3
    assert abs(g1["snr"] - gs["snr"]) <= 1e-4 * g1["snr"]
    ratio = gs["peak"] / g1["peak"]
    assert abs(ratio / 1e3 ** (2 - 2 * p) - 1) <= 1e-4
    r = O.match_pair((a * 1e3).numpy().astype(np.float64), (b * 1e3).numpy().astype(np.float64),
                     tha[0].astype(np.float64), thb[0].astype(np.float64), n, O.Params(p=p), return_surface=True)
    compare(gs, r, n, rs["surfaces"].view(n, n).cpu().numpy(), "fp32 x1e3 p=%g" % p)


@pytest.mark.parametrize("n,R,max_shift", [(128, 1, 0), (256, 3, 0), (256, 3, 24), (512, 8, 40), (64, 2, 0)])
def test_snr_background_exclusion(ctx, n, R, max_shift):
    """snr_exclude_r = R: the background mean and std leave out the (2R+1)^2
    box around the peak; records as the oracle's, whole search and pruned."""
    import paper_1612_04787_amd as sw
    from datagen import make_section_pair
    print("case snr exclusion n=%d R=%d r=%d" % (n, R, max_shift), flush=True)
    a, b, _, _ = make_section_pair(900, 900, 71, 771, device="cpu", max_shift=5.0)
    rng = np.random.default_rng(n + R)
    k = 3
    tha = np.array([_ident(rng.uniform(n / 2 + 20, 880 - n / 2), rng.uniform(n / 2 + 20, 880 - n / 2),
                           rng.uniform(-1, 1), rng.uniform(-1, 1)) for _ in range(k)], np.float32)
    thb = tha.copy()
    params = sw.make_params(p=0.65, snr_exclude_r=R, max_shift=max_shift)
    res = _run(ctx, [a, b], n, tha, thb, params, surfaces=max_shift == 0)
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                         O.Params(p=0.65, snr_exclude_r=R, max_shift=max_shift), return_surface=True)
        g = gpu_record(res, i)
        e = compare(g, r, n, None, "exclude n=%d R=%d %d" % (n, R, i))
        full = O.peak_stats(r["surface"])
        print("  ", i, g["snr"], r["snr"], "whole-surface snr", full["snr"], e, flush=True)


def test_snr_entry_exclusion(ctx):
    """swift_snr with snr_exclude_r = 2 on given surfaces against the
    oracle's peak_stats; a box wider than the surface is refused."""
    import paper_1612_04787_amd as sw
    print("case swift_snr exclusion", flush=True)
    rng = np.random.default_rng(5)
    n, B = 64, 4
    s = rng.standard_normal((B, n, n)).astype(np.float32)
    for q in range(B):
        y, x = rng.integers(0, n, 2)
        s[q, y, x] += 12.0
        s[q, (y + 1) % n, x] += 5.0
        s[q, y, (x - 1) % n] += 4.0
    out = ctx.snr(torch.from_numpy(s).to(dev()), sw.make_params(snr_exclude_r=2))
    torch.cuda.synchronize()
    for q in range(B):
        r = O.peak_stats(s[q].astype(np.float64), exclude_r=2)
        assert (int(out["ix"][q]), int(out["iy"][q])) == (r["ix"], r["iy"])
        assert abs(float(out["snr"][q]) - r["snr"]) <= 1e-4 * r["snr"]
        assert abs(float(out["mean"][q]) - r["mean"]) <= 1e-6 and abs(float(out["std"][q]) - r["std"]) <= 1e-6
        assert abs(float(out["dx"][q]) - r["dx"]) <= 1e-4 and abs(float(out["dy"][q]) - r["dy"]) <= 1e-4
    with pytest.raises(sw.SwiftError):
        ctx.snr(torch.zeros((1, 8, 8), device=dev()), sw.make_params(snr_exclude_r=4))


def test_exclusion_refused_where_undefined(ctx):
    """The adjoint entry points and the Pearson mode take the whole surface:
    snr_exclude_r > 0 is refused there, and out of range everywhere."""
    import paper_1612_04787_amd as sw
    print("case exclusion validation", flush=True)
    a = make_section(300, 300, 5)
    th = torch.tensor([_ident(150, 150)], dtype=torch.float32)
    z = torch.zeros(1, dtype=torch.int32)
    res = ctx.match_batch([a.to(dev())], [128], z, z, th, th, sw.make_params(), save=True)
    with pytest.raises(sw.SwiftError) as ei:
        ctx.match_backward(res, sw.make_params(snr_exclude_r=1), None, torch.ones(1, device=dev()))
    assert ei.value.code == -2
    with pytest.raises(sw.SwiftError):
        ctx.match_batch([a.to(dev())], [128], z, z, th, th, sw.make_params(snr_exclude_r=1, flags=sw.FLAG_PEARSON))
    with pytest.raises(sw.SwiftError):
        ctx.match_batch([a.to(dev())], [128], z, z, th, th, sw.make_params(snr_exclude_r=9))


def test_tune_cache_round_trip(ctx, tmp_path):
    """swift_autotune writes the plans it finds to the context's tune cache;
    a new context on the same file starts with them; other devices' lines are
    kept."""
    import paper_1612_04787_amd as sw
    print("case tune cache", flush=True)
    path = str(tmp_path / "plans.txt")
    with open(path, "w") as f:
        f.write("otherdevice/cu4 64 1 1\n")
    c1 = sw.Swift(0, tune_cache=path)
    c1.plan(64, 1, 1)
    c1.autotune(sizes=[64, 256], pairs_per_size=256)
    p64, p256 = c1.plan(64), c1.plan(256)
    c1.close()
    text = open(path).read()
    print(text, flush=True)
    assert "otherdevice/cu4 64 1 1" in text
    mine = [ln.split() for ln in text.splitlines() if ln and not ln.startswith("#") and "otherdevice" not in ln]
    assert sorted(int(t[1]) for t in mine) == [64, 256]
    c2 = sw.Swift(0, tune_cache=path)
    assert c2.plan(64) == p64 and c2.plan(256) == p256
    c2.close()
    c3 = sw.Swift(0, tune_cache=os.path.join(str(tmp_path), "absent.txt"))  # a missing file is not an error
    c3.close()
