"""GPU parity of the HIP match path (through the C ABI) against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from datagen import make_pair64, make_section, make_section_pair
from parity_util import compare, gpu_record

pytestmark = pytest.mark.gpu
SIZES = (64, 128, 256, 512, 1024)


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def _params(p, eps=1e-4, taper=0.25):
    import paper_1612_04787_amd as sw
    return sw.make_params(p=p, eps_rel=eps, taper_frac=taper)


@pytest.mark.parametrize("p", [0.0, 0.5, 1.0])
def test_pair64(ctx, p):
    print("case pair64 p=%g" % p, flush=True)
    a, b = make_pair64()
    th = torch.tensor([[32, 32, 1, 0, 0, 0, 1, 0]], dtype=torch.float32)
    res = ctx.match_batch([torch.from_numpy(a).to(dev()), torch.from_numpy(b).to(dev())], [64],
                          torch.tensor([0]), torch.tensor([1]), th, th, _params(p), surfaces=True)
    torch.cuda.synchronize()
    g = gpu_record(res, 0)
    r = O.match_pair(a.astype(np.float64), b.astype(np.float64), th[0].double().numpy(), th[0].double().numpy(),
                     64, O.Params(p=p), return_surface=True)
    e = compare(g, r, 64, res["surfaces"].view(64, 64).cpu().numpy(), "pair64")
    assert (g["iy"], g["ix"]) == (61, 7)
    print("  errors", e, flush=True)


def _random_thetas(rng, k, n, h, w, edge=False):
    th = np.zeros((k, 8), np.float32)
    for i in range(k):
        ang = math.radians(rng.uniform(-0.5, 0.5))
        s = 1 + rng.uniform(-0.002, 0.002)
        m = s * np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
        cx = rng.uniform(n / 2 + 8, w - n / 2 - 8)
        cy = rng.uniform(n / 2 + 8, h - n / 2 - 8)
        if edge and i == k - 1:
            cx, cy = n / 2 - 5.5, h - n / 2 + 3.25  # partly outside: clamped reads
        th[i] = [cx, cy, m[0, 0], m[0, 1], rng.uniform(-3, 3), m[1, 0], m[1, 1], rng.uniform(-3, 3)]
    return th


@pytest.fixture(scope="module")
def section_pair_small():
    a, b, m, bv = make_section_pair(1600, 1600, 31, 331, device="cpu", max_shift=6.0)
    return a, b


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [0.65, 0.0, 1.0])
def test_sizes_random_affines(ctx, section_pair_small, n, p):
    print("case sizes n=%d p=%g" % (n, p), flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(1000 + n + int(100 * p))
    k = {64: 8, 128: 6, 256: 4, 512: 3, 1024: 2}[n]
    tha = _random_thetas(rng, k, n, 1600, 1600, edge=True)
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb),
                          _params(p), surfaces=True)
    torch.cuda.synchronize()
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=p),
                         return_surface=True)
        e = compare(gpu_record(res, i), r, n, surf[i], "n=%d p=%g i=%d" % (n, p, i))
        print("  ", i, e, flush=True)


@pytest.mark.parametrize("n", SIZES)
def test_translation_windows(ctx, section_pair_small, n):
    """Windows with an identity linear part (the constant-weight gather):
    fractional translations on both sides, one window partly outside the
    section (clamped reads), one at an integer position."""
    print("case translation n=%d" % n, flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(3000 + n)
    k = {64: 6, 128: 5, 256: 4, 512: 3, 1024: 3}[n]
    tha = np.zeros((k, 8), np.float32)
    for i in range(k):
        tha[i] = [rng.uniform(n / 2 + 8, 1600 - n / 2 - 8), rng.uniform(n / 2 + 8, 1600 - n / 2 - 8), 1, 0,
                  rng.uniform(-3, 3), 0, 1, rng.uniform(-3, 3)]
    tha[-1] = [n / 2 - 5.5, 1600 - n / 2 + 3.25, 1, 0, 0.375, 0, 1, -0.625]
    tha[0, 4] = tha[0, 7] = 0.0
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-2, 2, k).astype(np.float32)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb),
                          _params(0.65), surfaces=True)
    torch.cuda.synchronize()
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                         return_surface=True)
        e = compare(gpu_record(res, i), r, n, surf[i], "translation n=%d i=%d" % (n, i))
        print("  ", i, e, flush=True)
    assert int(res["status"][k - 1]) & O.swift_oracle.STATUS_CLAMPED


def test_ragged_batch_all_sizes(ctx, section_pair_small):
    print("case ragged", flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(77)
    ns, tha = [], []
    for n in SIZES:
        for t in _random_thetas(rng, 2, n, 1600, 1600):
            ns.append(n)
            tha.append(t)
    tha = np.array(tha, np.float32)
    P = len(ns)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], ns, torch.zeros(P, dtype=torch.int32),
                          torch.ones(P, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(tha),
                          _params(0.65), surfaces=True)
    torch.cuda.synchronize()
    flat = res["surfaces"].cpu().numpy()
    off = 0
    for i, n in enumerate(ns):
        r = O.match_pair(a.numpy(), b.numpy(), tha[i].astype(np.float64), tha[i].astype(np.float64), n,
                         O.Params(p=0.65), return_surface=True)
        g = gpu_record(res, i)
        assert g["n"] == n
        compare(g, r, n, flat[off:off + n * n].reshape(n, n), "ragged i=%d n=%d" % (i, n))
        off += n * n


def test_degenerate_constant_window(ctx):
    print("case degenerate", flush=True)
    a = torch.full((300, 300), 77, dtype=torch.uint8, device=dev())
    b = make_section(300, 300, 5, device="cpu").to(dev())
    th = torch.tensor([[150, 150, 1, 0, 0, 0, 1, 0]] * 2, dtype=torch.float32)
    res = ctx.match_batch([a, b], [128, 128], torch.tensor([0, 1]), torch.tensor([1, 0]), th, th, _params(0.65))
    torch.cuda.synchronize()
    for i in range(2):
        g = gpu_record(res, i)
        assert g["status"] & 2 and g["snr"] == 0.0 and g["std"] == 0.0, g
        assert (g["ix"], g["iy"]) == (0, 0) and g["dx"] == 0.0 and g["dy"] == 0.0


def test_empty_batch_and_validation(ctx):
    import paper_1612_04787_amd as sw
    print("case empty/validation", flush=True)
    a = make_section(256, 256, 6).to(dev())
    e = torch.zeros(0, dtype=torch.int32, device=dev())
    t = torch.zeros((0, 8), dtype=torch.float32, device=dev())
    res = ctx.match_batch([a], [], e, e, t, t, _params(0.5))
    assert res["dx"].numel() == 0
    th = torch.tensor([[128, 128, 1, 0, 0, 0, 1, 0]], dtype=torch.float32)
    with pytest.raises(sw.SwiftError) as ei:
        ctx.match_batch([a], [64], torch.tensor([0]), torch.tensor([0]), th, th, _params(1.5))
    assert ei.value.code == -1
    with pytest.raises(sw.SwiftError) as ei:
        ctx.match_batch([a], [64], torch.tensor([0]), torch.tensor([0]), th, th,
                        sw.make_params(p=0.5, centroid_r=2))
    assert ei.value.code == -2


def test_snr_entry_point(ctx):
    print("case snr", flush=True)
    rng = np.random.default_rng(5)
    n = 128
    surfs = []
    for i in range(4):
        wA, _ = O.prepare(rng.standard_normal((n, n)), O.taper_2d(n, 0.25))
        wB = np.roll(wA, (3 * i - 2, 5 - i), axis=(0, 1)) + 0.3 * rng.standard_normal((n, n))
        surfs.append(O.whitened_surface(wA, wB, 0.65, 1e-4))
    s32 = np.stack(surfs).astype(np.float32)
    res = ctx.snr(torch.from_numpy(s32).to(dev()), _params(0.65))
    torch.cuda.synchronize()
    for i in range(4):
        r = O.peak_stats(s32[i].astype(np.float64))
        g = {k: res[k][i].item() for k in res}
        assert (g["ix"], g["iy"]) == (r["ix"], r["iy"])
        assert abs(g["dx"] - r["dx"]) < 1e-5 and abs(g["dy"] - r["dy"]) < 1e-5
        assert abs(g["snr"] - r["snr"]) < 1e-5 * r["snr"]
        assert abs(g["std"] - r["std"]) < 1e-9 * r["std"]


@pytest.mark.parametrize("w", [48, 45])
@pytest.mark.parametrize("k", [1, 2, 3, 8])
def test_project_bit_exact(ctx, w, k):
    print("case project w=%d k=%d" % (w, k), flush=True)
    rng = np.random.default_rng(w * 10 + k)
    st = rng.integers(0, 256, size=(11, 37, w)).astype(np.uint8)
    excl = np.zeros(11, bool)
    excl[4] = True
    out = ctx.project(torch.from_numpy(st).to(dev()), k=k, exclude=excl)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for s in range(11):
        try:
            ref = O.project(st, s, k, excl)
        except ValueError:
            ref = np.zeros_like(st[0])
        np.testing.assert_array_equal(got[s], ref, err_msg="s=%d" % s)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_project_extremes(ctx, k):
    # near-saturated sums and every neighbour count from 1 to 2k: sections of
    # 255 with a sprinkling of 254/0 pixels, 14 sections (a whole number of
    # rounds for k = 3) and an exclusion pattern that thins the windows
    print("case project extremes k=%d" % k, flush=True)
    rng = np.random.default_rng(400 + k)
    S = 14
    st = np.full((S, 9, 64), 255, np.uint8)
    st[rng.random(st.shape) < 0.2] = 254
    st[rng.random(st.shape) < 0.05] = 0
    excl = np.zeros(S, bool)
    excl[[1, 5, 6, 12]] = True
    out = ctx.project(torch.from_numpy(st).to(dev()), k=k, exclude=excl).cpu().numpy()
    for s in range(S):
        try:
            ref = O.project(st, s, k, excl)
        except ValueError:
            ref = np.zeros_like(st[0])
        np.testing.assert_array_equal(out[s], ref, err_msg="s=%d" % s)


@pytest.mark.parametrize("hw", [(64, 96), (37, 51)])
def test_pyramid_bit_exact(ctx, hw):
    print("case pyramid", hw, flush=True)
    rng = np.random.default_rng(sum(hw))
    img = rng.integers(0, 256, size=hw).astype(np.uint8)
    got = ctx.pyramid(torch.from_numpy(img).to(dev()))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), O.pyramid(img))


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("rot_deg", [0.4, 4.0])
def test_rotated_windows_tile_and_direct_gather(ctx, section_pair_small, n, rot_deg):
    """Small rotations gather through the LDS source tile, large ones straight
    from global memory; both must match the oracle."""
    print("case rotation n=%d rot=%g" % (n, rot_deg), flush=True)
    a, b = section_pair_small
    k = 3
    th = np.zeros((k, 8), np.float32)
    for i in range(k):
        ang = math.radians(rot_deg * (1 if i % 2 == 0 else -1))
        th[i] = [700 + 60 * i, 800 - 40 * i, math.cos(ang), -math.sin(ang), 0.37 * i, math.sin(ang),
                 math.cos(ang), -0.21 * i]
    thb = th.copy()
    thb[:, 2:4] = [1, 0]
    thb[:, 5:7] = [0, 1]
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(th), torch.from_numpy(thb),
                          _params(0.65), surfaces=True)
    torch.cuda.synchronize()
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    for i in range(k):
        r = O.match_pair(a.numpy(), b.numpy(), th[i].astype(np.float64), thb[i].astype(np.float64), n,
                         O.Params(p=0.65), return_surface=True)
        compare(gpu_record(res, i), r, n, surf[i], "rot n=%d i=%d" % (n, i))


@pytest.mark.parametrize("n", [256, 512])
def test_mixed_tile_and_direct_images(ctx, section_pair_small, n):
    """Pairs whose two images take different gathers: a 16-aligned uint8
    section (LDS source tile), the same section cut to an odd width and an
    fp32 copy (both gathered straight from memory).  Covers every order of
    tiled and direct images within one workgroup."""
    print("case mixed tile/direct n=%d" % n, flush=True)
    a, b = section_pair_small
    b_odd = b[:, :1599].contiguous()
    a_f32 = a.to(torch.float32)
    imgs = [a, b, b_odd, a_f32]
    pairs = [(0, 2), (2, 0), (3, 2), (0, 1), (3, 1)]
    k = len(pairs)
    rng = np.random.default_rng(4100 + n)
    tha = np.zeros((k, 8), np.float32)
    for i in range(k):
        tha[i] = [rng.uniform(n / 2 + 8, 1599 - n / 2 - 8), rng.uniform(n / 2 + 8, 1600 - n / 2 - 8), 1, 0,
                  rng.uniform(-3, 3), 0, 1, rng.uniform(-3, 3)]
    tha[1, 2:4] = [math.cos(0.004), -math.sin(0.004)]  # a general affine on one side
    tha[1, 5:7] = [math.sin(0.004), math.cos(0.004)]
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    ia = torch.tensor([p[0] for p in pairs], dtype=torch.int32)
    ib = torch.tensor([p[1] for p in pairs], dtype=torch.int32)
    res = ctx.match_batch([x.to(dev()) for x in imgs], [n] * k, ia, ib, torch.from_numpy(tha),
                          torch.from_numpy(thb), _params(0.65), surfaces=True)
    torch.cuda.synchronize()
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    host = [x.numpy().astype(np.float64) for x in imgs]
    for i, (pa, pb) in enumerate(pairs):
        r = O.match_pair(host[pa], host[pb], tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                         O.Params(p=0.65), return_surface=True)
        e = compare(gpu_record(res, i), r, n, surf[i], "mixed n=%d i=%d (%d,%d)" % (n, i, pa, pb))
        print("  ", i, e, flush=True)


@pytest.mark.parametrize("n", [128, 512])
@pytest.mark.parametrize("p,eps,taper", [(1.0, 0.0, 0.25), (0.65, 0.0, 0.0), (0.0, 1e-4, 1.0), (0.65, 1e-2, 0.5)])
def test_parameter_edge_cases(ctx, section_pair_small, n, p, eps, taper):
    """No whitening floor (eps = 0), no taper (T = 1: the deferred mean falls
    entirely on the DC term), a taper over the whole window, a large floor;
    translation and affine windows, one wholly outside the section (every
    sample clamped to the border)."""
    print("case params n=%d p=%g eps=%g taper=%g" % (n, p, eps, taper), flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(int(5000 + n + 100 * p + 1e4 * eps + 10 * taper))
    k = 3
    tha = _random_thetas(rng, k, n, 1600, 1600)
    tha[0, 2:4] = [1, 0]
    tha[0, 5:7] = [0, 1]
    tha[2, 0:2] = [-n - 40.5, 1600 + n + 17.25]  # outside: all samples clamped
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb),
                          _params(p, eps=eps, taper=taper), surfaces=True)
    torch.cuda.synchronize()
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    for i in range(k):
        r = O.match_pair(a.numpy(), b.numpy(), tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                         O.Params(p=p, eps_rel=eps, taper_frac=taper), return_surface=True)
        g = gpu_record(res, i)
        if r["status"] & O.swift_oracle.STATUS_DEGENERATE:
            # a constant window: sigma = 0, SNR 0, flagged on both sides
            assert g["status"] & O.swift_oracle.STATUS_DEGENERATE and g["snr"] == 0.0, (i, g)
            continue
        e = compare(g, r, n, surf[i], "params n=%d i=%d" % (n, i))
        print("  ", i, e, flush=True)
    assert int(res["status"][2]) & O.swift_oracle.STATUS_CLAMPED
