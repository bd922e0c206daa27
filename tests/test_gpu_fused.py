"""The one-workgroup match (forward plan variant 2, n = 64 and 128: the pair's
packed spectrum stays in LDS) against the FP64 oracle, and against the
five-kernel path on a section-sized batch."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from datagen import make_section, make_section_pair
from parity_util import compare, gpu_record

pytestmark = pytest.mark.gpu
FUSED = 2
SMALL = (64, 128)


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    for n in SMALL:
        c.plan(n, FUSED, 0, 1)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx5():
    """The five-kernel path for the same sizes."""
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    for n in SMALL:
        c.plan(n, 0, 0, 1)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def _run(ctx, images, n, tha, thb, params, surfaces=True, ia=None, ib=None, save=False):
    k = tha.shape[0]
    ia = torch.zeros(k, dtype=torch.int32) if ia is None else ia
    ib = torch.ones(k, dtype=torch.int32) if ib is None else ib
    res = ctx.match_batch([im.to(dev()) for im in images], [n] * k, ia, ib, torch.from_numpy(tha),
                          torch.from_numpy(thb), params, surfaces=surfaces, save=save)
    torch.cuda.synchronize()
    return res


def _ident(cx, cy, tx=0.0, ty=0.0):
    return [cx, cy, 1, 0, tx, 0, 1, ty]


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
    a, b, _, _ = make_section_pair(1600, 1600, 31, 331, device="cpu", max_shift=6.0)
    return a, b


def test_plan_reports_the_one_workgroup_variant(ctx):
    import paper_1612_04787_amd as sw
    for n in SMALL:
        assert ctx.plan(n, full=True) == (n, n, 1)
    with pytest.raises(sw.SwiftError):
        ctx.plan(256, FUSED)
    fresh = sw.Swift(0)
    try:
        assert fresh.plan(64, full=True) == (64, 64, 1)  # the default at n = 64
        assert fresh.plan(128, full=True)[0] < 128
    finally:
        fresh.close()


@pytest.mark.parametrize("plan", ["fused", "five"])
@pytest.mark.parametrize("n", SMALL)
@pytest.mark.parametrize("p", [0.65, 0.0, 1.0])
def test_random_affines(request, section_pair_small, n, p, plan):
    """Affine windows (one partly outside the section), records and whole
    surfaces against the oracle, through either plan."""
    import paper_1612_04787_amd as sw
    ctx = request.getfixturevalue("ctx" if plan == "fused" else "ctx5")
    print("case %s affines n=%d p=%g" % (plan, n, p), flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(5000 + n + int(100 * p))
    k = 8
    tha = _random_thetas(rng, k, n, 1600, 1600, edge=True)
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    res = _run(ctx, [a, b], n, tha, thb, sw.make_params(p=p))
    surf = res["surfaces"].view(k, n, n).cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=p),
                         return_surface=True)
        e = compare(gpu_record(res, i), r, n, surf[i], "fused n=%d p=%g i=%d" % (n, p, i))
        print("  ", i, e, flush=True)


@pytest.mark.parametrize("n", SMALL)
def test_translation_windows_and_fp32_source(ctx, section_pair_small, n):
    """Translation windows (fractional and integer offsets, one clamped) on
    uint8 sections, and the same windows on fp32 copies scaled by 1e3."""
    import paper_1612_04787_amd as sw
    print("case fused translation n=%d" % n, flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(6000 + n)
    k = 5
    tha = np.array([_ident(rng.uniform(n / 2 + 8, 1592 - n / 2), rng.uniform(n / 2 + 8, 1592 - n / 2),
                           rng.uniform(-3, 3), rng.uniform(-3, 3)) for _ in range(k)], np.float32)
    tha[-1] = _ident(n / 2 - 5.5, 1600 - n / 2 + 3.25, 0.375, -0.625)
    tha[0, 4] = tha[0, 7] = 0.0
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-2, 2, k).astype(np.float32)
    for scale, imgs in ((1.0, [a, b]), (1e3, [a.float() * 1e3, b.float() * 1e3])):
        res = _run(ctx, imgs, n, tha, thb, sw.make_params(p=0.65))
        surf = res["surfaces"].view(k, n, n).cpu().numpy()
        an, bn = (imgs[0].numpy().astype(np.float64), imgs[1].numpy().astype(np.float64))
        for i in range(k):
            r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                             return_surface=True)
            e = compare(gpu_record(res, i), r, n, surf[i], "fused translation n=%d x%g i=%d" % (n, scale, i))
            print("  ", scale, i, e, flush=True)


def test_near_constant_and_constant_windows(ctx):
    """A 64^2 window of 200 with one pixel at 201 is scored like the oracle;
    a constant window is degenerate (SNR 0)."""
    import paper_1612_04787_amd as sw
    print("case fused near-constant", flush=True)
    n = 64
    img = np.full((96, 96), 200, np.uint8)
    img[40, 37] = 201
    other = np.full((96, 96), 200, np.uint8)
    other[43, 36] = 201
    const = np.full((96, 96), 200, np.uint8)
    tha = np.array([_ident(48, 48), _ident(48, 48, 0.25, -0.5), _ident(48, 48)], np.float32)
    thb = np.array([_ident(48, 48), _ident(48, 48, -2.0, 1.5), _ident(48, 48)], np.float32)
    imgs = [torch.from_numpy(img), torch.from_numpy(other), torch.from_numpy(const)]
    ia = torch.tensor([0, 0, 2], dtype=torch.int32)
    ib = torch.tensor([1, 1, 1], dtype=torch.int32)
    res = _run(ctx, imgs, n, tha, thb, sw.make_params(p=0.65), ia=ia, ib=ib)
    surf = res["surfaces"].view(3, n, n).cpu().numpy()
    srcs = [img, other, const]
    for i in range(3):
        r = O.match_pair(srcs[int(ia[i])].astype(np.float64), srcs[int(ib[i])].astype(np.float64),
                         tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                         return_surface=True)
        g = gpu_record(res, i)
        compare(g, r, n, surf[i], "fused near-constant %d" % i)
        if i < 2:
            assert not g["status"] & sw.ST_DEGENERATE and g["snr"] > 1.0
        else:
            assert g["status"] & sw.ST_DEGENERATE and g["snr"] == 0.0


@pytest.mark.parametrize("n,R,max_shift", [(64, 2, 0), (128, 1, 0), (128, 3, 20), (64, 0, 12), (128, 8, 0)])
def test_exclusion_and_pruned_search(ctx, n, R, max_shift):
    """snr_exclude_r and max_shift: the background leaves out the box, the
    peak is searched within the radius."""
    import paper_1612_04787_amd as sw
    print("case fused exclusion n=%d R=%d r=%d" % (n, R, max_shift), flush=True)
    a, b, _, _ = make_section_pair(900, 900, 71, 771, device="cpu", max_shift=5.0)
    rng = np.random.default_rng(700 + n + R + max_shift)
    k = 4
    tha = np.array([_ident(rng.uniform(n / 2 + 20, 880 - n / 2), rng.uniform(n / 2 + 20, 880 - n / 2),
                           rng.uniform(-1, 1), rng.uniform(-1, 1)) for _ in range(k)], np.float32)
    thb = tha.copy()
    params = sw.make_params(p=0.65, snr_exclude_r=R, max_shift=max_shift)
    res = _run(ctx, [a, b], n, tha, thb, params, surfaces=False)
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                         O.Params(p=0.65, snr_exclude_r=R, max_shift=max_shift), return_surface=True)
        e = compare(gpu_record(res, i), r, n, None, "fused exclude n=%d R=%d r=%d %d" % (n, R, max_shift, i))
        print("  ", i, e, flush=True)


@pytest.mark.parametrize("n", SMALL)
def test_adjoint_from_the_fused_forward(ctx, n):
    """The adjoint reads the state the one-workgroup forward saves: gradients
    as the oracle's chain rule (normalised parameters, 1e-3)."""
    import paper_1612_04787_amd as sw
    print("case fused adjoint n=%d" % n, flush=True)
    a, b, _, _ = make_section_pair(1200, 1200, 41, 441, device="cpu", max_shift=4.0)
    rng = np.random.default_rng(80 + n)
    k = 3
    ta = np.zeros((k, 8), np.float32)
    tb = np.zeros((k, 8), np.float32)
    for i in range(k):
        cx, cy = rng.uniform(n / 2 + 20, 1180 - n / 2, 2)
        e = rng.uniform(-1e-3, 1e-3, 4)
        ta[i] = [cx, cy, 1 + e[0], e[1], rng.uniform(-0.5, 0.5), e[2], 1 + e[3], rng.uniform(-0.5, 0.5)]
        tb[i] = [cx, cy, 1, 0, rng.uniform(-1, 1), 0, 1, rng.uniform(-1, 1)]
    params = sw.make_params(p=0.65)
    res = _run(ctx, [a, b], n, ta, tb, params, surfaces=False, save=True)
    gpk = torch.full((k,), 0.3, device=dev())
    gsn = torch.full((k,), -0.7, device=dev())
    ga, gb, _ = ctx.match_backward(res, params, gpk, gsn, want_hess=True)
    torch.cuda.synchronize()
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    s = np.array([2.0 / n, 2.0 / n, 1.0, 2.0 / n, 2.0 / n, 1.0])
    checked = 0
    for i in range(k):
        rec, ra, rb = O.match_grad(a.numpy(), b.numpy(), ta[i].astype(np.float64), tb[i].astype(np.float64), n,
                                   O.Params(p=0.65), g_peak=0.3, g_snr=-0.7)
        if (rec["peak"] - rec["second"]) <= 2e-4 * abs(rec["peak"]):
            continue
        for g_gpu, g_ref, tag in ((ga[i], ra, "A"), (gb[i], rb, "B")):
            err = np.linalg.norm((g_gpu - g_ref) * s) / np.linalg.norm(g_ref * s)
            print("   ", i, tag, "rel err %.2e" % err, flush=True)
            assert err <= 1e-3, (i, tag, err)
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("n", SMALL)
def test_section_batch_against_five_kernel_path(ctx, ctx5, n):
    """2048 affine windows of a 4096^2 section pair (some clamped) through
    both plans: the same integer peaks away from near ties, and records that
    agree to FP32 rounding; three sampled pairs against the oracle."""
    import paper_1612_04787_amd as sw
    print("case fused vs five-kernel n=%d" % n, flush=True)
    a, b, _, _ = make_section_pair(4096, 4096, 51, 551, device=dev(), max_shift=6.0)
    rng = np.random.default_rng(900 + n)
    k = 2048
    tha = _random_thetas(rng, k, n, 4096, 4096)
    tha[:16, 0] = rng.uniform(-n / 4, n / 2, 16)  # clamped reads at the left edge
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-3, 3, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-3, 3, k).astype(np.float32)
    params = sw.make_params(p=0.65)
    rf = _run(ctx, [a, b], n, tha, thb, params, surfaces=False)
    r5 = _run(ctx5, [a, b], n, tha, thb, params, surfaces=False)
    tie = ((rf["status"] | r5["status"]) & sw.ST_NEAR_TIE) != 0
    same = (rf["ix"] == r5["ix"]) & (rf["iy"] == r5["iy"])
    assert bool((same | tie).all()), int((~same & ~tie).sum())
    assert torch.equal(rf["status"] & sw.ST_CLAMPED, r5["status"] & sw.ST_CLAMPED)
    assert int((rf["status"] & sw.ST_CLAMPED != 0).sum()) >= 8
    m = same & ~tie
    snr_rel = ((rf["snr"] - r5["snr"]).abs() / r5["snr"].abs().clamp_min(1e-12))[m]
    dd = torch.maximum((rf["dx"] - r5["dx"]).abs(), (rf["dy"] - r5["dy"]).abs())[m]
    print("  max snr rel %.2e, max shift diff %.2e px" % (float(snr_rel.max()), float(dd.max())), flush=True)
    assert float(snr_rel.max()) <= 1e-4
    assert float(dd.max()) <= 1e-3
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    for i in (3, 700, 2047):
        r = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, O.Params(p=0.65),
                         return_surface=True)
        compare(gpu_record(rf, i), r, n, None, "fused section n=%d i=%d" % (n, i))


def test_graph_replay_matches_direct_call(ctx):
    """A ragged batch (64 and 128 one-workgroup groups beside 256) captured as
    a graph and replayed three times gives the direct call's records."""
    import paper_1612_04787_amd as sw
    print("case fused graph", flush=True)
    a = make_section(1024, 1024, 61, device=dev())
    rng = np.random.default_rng(61)
    n_list = [64] * 40 + [128] * 30 + [256] * 10
    k = len(n_list)
    th = np.zeros((k, 8), np.float32)
    for i, n in enumerate(n_list):
        th[i] = _ident(rng.uniform(n / 2, 1024 - n / 2), rng.uniform(n / 2, 1024 - n / 2))
    thb = th.copy()
    thb[:, 4] += rng.uniform(-2, 2, k).astype(np.float32)
    prm = sw.make_params(p=0.65, flags=sw.FLAG_CONCURRENT_SIZES)
    ia = torch.zeros(k, dtype=torch.int32)
    prep = ctx.prepare([a], n_list, ia, ia, torch.from_numpy(th), torch.from_numpy(thb))
    need, _ = ctx.workspace_size(prep["pairs"], prm)
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    out_d = torch.empty((k, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
    out_g = torch.empty_like(out_d)
    ctx.match_batch_raw(prep["table"], 1, prep["pairs"], prm, out_d, ws=ws)
    torch.cuda.synchronize()
    for _ in range(3):
        out_g.zero_()
        ctx.match_batch_raw(prep["table"], 1, prep["pairs"], prm, out_g, ws=ws, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_d)
