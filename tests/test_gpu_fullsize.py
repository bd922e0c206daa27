"""Parity at full size, in the launch configuration the benchmark times: the
whole batch goes through the C ABI in one call and sampled outputs are checked
one by one against the FP64 oracle (which reads the same input bytes, cropped
with a margin that reproduces every read of the window, including clamped
reads at the section border).  Properties that hold for every output are
checked on all of them."""
import numpy as np
import pytest
import torch

import oracle as O
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


def _crop(cx, cy, n, H, W, m=4):
    x0, y0 = int(max(cx - n // 2 - m, 0)), int(max(cy - n // 2 - m, 0))
    x1, y1 = int(min(cx + n // 2 + m, W)), int(min(cy + n // 2 + m, H))
    return x0, y0, x1, y1


def _check_all_records(res, n, P):
    assert res["n"].shape[0] == P
    assert bool((res["n"] == n).all())
    for key in ("dx", "dy", "peak", "snr"):
        assert bool(torch.isfinite(res[key]).all()), key
    assert bool((res["std"] > 0).all())
    assert bool((res["snr"] > 0).all())
    # the record's shift is the wrapped integer peak plus a centroid inside the 3 x 3 box
    ix, iy = res["ix"].long(), res["iy"].long()
    sx = torch.where(ix >= n // 2, ix - n, ix).float()
    sy = torch.where(iy >= n // 2, iy - n, iy).float()
    assert bool(((res["dx"] - sx).abs() <= 1.0).all()) and bool(((res["dy"] - sy).abs() <= 1.0).all())


def test_headline_batch_4096_pairs_512(ctx):
    """64 sections of 4096^2 (drift + affine distortion), references = +-3
    z-projections, 8 x 8 windows of 512^2 per section: 4096 pairs in one call."""
    import paper_1612_04787_amd as sw
    from datagen.workloads import distorted_stack, section_grid_pairs
    S, size, n, k = 64, 4096, 512, 3
    print("case headline generate", flush=True)
    stack, _ = distorted_stack(S, size, seed=5, device=dev())
    refs = ctx.project(stack, k=k)
    images = [stack[s] for s in range(S)] + [refs[s] for s in range(S)]
    n_list, ia, ib, ta, tb, cen = section_grid_pairs(S, size, n, 8, dev())
    P = len(n_list)
    print("case headline match P=%d" % P, flush=True)
    res = ctx.match_batch(images, n_list, ia, ib, ta, tb, sw.make_params(p=0.65))
    torch.cuda.synchronize()
    _check_all_records(res, n, P)
    rng = np.random.default_rng(2024)
    picks = rng.choice(P, 12, replace=False)
    for i in picks:
        s, w = int(i) // len(cen), int(i) % len(cen)
        cx, cy = cen[w]
        x0, y0, x1, y1 = _crop(cx, cy, n, size, size)
        lo, hi = max(0, s - k), min(S, s + k + 1)
        sub = stack[lo:hi, y0:y1, x0:x1].cpu().numpy()
        ref_o = O.project(sub, s - lo, k)
        ref_g = refs[s, y0:y1, x0:x1].cpu().numpy()
        assert np.array_equal(ref_g, ref_o), ("projection", s, w)
        th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
        r = O.match_pair(sub[s - lo], ref_o, th, th, n, O.Params(p=0.65))
        e = compare(gpu_record(res, int(i)), r, n, tag="headline pair %d" % i)
        print("   pair %d (section %d window %d):" % (i, s, w), e, flush=True)
    # the same batch with the pruned inverse at the benchmark's radius n/8
    print("case headline pruned r=%d" % (n // 8), flush=True)
    rp = ctx.match_batch(images, n_list, ia, ib, ta, tb, sw.make_params(p=0.65, max_shift=n // 8))
    torch.cuda.synchronize()
    _check_all_records(rp, n, P)
    assert bool((rp["mean"] == 0).all())
    for i in picks:
        s, w = int(i) // len(cen), int(i) % len(cen)
        cx, cy = cen[w]
        x0, y0, x1, y1 = _crop(cx, cy, n, size, size)
        lo, hi = max(0, s - k), min(S, s + k + 1)
        sub = stack[lo:hi, y0:y1, x0:x1].cpu().numpy()
        ref_o = O.project(sub, s - lo, k)
        th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
        r = O.match_pair(sub[s - lo], ref_o, th, th, n, O.Params(p=0.65, max_shift=n // 8))
        e = compare(gpu_record(rp, int(i)), r, n, tag="pruned pair %d" % i)
        print("   pruned pair %d:" % i, e, flush=True)
    # every shift of this batch lies well inside the radius: the pruned records
    # agree with the full ones on all pairs (peak exact, background to rounding)
    same = (rp["ix"] == res["ix"]) & (rp["iy"] == res["iy"])
    assert float(same.float().mean()) > 0.999
    assert float((rp["dx"] - res["dx"])[same].abs().max()) <= 0.01
    assert float(((rp["snr"] - res["snr"]) / res["snr"]).abs().max()) <= 1e-3


def test_section_pair_256_windows_1024(ctx):
    """A 16384^2 section pair (B = bilinear affine warp of A plus noise) on a
    16 x 16 grid of 1024^2 windows: 256 pairs in one call; sampled windows
    against the oracle, and every window's shift against the known warp."""
    import paper_1612_04787_amd as sw
    from datagen.workloads import section_pair_1024
    print("case 1024 generate", flush=True)
    a, b, m, bv, n_list, ia, ib, ta, tb = section_pair_1024(16384, dev())
    P, n = len(n_list), 1024
    print("case 1024 match P=%d" % P, flush=True)
    res = ctx.match_batch([a, b], n_list, ia, ib, ta, tb, sw.make_params(p=0.65))
    torch.cuda.synchronize()
    _check_all_records(res, n, P)
    # B(q) = A(M q + b) = A(q - d(q)) with d(q) = q - M q - b, so the peak of a
    # window centred at q is near +d(q) (the centroid is biased toward the integer)
    cen = ta[:, :2].cpu().numpy().astype(np.float64)
    d_true = cen - cen @ np.asarray(m, np.float64).T - np.asarray(bv, np.float64)
    got = np.stack([res["dx"].cpu().numpy(), res["dy"].cpu().numpy()], 1)
    err = np.abs(got - d_true).max(1)
    print("   |d - d_true|: median %.3f max %.3f px" % (np.median(err), err.max()), flush=True)
    assert np.median(err) <= 0.5 and err.max() <= 1.5
    rng = np.random.default_rng(7)
    for i in rng.choice(P, 4, replace=False):
        cx, cy = cen[i]
        x0, y0, x1, y1 = _crop(cx, cy, n, 16384, 16384)
        ca = a[y0:y1, x0:x1].cpu().numpy()
        cb = b[y0:y1, x0:x1].cpu().numpy()
        th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
        r = O.match_pair(ca, cb, th, th, n, O.Params(p=0.65))
        e = compare(gpu_record(res, int(i)), r, n, tag="1024 pair %d" % i)
        print("   pair %d:" % i, e, flush=True)


def test_headline_jacobian_4096_pairs_512(ctx):
    """The centroid Jacobian in the configuration the refinement benchmark
    times: 4096 windows of 512^2 on the 64-section stack, window B at a
    fractional translation t*, window A U(-0.5, 0.5)^2 px away, translation
    columns only (SWIFT_FLAG_JAC_TRANSLATION).  Sampled pairs against the FP64
    oracle; every pair finite with zeros outside the translation columns."""
    import paper_1612_04787_amd as sw
    from datagen.workloads import distorted_stack, section_grid_pairs
    S, size, n = 64, 4096, 512
    print("case headline jacobian generate", flush=True)
    stack, _ = distorted_stack(S, size, seed=5, device=dev())
    _, _, _, _, _, cen = section_grid_pairs(S, size, n, 8, dev())
    rng = np.random.default_rng(9)
    P = S * len(cen)
    tb = np.zeros((P, 8), np.float32)
    k = 0
    for s in range(S):
        for (cx, cy) in cen:
            tb[k] = [cx, cy, 1, 0, rng.uniform(-0.5, 0.5), 0, 1, rng.uniform(-0.5, 0.5)]
            k += 1
    ta = tb.copy()
    ta[:, 4] += rng.uniform(-0.5, 0.5, P).astype(np.float32)
    ta[:, 7] += rng.uniform(-0.5, 0.5, P).astype(np.float32)
    idx = torch.arange(S, dtype=torch.int32).repeat_interleave(len(cen))
    params = sw.make_params(p=0.65)
    print("case headline jacobian P=%d" % P, flush=True)
    res = ctx.match_batch([stack[s] for s in range(S)], [n] * P, idx, idx, torch.from_numpy(ta),
                          torch.from_numpy(tb), params, save=True)
    jac = ctx.centroid_jacobian(res, sw.make_params(p=0.65, flags=sw.FLAG_JAC_TRANSLATION))
    torch.cuda.synchronize()
    jac = jac.cpu().numpy()
    assert np.isfinite(jac).all()
    assert not jac[:, :, [0, 1, 3, 4]].any()
    for i in rng.choice(P, 3, replace=False):
        s = int(i) // len(cen)
        cx, cy = float(tb[i, 0]), float(tb[i, 1])
        x0, y0, x1, y1 = _crop(cx, cy, n, size, size, m=6)
        img = stack[s, y0:y1, x0:x1].cpu().numpy().astype(np.float64)
        tha, thb = ta[i].astype(np.float64), tb[i].astype(np.float64)
        tha[0] -= x0
        tha[1] -= y0
        thb[0] -= x0
        thb[1] -= y0
        rec, ref = O.centroid_jacobian(img, img, tha, thb, n, O.Params(p=0.65))
        assert (int(res["ix"][i]), int(res["iy"][i])) == (rec["ix"], rec["iy"])
        for row in range(2):
            g, r = jac[i, row, [2, 5]].astype(np.float64), ref[row][[2, 5]]
            err = np.linalg.norm(g - r) / np.linalg.norm(r)
            print("   pair %d d%s/dt rel err %.2e" % (i, "xy"[row], err), flush=True)
            assert err <= 1e-3, (i, row, g, r)


def test_config3_ragged_batch_sampled(ctx):
    """Config 3 at full size: a 32-section 8192^2 stack, 4 pyramid levels,
    +-3 projections per level, 8 x 8 windows per section and level: 8192
    pairs of 128/256/512/1024 in one ragged call (size groups concurrent).
    Three pairs per window edge against the oracle, which builds its own
    pyramid levels (2 x 2 box, from the raw stack bytes) and projections on
    crops aligned to the level's blocks."""
    import paper_1612_04787_amd as sw
    from datagen.workloads import level_stack, ragged_level_pairs
    from paper_1612_04787_amd.stack import build_pyramid
    S, size, levels, k = 32, 8192, 4, 3
    print("case config3 generate", flush=True)
    stack = level_stack(S, size, seed=3, device=dev())
    pyr = build_pyramid(ctx, stack, levels - 1)
    images = []
    refs = []
    for lv in pyr:
        ref = ctx.project(lv, k=k)
        refs.append(ref)
        images += [lv[s] for s in range(S)] + [ref[s] for s in range(S)]
    n_list, ia, ib, ta, tb = ragged_level_pairs(S, size, levels, 8, dev())
    P = len(n_list)
    print("case config3 match P=%d" % P, flush=True)
    res = ctx.match_batch(images, n_list, ia, ib, ta, tb, sw.make_params(p=0.65, flags=sw.FLAG_CONCURRENT_SIZES))
    torch.cuda.synchronize()
    ns = np.array(n_list)
    for n in (128, 256, 512, 1024):
        sel = torch.from_numpy(np.nonzero(ns == n)[0]).to(dev())
        _check_all_records({key: v[sel] for key, v in res.items() if torch.is_tensor(v) and v.dim() == 1}, n,
                           int(sel.numel()))
    tha = ta.cpu().numpy()
    iac = ia.cpu().numpy()
    rng = np.random.default_rng(33)
    for n in (128, 256, 512, 1024):
        lvl = {1024: 0, 512: 1, 256: 2, 128: 3}[n]
        side = size >> lvl
        for i in rng.choice(np.nonzero(ns == n)[0], 3, replace=False):
            s = int(iac[i]) - 2 * S * lvl
            cx, cy = float(tha[i, 0]), float(tha[i, 1])
            x0, y0, x1, y1 = _crop(cx, cy, n, side, side)
            f = 1 << lvl
            lo, hi = max(0, s - k), min(S, s + k + 1)
            sub = stack[lo:hi, y0 * f:y1 * f, x0 * f:x1 * f].cpu().numpy()
            lev = []
            for q in range(hi - lo):
                im = sub[q]
                for _ in range(lvl):
                    im = O.pyramid(im)
                lev.append(im)
            lev = np.stack(lev)
            got = pyr[lvl][s, y0:y1, x0:x1].cpu().numpy()
            assert np.array_equal(got, lev[s - lo]), ("pyramid", n, i)
            ref_o = O.project(lev, s - lo, k)
            assert np.array_equal(refs[lvl][s, y0:y1, x0:x1].cpu().numpy(), ref_o), ("projection", n, i)
            th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
            r = O.match_pair(lev[s - lo], ref_o, th, th, n, O.Params(p=0.65))
            e = compare(gpu_record(res, int(i)), r, n, tag="config3 n=%d pair %d" % (n, i))
            print("   n=%d pair %d (section %d):" % (n, i, s), e, flush=True)
