"""GPU parity of the Pearson-normalised correlation mode (SWIFT_FLAG_PEARSON:
the central n/2 template of window A against every placement inside window
B, FFT correlation plus the cumulative-area correction) against the FP64
oracle's direct per-placement Pearson coefficients."""
import numpy as np
import pytest
import torch

import oracle as O
from datagen import make_section_pair
from parity_util import SNR_RTOL, SUBPIX_TOL, TIE_REL, gpu_record

pytestmark = pytest.mark.gpu
GAMMA_TOL = 1e-4  # absolute, on coefficients in [-1, 1]


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def section_pair_small():
    a, b, m, bv = make_section_pair(1600, 1600, 31, 331, device="cpu", max_shift=6.0)
    return a, b


def _params(flags=0):
    import paper_1612_04787_amd as sw
    return sw.make_params(p=0.65, flags=sw.FLAG_PEARSON | flags)


def _windows(rng, k, n, size=1600):
    """Translation and mildly affine windows, B offset by up to n/4 + 2 (so a
    few true shifts lie beyond the placement range); one window partly
    outside the section."""
    tha = np.zeros((k, 8), np.float32)
    for i in range(k):
        e = rng.uniform(-2e-3, 2e-3, 4) if i % 2 else np.zeros(4)
        tha[i] = [rng.uniform(n / 2 + 8, size - n / 2 - 8), rng.uniform(n / 2 + 8, size - n / 2 - 8),
                  1 + e[0], e[1], rng.uniform(-0.5, 0.5), e[2], 1 + e[3], rng.uniform(-0.5, 0.5)]
    tha[-1, 0:2] = [n / 2 - 5.5, size - n / 2 + 3.25]
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-n / 4 - 2, n / 4 + 2, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-n / 4 - 2, n / 4 + 2, k).astype(np.float32)
    return tha, thb


def _compare(g, r, n, tag):
    if r["status"] & O.swift_oracle.STATUS_DEGENERATE:
        assert g["status"] & O.swift_oracle.STATUS_DEGENERATE and g["snr"] == 0.0, (tag, g)
        return
    margin = (r["peak"] - r["second"]) / max(abs(r["peak"]), 1e-30)
    assert abs(g["peak"] - r["peak"]) <= GAMMA_TOL, (tag, g["peak"], r["peak"])
    if margin > max(TIE_REL, 4 * GAMMA_TOL):
        assert (g["ix"], g["iy"]) == (r["ix"], r["iy"]), (tag, g, r["ix"], r["iy"], margin)
        assert abs(g["dx"] - r["dx"]) <= SUBPIX_TOL and abs(g["dy"] - r["dy"]) <= SUBPIX_TOL, (tag, g, r["dx"],
                                                                                             r["dy"])
    else:
        # several placements score within the tolerance: the GPU's must be one of them
        R = n // 4
        sx = g["ix"] - n if g["ix"] >= n // 2 else g["ix"]
        sy = g["iy"] - n if g["iy"] >= n // 2 else g["iy"]
        assert r["surface"][sy + R, sx + R] >= r["peak"] - 4 * GAMMA_TOL, (tag, g)
    assert abs(g["mean"] - r["mean"]) <= GAMMA_TOL, (tag, g["mean"], r["mean"])
    assert abs(g["std"] - r["std"]) <= SNR_RTOL * r["std"], (tag, g["std"], r["std"])
    assert abs(g["snr"] - r["snr"]) <= SNR_RTOL * abs(r["snr"]) + 1e-3, (tag, g["snr"], r["snr"])
    assert (g["status"] & O.swift_oracle.STATUS_CLAMPED) == (r["status"] & O.swift_oracle.STATUS_CLAMPED), tag


@pytest.mark.parametrize("n", [64, 128, 256])
def test_pearson_matches_oracle(ctx, section_pair_small, n):
    print("case pearson n=%d" % n, flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(9100 + n)
    k = {64: 8, 128: 5, 256: 3}[n]
    tha, thb = _windows(rng, k, n)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb), _params())
    torch.cuda.synchronize()
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.pearson_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, return_surface=True)
        g = gpu_record(res, i)
        _compare(g, r, n, "pearson n=%d i=%d" % (n, i))
        print("   ", i, g["peak"], r["peak"], g["snr"], r["snr"], flush=True)
    assert int(res["status"][k - 1]) & O.swift_oracle.STATUS_CLAMPED


@pytest.mark.parametrize("n", [512, 1024])
def test_pearson_large_windows_sampled(ctx, section_pair_small, n):
    """Large windows: B is A's own section moved by a known integer shift, so
    the best placement is that shift with a coefficient of 1; the oracle
    checks the coefficient of the GPU's placement and of its 3 x 3
    neighbours, one placement at a time."""
    print("case pearson large n=%d" % n, flush=True)
    a, _ = section_pair_small
    an = a.numpy()
    rng = np.random.default_rng(9200 + n)
    k = 2
    tha = np.zeros((k, 8), np.float32)
    thb = np.zeros((k, 8), np.float32)
    shifts = [(rng.integers(-n // 4, n // 4), rng.integers(-n // 4, n // 4)) for _ in range(k)]
    for i, (dx, dy) in enumerate(shifts):
        cx, cy = 800.0, 800.0
        tha[i] = [cx, cy, 1, 0, 0, 0, 1, 0]
        thb[i] = [cx - dx, cy - dy, 1, 0, 0, 0, 1, 0]
    res = ctx.match_batch([a.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32), torch.zeros(k, dtype=torch.int32),
                          torch.from_numpy(tha), torch.from_numpy(thb), _params())
    torch.cuda.synchronize()
    m, c0 = n // 2, n // 4
    for i, (dx, dy) in enumerate(shifts):
        g = gpu_record(res, i)
        sx = g["ix"] - n if g["ix"] >= n // 2 else g["ix"]
        sy = g["iy"] - n if g["iy"] >= n // 2 else g["iy"]
        assert (sx, sy) == (int(dx), int(dy)), (i, g, dx, dy)
        assert abs(g["peak"] - 1.0) <= GAMMA_TOL, g
        wa, _ = O.gather(an, tha[i].astype(np.float64), n)
        wb, _ = O.gather(an, thb[i].astype(np.float64), n)
        t = wa[c0:c0 + m, c0:c0 + m]
        for ddy in (-1, 0, 1):
            for ddx in (-1, 0, 1):
                if abs(sx + ddx) > n // 4 or abs(sy + ddy) > n // 4:
                    continue
                p = wb[c0 + sy + ddy:c0 + sy + ddy + m, c0 + sx + ddx:c0 + sx + ddx + m]
                ref = np.corrcoef(t.ravel(), p.ravel())[0, 1]
                assert ref <= g["peak"] + GAMMA_TOL
        assert abs(g["dx"] - dx) < 0.5 and abs(g["dy"] - dy) < 0.5


def test_pearson_512_records(ctx, section_pair_small):
    """The size the bench's Pearson block times: two 512^2 pairs of real
    section content (B a warped, noisy copy of A; one window with a small
    affine), full records (coefficient, SNR, mean, std, centroid) against
    the oracle's direct per-placement coefficients."""
    print("case pearson 512 records", flush=True)
    a, b = section_pair_small
    n, k = 512, 2
    tha = np.array([[800.0, 760.0, 1, 0, 0.25, 0, 1, -0.5],
                    [700.0, 850.0, 1 + 1e-3, -8e-4, -0.375, 6e-4, 1 - 5e-4, 0.125]], np.float32)
    thb = tha.copy()
    thb[:, 4] += np.array([37.0, -61.5], np.float32)
    thb[:, 7] += np.array([-22.0, 18.25], np.float32)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb), _params())
    torch.cuda.synchronize()
    an, bn = a.numpy(), b.numpy()
    for i in range(k):
        r = O.pearson_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n, return_surface=True)
        g = gpu_record(res, i)
        print("   ", i, g, r["peak"], r["snr"], r["dx"], r["dy"], flush=True)
        _compare(g, r, n, "pearson 512 i=%d" % i)
        assert r["snr"] > 5.0 and r["peak"] > 0.5


def test_pearson_degenerate_ragged_and_graph(ctx, section_pair_small):
    """A constant template is degenerate; one ragged call over 64..256 on
    the concurrent groups and as graph replays gives identical records."""
    import paper_1612_04787_amd as sw
    print("case pearson ragged", flush=True)
    a, b = section_pair_small
    flat = torch.full((400, 400), 77, dtype=torch.uint8)
    rng = np.random.default_rng(9300)
    ns, tha, thb = [], [], []
    for n in (64, 128, 256):
        ta, tb = _windows(rng, 2, n)
        ns += [n, n]
        tha.append(ta)
        thb.append(tb)
    tha, thb = np.concatenate(tha), np.concatenate(thb)
    k = len(ns)
    ia = torch.zeros(k, dtype=torch.int32)
    ia[0] = 2  # the constant image
    tha[0, 0:2] = [200, 200]
    args = ([a.to(dev()), b.to(dev()), flat.to(dev())], ns, ia, torch.ones(k, dtype=torch.int32),
            torch.from_numpy(tha), torch.from_numpy(thb))
    res = ctx.match_batch(*args, _params())
    res_c = ctx.match_batch(*args, _params(sw.FLAG_CONCURRENT_SIZES))
    torch.cuda.synchronize()
    assert int(res["status"][0]) & O.swift_oracle.STATUS_DEGENERATE and float(res["snr"][0]) == 0.0
    for key in ("dx", "dy", "ix", "iy", "snr", "peak", "status"):
        assert torch.equal(res[key], res_c[key]), key
    prep = ctx.prepare(*args)
    for rep in range(3):
        out = torch.empty((k, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
        ctx.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], _params(sw.FLAG_CONCURRENT_SIZES), out,
                            graph=True)
        torch.cuda.synchronize()
        rg = sw.parse_records(out)
        for key in ("dx", "dy", "ix", "iy", "snr", "peak", "status"):
            assert torch.equal(res[key], rg[key]), (rep, key)
    an, bn = a.numpy(), b.numpy()
    for i in range(1, k):
        r = O.pearson_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), ns[i], return_surface=True)
        _compare(gpu_record(res, i), r, ns[i], "pearson ragged i=%d" % i)


def test_pearson_validation(ctx, section_pair_small):
    import paper_1612_04787_amd as sw
    print("case pearson validation", flush=True)
    a, b = section_pair_small
    th = torch.tensor([[800, 800, 1, 0, 0, 0, 1, 0]], dtype=torch.float32)
    args = ([a.to(dev()), b.to(dev())], [128], torch.zeros(1, dtype=torch.int32), torch.ones(1, dtype=torch.int32),
            th, th.clone())
    with pytest.raises(sw.SwiftError):
        ctx.match_batch(*args, _params(), surfaces=True)
    with pytest.raises(sw.SwiftError):
        ctx.match_batch(*args, sw.make_params(flags=sw.FLAG_PEARSON, max_shift=8))
    with pytest.raises(sw.SwiftError):
        ctx.match_batch(*args, _params(), save=True)
