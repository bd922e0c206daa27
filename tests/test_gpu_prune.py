"""GPU parity of the pruned inverse (a search radius r on the integer peak;
only the surface rows near the origin are transformed back and the SNR
background comes from the spectrum by Parseval) against the FP64 oracle's
windowed peak search."""
import numpy as np
import pytest
import torch

import oracle as O
from datagen import make_section_pair
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


@pytest.fixture(scope="module")
def section_pair_small():
    a, b, m, bv = make_section_pair(1600, 1600, 31, 331, device="cpu", max_shift=6.0)
    return a, b


def _windows(rng, k, n, r, size=1600):
    """Translation and mildly affine windows whose B side is offset by up to
    1.5 r, so some true shifts lie inside the search window and some outside;
    one window partly outside the section."""
    tha = np.zeros((k, 8), np.float32)
    for i in range(k):
        e = rng.uniform(-2e-3, 2e-3, 4) if i % 2 else np.zeros(4)
        tha[i] = [rng.uniform(n / 2 + 8, size - n / 2 - 8), rng.uniform(n / 2 + 8, size - n / 2 - 8),
                  1 + e[0], e[1], rng.uniform(-0.5, 0.5), e[2], 1 + e[3], rng.uniform(-0.5, 0.5)]
    tha[-1, 0:2] = [n / 2 - 5.5, size - n / 2 + 3.25]
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-1.5 * r, 1.5 * r, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-1.5 * r, 1.5 * r, k).astype(np.float32)
    return tha, thb


def _check(res, a, b, tha, thb, n, p, r, tag):
    an, bn = a.numpy(), b.numpy()
    inside = 0
    for i in range(tha.shape[0]):
        ref = O.match_pair(an, bn, tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                           O.Params(p=p, max_shift=r), return_surface=True)
        g = gpu_record(res, i)
        # the integer peak lies within the search window
        assert abs(g["ix"] - n if g["ix"] >= n // 2 else g["ix"]) <= r, (tag, i, g)
        assert abs(g["iy"] - n if g["iy"] >= n // 2 else g["iy"]) <= r, (tag, i, g)
        assert g["mean"] == 0.0, (tag, i, g)
        e = compare(g, ref, n, None, "%s i=%d" % (tag, i))
        full = O.peak_stats(ref["surface"])
        inside += (full["ix"], full["iy"]) == (ref["ix"], ref["iy"])
        print("  ", i, e, flush=True)
    return inside


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("rfrac", [0, 8, 2])
def test_pruned_search_matches_oracle(ctx, section_pair_small, n, rfrac):
    """Search radii 3 (a few rows), n/8 and n/2 - 1 (every row block runs,
    the search window and the Parseval background still apply)."""
    r = {0: 3, 8: n // 8, 2: n // 2 - 1}[rfrac]
    print("case prune n=%d r=%d" % (n, r), flush=True)
    import paper_1612_04787_amd as sw
    a, b = section_pair_small
    rng = np.random.default_rng(7000 + n + r)
    k = {64: 8, 128: 6, 256: 5, 512: 4, 1024: 3}[n]
    tha, thb = _windows(rng, k, n, r)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb),
                          sw.make_params(p=0.65, max_shift=r))
    torch.cuda.synchronize()
    _check(res, a, b, tha, thb, n, 0.65, r, "prune n=%d r=%d" % (n, r))


@pytest.mark.parametrize("p", [0.0, 1.0])
def test_pruned_search_plain_and_phase_only(ctx, section_pair_small, p):
    import paper_1612_04787_amd as sw
    n, r = 256, 12
    print("case prune p=%g" % p, flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(7100 + int(p))
    k = 5
    tha, thb = _windows(rng, k, n, r)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(tha), torch.from_numpy(thb),
                          sw.make_params(p=p, max_shift=r))
    torch.cuda.synchronize()
    _check(res, a, b, tha, thb, n, p, r, "prune p=%g" % p)


def test_pruned_ragged_batch_and_graph(ctx, section_pair_small):
    """One ragged call over every window size with radius 5, on the concurrent
    size groups and as a graph replayed twice: records identical across the
    three, and each matching the oracle."""
    import paper_1612_04787_amd as sw
    print("case prune ragged", flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(7200)
    r = 5
    ns, tha, thb = [], [], []
    for n in SIZES:
        ta, tb = _windows(rng, 2, n, r)
        ns += [n, n]
        tha.append(ta)
        thb.append(tb)
    tha, thb = np.concatenate(tha), np.concatenate(thb)
    k = len(ns)
    args = ([a.to(dev()), b.to(dev())], ns, torch.zeros(k, dtype=torch.int32), torch.ones(k, dtype=torch.int32),
            torch.from_numpy(tha), torch.from_numpy(thb))
    res = ctx.match_batch(*args, sw.make_params(p=0.65, max_shift=r))
    res_c = ctx.match_batch(*args, sw.make_params(p=0.65, max_shift=r, flags=sw.FLAG_CONCURRENT_SIZES))
    torch.cuda.synchronize()
    for key in ("dx", "dy", "ix", "iy", "snr", "std", "status"):
        assert torch.equal(res[key], res_c[key]), key
    for i, n in enumerate(ns):
        ref = O.match_pair(a.numpy(), b.numpy(), tha[i].astype(np.float64), thb[i].astype(np.float64), n,
                           O.Params(p=0.65, max_shift=r), return_surface=True)
        compare(gpu_record(res, i), ref, n, None, "prune ragged i=%d n=%d" % (i, n))
    prep = ctx.prepare(*args)
    prm = sw.make_params(p=0.65, max_shift=r, flags=sw.FLAG_CONCURRENT_SIZES)
    for rep in range(3):
        out = torch.empty((k, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
        ctx.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], prm, out, graph=True)
        torch.cuda.synchronize()
        rg = sw.parse_records(out)
        for key in ("dx", "dy", "ix", "iy", "snr", "std", "status"):
            assert torch.equal(res[key], rg[key]), (rep, key)


def test_pruned_rejects_surfaces_and_negative_radius(ctx, section_pair_small):
    import paper_1612_04787_amd as sw
    print("case prune validation", flush=True)
    a, b = section_pair_small
    th = torch.tensor([[800, 800, 1, 0, 0, 0, 1, 0]], dtype=torch.float32)
    args = ([a.to(dev()), b.to(dev())], [256], torch.zeros(1, dtype=torch.int32), torch.ones(1, dtype=torch.int32),
            th, th.clone())
    with pytest.raises(sw.SwiftError):
        ctx.match_batch(*args, sw.make_params(max_shift=8), surfaces=True)
    with pytest.raises(sw.SwiftError):
        ctx.match_batch(*args, sw.make_params(max_shift=-1))
    # a radius of half the window or more searches the whole surface: surfaces allowed
    res = ctx.match_batch(*args, sw.make_params(max_shift=128), surfaces=True)
    full = ctx.match_batch(*args, sw.make_params())
    torch.cuda.synchronize()
    for key in ("dx", "dy", "ix", "iy", "snr", "std"):
        assert torch.equal(res[key], full[key]), key


def test_pruned_forward_feeds_the_adjoint(ctx, section_pair_small):
    """The adjoint reads the saved forward spectra and records, not the
    surface rows: after a pruned forward whose shifts all lie inside the
    radius, the centroid Jacobian and the SNR gradient equal those after the
    full forward (to rounding of the background statistics)."""
    import paper_1612_04787_amd as sw
    print("case prune adjoint", flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(7300)
    n, k, r = 256, 4, 16
    tha = np.zeros((k, 8), np.float32)
    for i in range(k):
        tha[i] = [rng.uniform(300, 1300), rng.uniform(300, 1300), 1, 0, rng.uniform(-0.5, 0.5), 0, 1,
                  rng.uniform(-0.5, 0.5)]
    thb = tha.copy()
    thb[:, 4] += rng.uniform(-3, 3, k).astype(np.float32)
    thb[:, 7] += rng.uniform(-3, 3, k).astype(np.float32)
    args = ([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32), torch.ones(k, dtype=torch.int32),
            torch.from_numpy(tha), torch.from_numpy(thb))
    pf, pp = sw.make_params(p=0.65), sw.make_params(p=0.65, max_shift=r)
    full = ctx.match_batch(*args, pf, save=True)
    prun = ctx.match_batch(*args, pp, save=True)
    jf = ctx.centroid_jacobian(full, pf)
    jp = ctx.centroid_jacobian(prun, pp)
    gf, _ = ctx.match_backward(full, pf, g_snr=torch.ones(k))
    gp, _ = ctx.match_backward(prun, pp, g_snr=torch.ones(k))
    torch.cuda.synchronize()
    assert torch.equal(full["ix"], prun["ix"]) and torch.equal(full["iy"], prun["iy"])
    scale = jf.abs().max().item()
    assert (jf - jp).abs().max().item() <= 1e-4 * scale
    assert (gf - gp).abs().max().item() <= 1e-3 * gf.abs().max().item()


def test_pruned_and_pearson_with_alternative_row_plans(ctx, section_pair_small):
    """The pruned row blocks follow the inverse pass's row count: with the
    alternative row-count variants the pruned and Pearson records agree with
    the default plan's (same peaks; sums in another order)."""
    import paper_1612_04787_amd as sw
    print("case prune / pearson plans", flush=True)
    a, b = section_pair_small
    rng = np.random.default_rng(7400)
    ns, tha, thb = [], [], []
    for n in (128, 256, 512):
        ta, tb = _windows(rng, 2, n, 8)
        ns += [n, n]
        tha.append(ta)
        thb.append(tb)
    tha, thb = np.concatenate(tha), np.concatenate(thb)
    k = len(ns)
    args = ([a.to(dev()), b.to(dev())], ns, torch.zeros(k, dtype=torch.int32), torch.ones(k, dtype=torch.int32),
            torch.from_numpy(tha), torch.from_numpy(thb))
    prms = [sw.make_params(p=0.65, max_shift=8), sw.make_params(flags=sw.FLAG_PEARSON)]
    ref = [ctx.match_batch(*args, pr) for pr in prms]
    saved = {n: ctx.plan(n) for n in (128, 256, 512)}
    try:
        for n in (128, 256, 512):
            ctx.plan(n, 1, 1)
        alt = [ctx.match_batch(*args, pr) for pr in prms]
        torch.cuda.synchronize()
    finally:
        for n in (128, 256, 512):
            ctx.plan(n, 0, 0)
    for r0, r1 in zip(ref, alt):
        assert torch.equal(r0["ix"], r1["ix"]) and torch.equal(r0["iy"], r1["iy"])
        assert float((r0["dx"] - r1["dx"]).abs().max()) <= 1e-4
        assert float((r0["dy"] - r1["dy"]).abs().max()) <= 1e-4
        assert float(((r0["snr"] - r1["snr"]) / r0["snr"]).abs().max()) <= 1e-4
    assert saved[512] == ctx.plan(512)
