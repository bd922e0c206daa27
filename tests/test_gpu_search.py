"""Search with an SNR stop on the GPU (Section III, SNR paragraph): the driver's
kept candidate, kept record and per-candidate batch sizes against an
exhaustive search over the same candidates reduced by the oracle's selection
rule; the kept records against the oracle's matches; the found offsets against
the generator's known warp; swift_search_keep's rules on hand-made records."""
import numpy as np
import pytest
import torch

import oracle as O
from datagen.workloads import search_pair
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


@pytest.fixture(scope="module")
def case():
    a, b, m, bv, nl, ia, ib, ta, tb, cen = search_pair(2048, 128, 6, device=dev(), shift=(115.0, -75.0))
    return dict(a=a, b=b, m=m, bv=bv, nl=nl, ia=ia, ib=ib, ta=ta, tb=tb, cen=cen)


def _shifted(ta, o):
    t = ta.clone()
    t[:, 4] += float(o[0])
    t[:, 7] += float(o[1])
    return t


def _exhaustive(ctx, c, params, offsets):
    """[K, P, 64] records of every window at every candidate."""
    out = []
    for k in range(offsets.shape[0]):
        r = ctx.match_batch([c["a"], c["b"]], c["nl"], c["ia"], c["ib"], _shifted(c["ta"], offsets[k]), c["tb"],
                            params)
        out.append(r["raw"].clone())
    return torch.stack(out)


@pytest.mark.parametrize("accept,radius,ahead", [(15.0, 0, 1), (30.0, 0, 1), (0.0, 0, 1), (float("inf"), 0, 1),
                                                (15.0, 36, 1), (15.0, 36, 2), (15.0, 0, 3), (30.0, 0, 4)])
def test_search_matches_exhaustive_selection(ctx, case, accept, radius, ahead):
    import paper_1612_04787_amd as sw
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    print("case search accept=%g radius=%d lookahead=%d" % (accept, radius, ahead), flush=True)
    params = sw.make_params(p=0.65, max_shift=radius)
    offs = spiral_offsets(64.0, 2)
    K = offs.shape[0]
    full = _exhaustive(ctx, case, params, offs)
    snr = full.view(torch.float32).view(K, -1, 16)[:, :, 5].cpu().numpy()
    got = search_offsets(ctx, [case["a"], case["b"]], case["nl"], case["ia"], case["ib"], case["ta"], case["tb"],
                         params, offs, accept=accept, lookahead=ahead)
    torch.cuda.synchronize()
    cand = got["cand"].cpu().numpy()
    done = got["done"].cpu().numpy()
    best = got["best"].cpu()
    P = snr.shape[1]
    counts = np.zeros(P, np.int64)
    for w in range(P):
        arg, cnt = O.search_select(snr[:, w].tolist(), accept)
        counts[w] = cnt
        assert cand[w] == arg, (w, cand[w], arg, snr[:, w])
        assert done[w] == (1 if snr[arg, w] >= accept else 0), (w, done[w])
        # the kept record is the one the whole batch produced at that candidate
        assert torch.equal(best[w], full[arg, w].cpu()), w
    # a round starting at candidate k matches every window still searching
    # there at the next `ahead` candidates
    want, k = [], 0
    while k < K:
        n = int((counts > k).sum())
        if n == 0:
            want += [0] * (K - k)
            break
        b = min(ahead, K - k)
        want += [n] * b
        k += b
    assert got["matched"] == want, (got["matched"], want)
    print("   matched per candidate:", got["matched"], "of", P * K, flush=True)


def test_search_records_and_offsets(ctx, case):
    import paper_1612_04787_amd as sw
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    print("case search records vs oracle", flush=True)
    params = sw.make_params(p=0.65)
    offs = spiral_offsets(64.0, 2)
    got = search_offsets(ctx, [case["a"], case["b"]], case["nl"], case["ia"], case["ib"], case["ta"], case["tb"],
                         params, offs, accept=15.0)
    torch.cuda.synchronize()
    rec = sw.parse_records(got["best"])
    cand = got["cand"].cpu().numpy()
    done = got["done"].cpu().numpy().astype(bool)
    assert done.mean() > 0.9, done.mean()
    # the offset found, candidate minus the kept sub-pixel shift, is the
    # generator's displacement at the window centre to the accuracy of one
    # match (its centroid underestimates the shift; the window is rotated
    # 1 degree against its model) ...
    cen, m, bv = case["cen"], case["m"], case["bv"]
    truth = cen @ m.T + bv - cen
    o = offs.numpy().astype(np.float64)[cand]
    est = o - np.stack([rec["dx"].cpu().numpy(), rec["dy"].cpu().numpy()], 1)
    err = np.abs(est - truth).max(1)
    assert err[done].max() < 1.5, err[done]
    # ... and refinement from there, with window A given the section's linear
    # part (without it the content-weighted centre of a rotated window biases
    # the translation), reaches the displacement
    from paper_1612_04787_amd.refine import refine_adjoint
    t0 = case["ta"].clone()
    t0[:, 2], t0[:, 3], t0[:, 5], t0[:, 6] = float(m[0, 0]), float(m[0, 1]), float(m[1, 0]), float(m[1, 1])
    t0[:, 4] = torch.from_numpy(est[:, 0].astype(np.float32)).to(dev())
    t0[:, 7] = torch.from_numpy(est[:, 1].astype(np.float32)).to(dev())
    th, it, _ = refine_adjoint(ctx, [case["a"], case["b"]], case["nl"], case["ia"], case["ib"], t0, case["tb"],
                               params, tol=0.005)
    fin = th[:, [4, 7]].cpu().numpy().astype(np.float64)
    ferr = np.abs(fin - truth).max(1)
    print("   search err max %.3f px, after %d refinement steps %.3f px" % (err[done].max(), it, ferr[done].max()),
          flush=True)
    assert ferr[done].max() < 0.1, ferr[done]
    # the kept records against the oracle at their candidate
    an, bn = case["a"].cpu().numpy(), case["b"].cpu().numpy()
    ta = case["ta"].cpu().numpy().astype(np.float64)
    for w in (0, 14, 35):
        th = ta[w].copy()
        th[4] += o[w, 0]
        th[7] += o[w, 1]
        r = O.match_pair(an, bn, th, ta[w], 128, O.Params(p=0.65))
        e = compare(gpu_record(rec, w), r, 128, tag="search window %d" % w)
        print("   window %d cand %d err %.3f px:" % (w, cand[w], err[w]), e, flush=True)


@pytest.mark.parametrize("radius", [0, 36])
def test_search_oracle_selection(ctx, case, radius):
    # the oracle's own SNRs over the whole candidate list pick the same
    # candidate (unless an SNR lies within rounding of the threshold)
    import paper_1612_04787_amd as sw
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    print("case search oracle selection radius=%d" % radius, flush=True)
    params = sw.make_params(p=0.65, max_shift=radius)
    offs = spiral_offsets(64.0, 2)
    got = search_offsets(ctx, [case["a"], case["b"]], case["nl"], case["ia"], case["ib"], case["ta"], case["tb"],
                         params, offs, accept=15.0)
    cand = got["cand"].cpu().numpy()
    an, bn = case["a"].cpu().numpy(), case["b"].cpu().numpy()
    ta = case["ta"].cpu().numpy().astype(np.float64)
    for w in (7, 28):
        snrs = []
        for k in range(offs.shape[0]):
            th = ta[w].copy()
            th[4] += float(offs[k, 0])
            th[7] += float(offs[k, 1])
            snrs.append(O.match_pair(an, bn, th, ta[w], 128, O.Params(p=0.65, max_shift=radius))["snr"])
        arg, cnt = O.search_select(snrs, 15.0)
        near = [v for v in snrs[:cnt] if abs(v - 15.0) <= 1e-3 * 15.0]
        srt = sorted(snrs[:cnt])
        tie = len(srt) > 1 and srt[-1] - srt[-2] <= 1e-3 * srt[-1]
        print("   window %d: oracle cand %d after %d, gpu %d" % (w, arg, cnt, cand[w]), flush=True)
        if not near and not tie:
            assert cand[w] == arg, (w, cand[w], arg, snrs)


def _records(snrs):
    r = torch.zeros((len(snrs), 64), dtype=torch.uint8)
    r.view(torch.float32).view(len(snrs), 16)[:, 5] = torch.tensor(snrs, dtype=torch.float32)
    r.view(torch.float32).view(len(snrs), 16)[:, 0] = torch.arange(len(snrs), dtype=torch.float32)
    return r.to(dev())


def test_search_keep_rules(ctx):
    import paper_1612_04787_amd as sw
    print("case search_keep rules", flush=True)
    P = 4
    best = torch.zeros((P, 64), dtype=torch.uint8, device=dev())
    cand = torch.full((P,), -1, dtype=torch.int32, device=dev())
    done = torch.zeros(P, dtype=torch.uint8, device=dev())
    # entries outside [0, P) are ignored
    idx = torch.tensor([-1, 0, P, 2], dtype=torch.int32, device=dev())
    ctx.search_keep(P, idx, _records([99.0, 12.0, 99.0, 5.0]), 0, 10.0, best, cand, done)
    torch.cuda.synchronize()
    assert cand.tolist() == [0, -1, 0, -1]
    assert done.tolist() == [1, 0, 0, 0]
    # an equal SNR keeps the earlier candidate; a higher one replaces it
    ctx.search_keep(P, torch.tensor([2], dtype=torch.int32, device=dev()), _records([5.0]), 1, 10.0, best, cand,
                    done)
    ctx.search_keep(P, torch.tensor([2, 3], dtype=torch.int32, device=dev()), _records([11.0, 0.0]), 2, 10.0,
                    best, cand, done)
    torch.cuda.synchronize()
    assert cand.tolist() == [0, -1, 2, 2]
    assert done.tolist() == [1, 0, 1, 0]
    snr = best.view(torch.float32).view(P, 16)[:, 5].tolist()
    assert snr == [12.0, 0.0, 11.0, 0.0]
    # a window already done is left alone, even by a better match
    ctx.search_keep(P, torch.tensor([0, 2], dtype=torch.int32, device=dev()), _records([50.0, 60.0]), 3, 10.0, best,
                    cand, done)
    torch.cuda.synchronize()
    assert cand.tolist() == [0, -1, 2, 2]
    assert best.view(torch.float32).view(P, 16)[:, 5].tolist() == [12.0, 0.0, 11.0, 0.0]
    # n = 0 launches nothing
    e = torch.zeros(0, dtype=torch.int32, device=dev())
    ctx.search_keep(P, e, torch.zeros((0, 64), dtype=torch.uint8, device=dev()), 4, 10.0, best, cand, done)
    # n above P and a negative candidate are rejected
    with pytest.raises(sw.SwiftError):
        ctx.search_keep(2, idx[:3], _records([1.0, 2.0, 3.0]), 0, 10.0, best[:2], cand[:2], done[:2])
    with pytest.raises(sw.SwiftError):
        ctx.search_keep(P, idx, _records([1.0, 2.0, 3.0, 4.0]), -1, 10.0, best, cand, done)
    torch.cuda.synchronize()
    assert cand.tolist() == [0, -1, 2, 2]


@pytest.mark.parametrize("P", [1, 100, 1024, 2500])
def test_search_next_gathers_in_order(ctx, P):
    import paper_1612_04787_amd as sw
    print("case search_next P=%d" % P, flush=True)
    g = torch.Generator().manual_seed(P)
    done = (torch.rand(P, generator=g) < 0.4).to(torch.uint8)
    ia = torch.randint(0, 9, (P,), generator=g, dtype=torch.int32)
    ib = torch.randint(0, 9, (P,), generator=g, dtype=torch.int32)
    ta = torch.randn((P, 8), generator=g) * 100
    tb = torch.randn((P, 8), generator=g) * 100
    d = [t.to(dev()) for t in (done, ia, ib, ta, tb)]
    outs = [torch.full((P,), -7, dtype=torch.int32, device=dev()) for _ in range(3)]
    touts = [torch.full((P, 8), -7.0, device=dev()) for _ in range(2)]
    count = torch.zeros(1, dtype=torch.int32, device=dev())
    ctx.search_next(d[0], 64.0, -32.5, d[1], d[2], d[3], d[4], outs[0], outs[1], outs[2], touts[0], touts[1], count)
    torch.cuda.synchronize()
    keep = torch.nonzero(done == 0).flatten()
    n = int(count.item())
    assert n == keep.numel()
    assert torch.equal(outs[0][:n].cpu(), keep.to(torch.int32))
    assert torch.equal(outs[1][:n].cpu(), ia[keep]) and torch.equal(outs[2][:n].cpu(), ib[keep])
    want = ta[keep].clone()
    want[:, 4] += 64.0
    want[:, 7] += -32.5
    assert torch.equal(touts[0][:n].cpu(), want) and torch.equal(touts[1][:n].cpu(), tb[keep])
    # nothing past the count is written
    assert bool((outs[0][n:] == -7).all()) and bool((touts[0][n:] == -7.0).all())
    # every window done: nothing gathered; no windows at all: count 0
    ctx.search_next(torch.ones(P, dtype=torch.uint8, device=dev()), 0.0, 0.0, d[1], d[2], d[3], d[4], outs[0],
                    outs[1], outs[2], touts[0], touts[1], count)
    torch.cuda.synchronize()
    assert int(count.item()) == 0
    e = torch.zeros(0, dtype=torch.int32, device=dev())
    count.fill_(5)
    ctx.search_next(torch.zeros(0, dtype=torch.uint8, device=dev()), 0.0, 0.0, e, e, torch.zeros((0, 8), device=dev()),
                    torch.zeros((0, 8), device=dev()), e, e, e, torch.zeros((0, 8), device=dev()),
                    torch.zeros((0, 8), device=dev()), count)
    torch.cuda.synchronize()
    assert int(count.item()) == 0
    # outputs aliasing the inputs are rejected
    with pytest.raises(sw.SwiftError):
        ctx.search_next(d[0], 0.0, 0.0, d[1], d[2], d[3], d[4], outs[0], outs[1], outs[2], d[3], touts[1], count)


def test_search_mixed_window_sizes(ctx, case):
    # a batch of two window edges stays sorted through every round; the
    # selection still matches the exhaustive search
    import paper_1612_04787_amd as sw
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    print("case search mixed sizes", flush=True)
    params = sw.make_params(p=0.65)
    offs = spiral_offsets(64.0, 1)
    K = offs.shape[0]
    c = dict(case)
    c["nl"] = [64] * 18 + [128] * 18
    full = _exhaustive(ctx, c, params, offs)
    snr = full.view(torch.float32).view(K, -1, 16)[:, :, 5].cpu().numpy()
    got = search_offsets(ctx, [c["a"], c["b"]], c["nl"], c["ia"], c["ib"], c["ta"], c["tb"], params, offs, accept=15.0)
    torch.cuda.synchronize()
    cand = got["cand"].cpu().numpy()
    best = got["best"].cpu()
    counts = []
    for w in range(36):
        arg, cnt = O.search_select(snr[:, w].tolist(), 15.0)
        counts.append(cnt)
        assert cand[w] == arg, (w, cand[w], arg)
        assert torch.equal(best[w], full[arg, w].cpu()), w
    assert got["matched"] == [sum(1 for x in counts if x > k) for k in range(K)]
    assert int(sw.parse_records(got["best"])["n"].cpu()[0]) == 64
    print("   matched per candidate:", got["matched"], flush=True)


def test_search_bench_size_sampled(ctx):
    # the benchmark's search: 576 windows of 256^2 on an 8192^2 pair, 25
    # candidates 128 px apart, radius 68, stop at 15; the selection against the
    # exhaustive search, sampled records against the oracle
    import paper_1612_04787_amd as sw
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    print("case search bench size", flush=True)
    a, b, m, bv, nl, ia, ib, ta, tb, cen = search_pair(8192, 256, 24, device=dev())
    params = sw.make_params(p=0.65, max_shift=68)
    offs = spiral_offsets(128.0, 2)
    K, P = offs.shape[0], len(nl)
    full = []
    for k in range(K):
        r = ctx.match_batch([a, b], nl, ia, ib, _shifted(ta, offs[k]), tb, params)
        full.append(r["raw"].clone())
    full = torch.stack(full)
    snr = full.view(torch.float32).view(K, -1, 16)[:, :, 5].cpu().numpy()
    got = search_offsets(ctx, [a, b], nl, ia, ib, ta, tb, params, offs, accept=15.0)
    torch.cuda.synchronize()
    cand = got["cand"].cpu().numpy()
    best = got["best"].cpu()
    for w in range(P):
        arg, _ = O.search_select(snr[:, w].tolist(), 15.0)
        assert cand[w] == arg, (w, cand[w], arg)
        assert torch.equal(best[w], full[arg, w].cpu()), w
    assert bool(got["done"].all())
    rec = sw.parse_records(got["best"])
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    tn = ta.cpu().numpy().astype(np.float64)
    o = offs.numpy().astype(np.float64)
    for w in (0, 287, 575):
        th = tn[w].copy()
        th[4] += o[cand[w], 0]
        th[7] += o[cand[w], 1]
        r = O.match_pair(an, bn, th, tn[w], 256, O.Params(p=0.65, max_shift=68))
        e = compare(gpu_record(rec, w), r, 256, tag="bench-size search window %d" % w)
        print("   window %d cand %d:" % (w, cand[w]), e, flush=True)
