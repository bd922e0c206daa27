"""Stack loop on the GPU: mir rendering (bit-exact), swim window set-up and the
per-section affine fit against the oracle, and the whole coarse-to-fine loop
against the synthetic stack's known section warps."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def _affines(rng, S, shift=5.0, lin=0.01):
    a = np.zeros((S, 6))
    for s in range(S):
        e = rng.uniform(-lin, lin, 4)
        a[s] = [1 + e[0], e[1], rng.uniform(-shift, shift), e[2], 1 + e[3], rng.uniform(-shift, shift)]
    return a


@pytest.mark.parametrize("level", [0, 1, 2])
def test_render_bit_exact(ctx, level):
    print("case render level=%d" % level, flush=True)
    rng = np.random.default_rng(40 + level)
    S, h, w = 3, 90, 131
    src = rng.integers(0, 256, (S, h, w)).astype(np.uint8)
    aff = _affines(rng, S, shift=6.0 * (1 << level))
    aff[0] = [1, 0, 0, 0, 1, 0]
    out = ctx.render(torch.from_numpy(src).to(dev()), torch.from_numpy(aff).to(dev()), level, out_hw=(77, 140))
    out = out.cpu().numpy()
    for s in range(S):
        ref = O.render(src[s], aff[s], level, 77, 140)
        np.testing.assert_array_equal(out[s], ref, err_msg="section %d" % s)


def test_render_pitched_views(ctx):
    # a section-strided view with a row pitch wider than the width
    print("case render pitched", flush=True)
    rng = np.random.default_rng(7)
    big = rng.integers(0, 256, (2, 64, 100)).astype(np.uint8)
    src = torch.from_numpy(big).to(dev())[:, :, :80]
    aff = _affines(rng, 2)
    out = ctx.render(src, torch.from_numpy(aff).to(dev()), 0).cpu().numpy()
    for s in range(2):
        np.testing.assert_array_equal(out[s], O.render(big[s, :, :80], aff[s], 0, 64, 80))


def test_stack_windows_match_oracle(ctx):
    print("case stack windows", flush=True)
    rng = np.random.default_rng(9)
    S, level, grid, hl, wl = 4, 1, 4, 256, 320
    aff = _affines(rng, S, shift=9.0)
    ia, ib, ta, tb = ctx.stack_windows(torch.from_numpy(aff).to(dev()), level, grid, hl, wl, 3, 100)
    ta, tb = ta.cpu().numpy(), tb.cpu().numpy()
    assert ia.cpu().tolist() == [3 + s for s in range(S) for _ in range(grid * grid)]
    assert ib.cpu().tolist() == [100 + s for s in range(S) for _ in range(grid * grid)]
    for s in range(S):
        ra, rb = O.stack_windows(aff[s], level, 0, grid, hl, wl)
        sl = slice(s * grid * grid, (s + 1) * grid * grid)
        np.testing.assert_array_equal(ta[sl], ra.astype(np.float32))
        np.testing.assert_array_equal(tb[sl], rb.astype(np.float32))


def _records(P, rng, dxy, snr, status):
    rec = np.zeros((P, 64), np.uint8)
    f32 = rec.view(np.float32)
    i32 = rec.view(np.int32)
    f32[:, 0] = dxy[:, 0]
    f32[:, 1] = dxy[:, 1]
    f32[:, 5] = snr
    i32[:, 10] = status
    i32[:, 11] = 64
    return rec


def test_fit_sections_match_oracle(ctx):
    print("case fit sections", flush=True)
    rng = np.random.default_rng(12)
    S, level, grid = 5, 2, 8
    per = grid * grid
    true = _affines(rng, S, shift=20.0, lin=0.004)
    start = _affines(rng, S, shift=2.0, lin=0.001)
    _, _, ta, tb = ctx.stack_windows(torch.from_numpy(start).to(dev()), level, grid, 512, 512, 0, S)
    ta, tb = ta.cpu().numpy(), tb.cpu().numpy()
    P = S * per
    # shifts d that make each window's correspondence the true affine's, plus noise
    dxy = np.zeros((P, 2), np.float32)
    for i in range(P):
        s = i // per
        p, q0 = O.correspondence(ta[i], tb[i], 0.0, 0.0, level)
        qt = np.array(O.apply_affine(true[s], p[0], p[1]))
        dq = (np.array(q0) - qt) / float(1 << level) + rng.normal(0, 0.05, 2)
        L = np.array([[ta[i, 2], ta[i, 3]], [ta[i, 5], ta[i, 6]]], np.float64)
        dxy[i] = np.linalg.solve(L, dq)
    snr = rng.uniform(3, 40, P).astype(np.float32)
    status = np.where(rng.uniform(0, 1, P) < 0.1, O.swift_oracle.STATUS_DEGENERATE, 0).astype(np.int32)
    snr[per * 4:] = 1.0  # section 4: no weighted point, keeps its affine
    rec = _records(P, rng, dxy, snr, status)
    aff_d = torch.from_numpy(start.copy()).to(dev())
    st = ctx.fit_sections(torch.from_numpy(ta).to(dev()), torch.from_numpy(tb).to(dev()),
                          torch.from_numpy(rec).to(dev()), per, level, aff_d, min_snr=6.0)
    got, st = aff_d.cpu().numpy(), st.cpu().numpy()
    for s in range(S):
        pts, w = [], []
        for i in range(s * per, (s + 1) * per):
            p, q = O.correspondence(ta[i], tb[i], float(dxy[i, 0]), float(dxy[i, 1]), level)
            pts.append((p, q))
            w.append(O.match_weight(float(snr[i]), int(status[i]), 6.0))
        ref, rst = O.fit_section([a for a, _ in pts], [b for _, b in pts], w, start[s])
        assert st[s] == rst, s
        np.testing.assert_allclose(got[s][[0, 1, 3, 4]], ref[[0, 1, 3, 4]], rtol=0, atol=1e-10)
        np.testing.assert_allclose(got[s][[2, 5]], ref[[2, 5]], rtol=0, atol=1e-7)
        if rst == 0:
            assert np.abs(got[s] - true[s])[[2, 5]].max() < 0.5
    assert st[4] == 1 and np.array_equal(got[4], start[4])


@pytest.mark.parametrize("refine", ["adjoint", "plain"])
def test_align_stack_reduces_misalignment(ctx, refine):
    """16 sections of 1024^2 with random-walk drift (U(+-2)^2 px per section)
    and per-section rotation / scale / shear; two levels (64^2 windows at level
    1, 128^2 at level 0), 8 x 8 windows per section."""
    from datagen.evaluate import residuals
    from datagen.workloads import distorted_stack
    from paper_1612_04787_amd.stack import align_stack
    print("case align stack refine=%s" % refine, flush=True)
    S, size = 16, 1024
    raw, warps = distorted_stack(S, size, seed=31, device=dev())
    pts = np.array([(64 + 128 * i, 64 + 128 * j) for j in range(8) for i in range(8)], np.float64)
    ident = np.tile([1.0, 0, 0, 0, 1.0, 0], (S, 1))
    g0, n0 = residuals(ident, warps, pts)
    aff, rep = align_stack(ctx, raw, levels=(1, 0), ns=(64, 128), iters=(4, 2), refine=refine)
    g1, n1 = residuals(aff.cpu().numpy(), warps, pts)
    for r in rep:
        print("   ", r, flush=True)
    print("   residual px: global %.3f -> %.3f, neighbour %.3f -> %.3f" % (g0, g1, n0, n1), flush=True)
    assert n1 < 0.5 * n0
    assert rep[-1]["median_snr"] > rep[0]["median_snr"]
    assert rep[-1]["singular_sections"] == 0


def test_align_stack_search_finds_a_misplaced_section(ctx):
    """12 sections of 2048^2 with drift and section affines; section 6 is moved
    by a further (150, -110) px, 37.5 px at level 2: beyond what a 64^2 window
    captures there.  With the search in the first pass the loop aligns it;
    without, the section stays misplaced."""
    from datagen.evaluate import composed_points
    from datagen.synth import make_stack
    from datagen.workloads import stack_warps
    from paper_1612_04787_amd.stack import align_stack
    print("case align stack with search", flush=True)
    S, size, j = 12, 2048, 6
    warps = stack_warps(S, size, size, 41)
    m, b = warps[j]
    warps[j] = (m, b + np.array([150.0, -110.0]))
    raw = make_stack(S, size, size, 41, device=dev(), warps=warps)
    pts = np.array([(128 + 256 * i, 128 + 256 * k) for k in range(8) for i in range(8)], np.float64)

    def pair_res(a):
        c = composed_points(a.cpu().numpy(), warps, pts)
        return np.sqrt(np.mean(np.sum((c[1:] - c[:-1]) ** 2, 2), 1))

    kw = dict(levels=(2, 1, 0), ns=(64, 128, 256), iters=(2, 1, 1), ks=(3, 3, 3))
    aff_s, rep_s = align_stack(ctx, raw, search=dict(rings=2, accept=15.0), **kw)
    aff_n, rep_n = align_stack(ctx, raw, **kw)
    r_s, r_n = pair_res(aff_s), pair_res(aff_n)
    print("   search: %d matches; pair residuals with search max %.2f px, without: at the section %.1f / %.1f px"
          % (rep_s[0]["search_matches"], r_s.max(), r_n[j - 1], r_n[j]), flush=True)
    assert rep_s[0]["search_matches"] > 0 and rep_s[1]["search_matches"] == 0
    assert r_s.max() < 1.0
    assert min(r_n[j - 1], r_n[j]) > 20.0
