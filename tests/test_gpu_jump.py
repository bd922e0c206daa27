"""Jump repair on the GPU (Section III, model paragraphs): one-sided models
bit-exact against the oracle, the span blend and the break join against the
oracle's FP64 formulas, and the whole repair on a stack with a magnification
change against the generator's known section warps."""
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


@pytest.mark.parametrize("k", [1, 2, 3, 8])
@pytest.mark.parametrize("w", [48, 45])
def test_project_side_bit_exact(ctx, k, w):
    print("case project_side k=%d w=%d" % (k, w), flush=True)
    rng = np.random.default_rng(70 + k + w)
    st = rng.integers(0, 256, (11, 21, w)).astype(np.uint8)
    excl = np.zeros(11, np.uint8)
    excl[[2, 7]] = 1
    t = torch.from_numpy(st).to(dev())
    for side in (-1, 1):
        for ex in (None, excl):
            got = ctx.project_side(t, k, side, exclude=None if ex is None else torch.from_numpy(ex)).cpu().numpy()
            for s in range(11):
                ref = O.project_side(st, s, k, side, None if ex is None else ex.astype(bool))
                np.testing.assert_array_equal(got[s], ref, err_msg="side %d section %d" % (side, s))


def test_blend_and_join_match_oracle(ctx):
    print("case blend / join", flush=True)
    rng = np.random.default_rng(71)
    S = 9
    base = np.array([[1 + rng.uniform(-1e-3, 1e-3), rng.uniform(-1e-3, 1e-3), rng.uniform(-9, 9),
                      rng.uniform(-1e-3, 1e-3), 1 + rng.uniform(-1e-3, 1e-3), rng.uniform(-9, 9)] for _ in range(S)])
    L = base + rng.uniform(-0.5, 0.5, (S, 6)) * [1e-3, 1e-3, 2, 1e-3, 1e-3, 2]
    R = base + rng.uniform(-0.5, 0.5, (S, 6)) * [1e-3, 1e-3, 2, 1e-3, 1e-3, 2]
    aff = torch.from_numpy(base.copy()).to(dev())
    ctx.blend_span(3, 5, torch.from_numpy(L).to(dev()), torch.from_numpy(R).to(dev()), aff)
    got = aff.cpu().numpy()
    np.testing.assert_array_equal(got[:3], base[:3])
    np.testing.assert_array_equal(got[6:], base[6:])
    np.testing.assert_allclose(got[3:6], O.blend_span(L, R, 3, 5), rtol=0, atol=1e-12)
    Lj = base.copy()
    Lj[4] = [1.02, 0.001, -30.0, -0.002, 1.019, 42.0]
    out = ctx.join_break(4, torch.from_numpy(base).to(dev()), torch.from_numpy(Lj).to(dev())).cpu().numpy()
    np.testing.assert_allclose(out, O.join_break(base, Lj, 4), rtol=0, atol=1e-9)


def test_repair_joins_a_magnification_break(ctx):
    """10 sections of 2048^2 with drift, section affines and a 3% magnification
    change at section 5: the section-affine loop leaves a break between
    sections 4 and 5; the repair finds it and joins the two sides."""
    from datagen.evaluate import composed_points
    from datagen.workloads import jump_stack
    from paper_1612_04787_amd.stack import align_stack, repair_jumps
    print("case repair 10 x 2048^2", flush=True)
    S, size, j0 = 10, 2048, 5
    stack, warps = jump_stack(S, size, seed=17, j0=j0, mag=0.03, device=dev())
    aff, _ = align_stack(ctx, stack, levels=(1, 0), ns=(128, 256), iters=(2, 1), ks=(4, 3), grid=8)
    pts = np.array([(size // 16 + size // 8 * i, size // 16 + size // 8 * j) for j in range(8) for i in range(8)],
                   np.float64)

    def pair_res(a):
        c = composed_points(a.cpu().numpy(), warps, pts)
        return np.sqrt(np.mean(np.sum((c[1:] - c[:-1]) ** 2, 2), 1))

    r0 = pair_res(aff)
    aff2, rep = repair_jumps(ctx, stack, aff.clone(), level=0, n=256, grid=8, k=3)
    r1 = pair_res(aff2)
    print("pair residuals before", np.round(r0, 2), "after", np.round(r1, 2), rep["breaks"], rep["spans"], flush=True)
    _check_host_logic(rep)
    assert r0[j0 - 1] > 5.0  # the loop left a break
    assert [b["section"] for b in rep["breaks"]] == [j0]
    assert r1.max() < 0.25 * r0.max()


def test_repair_leaves_a_smooth_stack_alone(ctx):
    """The same stack without the magnification change: no break, no failed
    span, affines unchanged."""
    from datagen.workloads import jump_stack
    from paper_1612_04787_amd.stack import align_stack, repair_jumps
    print("case repair without a jump", flush=True)
    S, size = 10, 2048
    stack, _ = jump_stack(S, size, seed=17, j0=S, mag=0.03, device=dev())  # j0 = S: no section changes
    aff, _ = align_stack(ctx, stack, levels=(1, 0), ns=(128, 256), iters=(2, 1), ks=(4, 3), grid=8)
    before = aff.clone()
    aff2, rep = repair_jumps(ctx, stack, aff, level=0, n=256, grid=8, k=3)
    torch.cuda.synchronize()
    print("breaks", rep["breaks"], "spans", rep["spans"], flush=True)
    _check_host_logic(rep)
    assert rep["breaks"] == [] and rep["spans"] == []
    assert torch.equal(aff2, before)


def _check_host_logic(rep, frac=0.75):
    """The repair's host decisions against the oracle's FP64 definitions:
    every round's break scores, and the failed spans of the section SNRs."""
    for rd in rep["rounds"]:
        for s in range(len(rd["scores"])):
            ref = O.break_score(rd["aff"][s], rd["fit"][s], rep["centres"][s])
            assert abs(rd["scores"][s] - ref) <= 1e-9 * max(ref, 1.0), (s, rd["scores"][s], ref)
    assert rep["spans"] == O.failed_spans(rep["section_snr"], frac)


def test_repair_blends_a_failed_span(ctx):
    """10 sections of 2048^2 (drift, section affines, no jump) with sections
    4 and 5 buried in noise (sigma 70): their match SNR against the two-sided
    model falls below 0.75 of the stack median, so they form a failed span.
    Each is fitted against the one-sided models on either side (both
    omitting the span) and the span gets the Bezier blend of the two fits,
    checked against the oracle's blend of the same fits; the other sections
    keep their affines.  The break scores and the span test are checked
    against the oracle's definitions."""
    from datagen.workloads import jump_stack
    from paper_1612_04787_amd.stack import align_stack, repair_jumps
    print("case repair failed span 10 x 2048^2", flush=True)
    S, size = 10, 2048
    stack, _ = jump_stack(S, size, seed=19, j0=S, mag=0.0, device=dev())
    g = torch.Generator(device=dev()).manual_seed(77)
    for s in (4, 5):
        noisy = stack[s].float() + 70.0 * torch.randn(stack[s].shape, generator=g, device=dev())
        stack[s] = noisy.round().clamp(0, 255).to(torch.uint8)
    aff, _ = align_stack(ctx, stack, levels=(1, 0), ns=(128, 256), iters=(2, 1), ks=(4, 3), grid=8)
    before = aff.clone().cpu().numpy()
    aff2, rep = repair_jumps(ctx, stack, aff.clone(), level=0, n=256, grid=8, k=3)
    torch.cuda.synchronize()
    print("breaks", rep["breaks"], "spans", rep["spans"], "section snr", np.round(rep["section_snr"], 1), flush=True)
    _check_host_logic(rep)
    assert rep["breaks"] == []
    assert (4, 5) in rep["spans"]
    got = aff2.cpu().numpy()
    span_rows = {s for (a, b) in rep["spans"] for s in range(a, b + 1)}
    for s in range(S):
        if s not in span_rows:
            np.testing.assert_array_equal(got[s], before[s])
    for (a, b) in rep["spans"]:
        ref = O.blend_span(rep["side_fits"][-1], rep["side_fits"][1], a, b)
        np.testing.assert_allclose(got[a:b + 1], ref, rtol=0, atol=1e-9)


def test_jump_entry_points_reject_bad_arguments(ctx):
    import paper_1612_04787_amd as sw
    print("case jump validation", flush=True)
    lib = ctx.lib
    p = lambda t: sw.swift._ptr(t)  # noqa: E731
    st = torch.zeros((4, 8, 16), dtype=torch.uint8, device=dev())
    out = torch.empty_like(st)
    assert lib.swift_project_side(ctx.h, p(st), 4, 8, 16, 16, 128, None, 3, 0, p(out), 16, 128, ctx.stream()) == -1
    assert b"side" in lib.swift_last_error()
    assert lib.swift_project_side(ctx.h, p(st), 4, 8, 16, 16, 128, None, 9, 1, p(out), 16, 128, ctx.stream()) == -1
    aff = torch.zeros((4, 6), dtype=torch.float64, device=dev())
    other = torch.zeros_like(aff)
    assert lib.swift_blend_span(ctx.h, 4, 2, 4, p(aff), p(other), p(aff), ctx.stream()) == -1
    assert lib.swift_blend_span(ctx.h, 4, 3, 2, p(aff), p(other), p(aff), ctx.stream()) == -1
    assert lib.swift_join_break(ctx.h, 4, 1, p(aff), p(other), p(aff), ctx.stream()) == -1
    assert b"alias" in lib.swift_last_error()
    assert lib.swift_join_break(ctx.h, 4, 4, p(aff), p(other), p(other), ctx.stream()) == -1
