"""Row-count variants of the match kernels: every variant of every window
size matches the FP64 oracle; the autotuner times them and keeps one."""
import numpy as np
import pytest
import torch

import oracle as O
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
def pair():
    from datagen import make_section_pair
    a, b, _, _ = make_section_pair(1500, 1500, 71, 771, device="cpu", max_shift=5.0)
    return a, b


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("variant", [(0, 1), (1, 0), (1, 1)])
def test_variants_match_oracle(ctx, pair, n, variant):
    import paper_1612_04787_amd as sw
    fv, iv = variant
    rows = ctx.plan(n, fv, iv)
    print("case plan n=%d variant=%s rows=%s" % (n, variant, rows), flush=True)
    try:
        a, b = pair
        rng = np.random.default_rng(500 + n + 10 * fv + iv)
        k = 3
        th = np.zeros((k, 8), np.float32)
        for i in range(k):
            lin = [1, 0, 0, 1] if i == 0 else list(1 + rng.uniform(-2e-3, 2e-3, 1)) + \
                list(rng.uniform(-5e-3, 5e-3, 2)) + list(1 + rng.uniform(-2e-3, 2e-3, 1))
            th[i] = [rng.uniform(n / 2 + 8, 1500 - n / 2 - 8), rng.uniform(n / 2 + 8, 1500 - n / 2 - 8),
                     lin[0], lin[1], rng.uniform(-2, 2), lin[2], lin[3], rng.uniform(-2, 2)]
        thb = th.copy()
        thb[:, 4] += 0.7
        res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                              torch.ones(k, dtype=torch.int32), torch.from_numpy(th), torch.from_numpy(thb),
                              sw.make_params(p=0.65), surfaces=True)
        torch.cuda.synchronize()
        surf = res["surfaces"].view(k, n, n).cpu().numpy()
        for i in range(k):
            r = O.match_pair(a.numpy(), b.numpy(), th[i].astype(np.float64), thb[i].astype(np.float64), n,
                             O.Params(p=0.65), return_surface=True)
            e = compare(gpu_record(res, i), r, n, surf[i], "plan n=%d %s i=%d" % (n, variant, i))
            print("  ", i, e, flush=True)
    finally:
        ctx.plan(n, 0, 0)


def test_autotune_picks_a_timed_variant(ctx):
    print("case autotune", flush=True)
    out = ctx.autotune(SIZES, pairs_per_size=128)
    for n, (times, plan) in out.items():
        print("   n=%d times_ms=%s -> plan %s" % (n, ["%.3f" % t for t in times], plan), flush=True)
        assert times[0] > 0
        assert (times[7] > 0) == (n <= 128)  # slot 7: the one-workgroup kernel
        assert plan == ctx.plan(n, full=True)
        # the selection rule (FP32, as the library): a slot replaces the
        # running choice only when 2% faster; slot 0 (the defaults) first,
        # then the row variants and the one-workgroup kernel, then the chunk
        # counts of the chosen row variant
        f32 = np.float32
        keep = f32(1.0) - f32(0.02)
        best_t, best_v = f32(times[0]), 0
        for v in (1, 2, 3, 7):
            if times[v] > 0 and f32(times[v]) < best_t * keep:
                best_t, best_v = f32(times[v]), v
        row_best, chunks = best_t, 1
        for v in (4, 5, 6):
            if times[v] > 0 and f32(times[v]) < row_best * keep and f32(times[v]) < best_t:
                best_t, chunks = f32(times[v]), {4: 2, 5: 4, 6: 8}[v]
        if best_v == 7:
            assert n <= 128  # the one-workgroup kernel
            ctx.plan(n, 2, 0, 1)
        else:
            ctx.plan(n, best_v & 1, best_v >> 1, chunks)
        assert ctx.plan(n, full=True) == plan
    for n in SIZES:
        ctx.plan(n, 0, 0, 1)


@pytest.mark.parametrize("n", [64, 256, 512])
@pytest.mark.parametrize("chunks", [2, 4, 8])
def test_chunked_groups_are_bit_identical(ctx, pair, n, chunks):
    """A size group split into chunks on two streams gives the records,
    surfaces and saved state of one launch, also under graph replay and with
    a search radius."""
    import paper_1612_04787_amd as sw
    print("case chunks n=%d chunks=%d" % (n, chunks), flush=True)
    a, b = pair
    rng = np.random.default_rng(900 + n + chunks)
    k = 11
    th = np.zeros((k, 8), np.float32)
    for i in range(k):
        th[i] = [rng.uniform(n / 2 + 8, 1500 - n / 2 - 8), rng.uniform(n / 2 + 8, 1500 - n / 2 - 8), 1, 0,
                 rng.uniform(-2, 2), 0, 1, rng.uniform(-2, 2)]
    thb = th.copy()
    thb[:, 4] += 0.7
    args = ([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32), torch.ones(k, dtype=torch.int32),
            torch.from_numpy(th), torch.from_numpy(thb))
    try:
        for params in (sw.make_params(p=0.65), sw.make_params(p=0.65, max_shift=n // 8)):
            surf = params.max_shift == 0
            ctx.plan(n, 0, 0, 1)
            ref = ctx.match_batch(*args, params, surfaces=surf, save=surf)
            ctx.plan(n, 0, 0, chunks)
            got = ctx.match_batch(*args, params, surfaces=surf, save=surf)
            torch.cuda.synchronize()
            assert torch.equal(ref["raw"], got["raw"])
            if surf:
                assert torch.equal(ref["surfaces"], got["surfaces"])
                one = torch.ones(k, device=dev())
                ga_ref, _ = ctx.match_backward(ref, params, None, one)
                ga_got, _ = ctx.match_backward(got, params, None, one)
                assert torch.equal(ga_ref, ga_got)
            prep = ctx.prepare(*args)
            for rep in range(3):
                out = torch.empty((k, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
                ctx.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out, graph=True)
                torch.cuda.synchronize()
                assert torch.equal(out, ref["raw"]), rep
    finally:
        ctx.plan(n, 0, 0, 1)
