"""swift_match_batch_noalloc (the match with the library's fixed scratch
array instead of a caller workspace) against swift_match_batch, through the C
ABI: identical records on two calls in a row, the second with a smaller
batch, and a batch beyond the scratch refused."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda", 0)


def _batch(sw, ctx, a, b, ns, seed):
    rng = np.random.default_rng(seed)
    k = len(ns)
    th = np.zeros((k, 8), np.float32)
    for i, n in enumerate(ns):
        lin = [1, 0, 0, 1] if i % 2 == 0 else [1 + 1e-3, -2e-3, 1.5e-3, 1 - 1e-3]
        th[i] = [rng.uniform(n / 2 + 8, 1500 - n / 2 - 8), rng.uniform(n / 2 + 8, 1500 - n / 2 - 8),
                 lin[0], lin[1], rng.uniform(-2, 2), lin[2], lin[3], rng.uniform(-2, 2)]
    thb = th.copy()
    thb[:, 4] += 0.7
    thb[:, 7] -= 1.3
    return ctx.prepare([a.to(dev()), b.to(dev())], ns, torch.zeros(k, dtype=torch.int32),
                       torch.ones(k, dtype=torch.int32), torch.from_numpy(th), torch.from_numpy(thb))


def _noalloc(ctx, prep, params, out):
    from paper_1612_04787_amd import swift as S
    return ctx.lib.swift_match_batch_noalloc(ctx.h, S._ptr(prep["table"]), int(prep["n_imgs"]),
                                              C.byref(prep["pairs"]), C.byref(params), S._ptr(out), ctx.stream())


def test_noalloc_matches_match_batch():
    import paper_1612_04787_amd as sw
    from datagen import make_section_pair
    print("case noalloc", flush=True)
    ctx = sw.Swift(0)
    try:
        a, b, _, _ = make_section_pair(1500, 1500, 71, 771, device="cpu", max_shift=5.0)
        params = sw.make_params(p=0.65)
        # first call: a ragged batch of four sizes; second: fewer, smaller windows
        for ns, seed in (([64] * 5 + [128] * 4 + [256] * 3 + [512] * 2, 11), ([64] * 3 + [128] * 2, 12)):
            prep = _batch(sw, ctx, a, b, ns, seed)
            k = len(ns)
            ref = torch.empty((k, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
            ctx.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, ref)
            got = torch.full((k, sw.swift.REC_BYTES), 255, dtype=torch.uint8, device=dev())
            rc = _noalloc(ctx, prep, params, got)
            assert rc == 0, ctx.lib.swift_last_error()
            torch.cuda.synchronize()
            assert torch.equal(got, ref), ns
            r = sw.parse_records(got)
            assert bool((r["snr"] > 0).all())
            print("   %d pairs: records identical" % k, flush=True)
        # the pruned inverse through the scratch as well
        prm = sw.make_params(p=0.65, max_shift=16)
        ref = torch.empty((len(ns), sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
        ctx.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], prm, ref)
        got = torch.empty_like(ref)
        assert _noalloc(ctx, prep, prm, got) == 0
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        # beyond the scratch: 64 windows of 1024^2 need about 540 MB
        big = _batch(sw, ctx, a, b, [1024] * 64, 13)
        out = torch.empty((64, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev())
        assert _noalloc(ctx, big, params, out) == -3
        assert b"scratch" in ctx.lib.swift_last_error()
    finally:
        ctx.close()
