"""Ragged batches: the concurrent-size-group flag and the captured hipGraph
entry point give the same records as the plain sequential call, on every
replay, with the inputs' contents changed between replays."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def _batch(rng, size):
    ns, th = [], []
    for n in (64, 128, 256, 512, 1024):
        for _ in range(3):
            cx = rng.uniform(n / 2 + 8, size - n / 2 - 8)
            cy = rng.uniform(n / 2 + 8, size - n / 2 - 8)
            th.append([cx, cy, 1, 0, rng.uniform(-3, 3), 0, 1, rng.uniform(-3, 3)])
            ns.append(n)
    return ns, np.array(th, np.float32)


def test_concurrent_and_graph_match_sequential(ctx):
    import paper_1612_04787_amd as sw
    from datagen import make_section_pair
    print("case graph ragged", flush=True)
    a, b, _, _ = make_section_pair(1400, 1400, 51, 551, device=dev(), max_shift=5.0)
    rng = np.random.default_rng(5)
    ns, th = _batch(rng, 1400)
    P = len(ns)
    tha = torch.from_numpy(th).to(dev())
    thb = tha.clone()
    thb[:, 4] += 1.5
    z = torch.zeros(P, dtype=torch.int32, device=dev())
    prep = ctx.prepare([a, b], ns, z, z + 1, tha, thb)
    table, pr = prep["table"], prep["pairs"]
    tha_d, thb_d = prep["keep"][2], prep["keep"][3]
    need, _ = ctx.workspace_size(pr, sw.make_params())
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    seq = torch.empty((P, 64), dtype=torch.uint8, device=dev())
    con = torch.empty_like(seq)
    gra = torch.empty_like(seq)
    p_seq = sw.make_params(p=0.65)
    p_con = sw.make_params(p=0.65, flags=sw.FLAG_CONCURRENT_SIZES)
    for rep in range(4):
        # new window positions in the same buffers: the graph reads them when it runs
        tha_d[:, 4] = torch.from_numpy(rng.uniform(-3, 3, P).astype(np.float32)).to(dev())
        ctx.match_batch_raw(table, 2, pr, p_seq, seq, ws=ws)
        torch.cuda.synchronize()
        ref = seq.clone()
        ctx.match_batch_raw(table, 2, pr, p_con, con, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(con, ref), rep
        gra.zero_()
        ctx.match_batch_raw(table, 2, pr, p_con, gra, ws=ws, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(gra, ref), rep
        r = sw.parse_records(ref)
        assert bool((r["n"].cpu() == torch.tensor(ns, dtype=torch.int32)).all())
        print("   replay %d: %d records equal" % (rep, P), flush=True)


def test_mixed_group_sizes_match_sequential(ctx):
    """A ragged batch with one size group large enough to fill the GPU (130
    pairs of 512^2: 8320 forward row workgroups), which the concurrent flag
    keeps on the call's stream, beside small groups of 128^2 and 256^2 on the
    context's streams: the same records as the sequential call, direct and
    as graph replays."""
    import paper_1612_04787_amd as sw
    from datagen import make_section_pair
    print("case graph mixed group sizes", flush=True)
    a, b, _, _ = make_section_pair(1400, 1400, 53, 553, device=dev(), max_shift=5.0)
    rng = np.random.default_rng(12)
    ns, th = [], []
    for n, k in ((128, 3), (256, 3), (512, 130)):
        for _ in range(k):
            cx = rng.uniform(n / 2 + 8, 1400 - n / 2 - 8)
            cy = rng.uniform(n / 2 + 8, 1400 - n / 2 - 8)
            th.append([cx, cy, 1, 0, rng.uniform(-3, 3), 0, 1, rng.uniform(-3, 3)])
            ns.append(n)
    th = np.array(th, np.float32)
    P = len(ns)
    tha = torch.from_numpy(th).to(dev())
    thb = tha.clone()
    thb[:, 7] -= 1.25
    z = torch.zeros(P, dtype=torch.int32, device=dev())
    prep = ctx.prepare([a, b], ns, z, z + 1, tha, thb)
    table, pr = prep["table"], prep["pairs"]
    need, _ = ctx.workspace_size(pr, sw.make_params())
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    ref = torch.empty((P, 64), dtype=torch.uint8, device=dev())
    con = torch.empty_like(ref)
    gra = torch.empty_like(ref)
    p_con = sw.make_params(p=0.65, flags=sw.FLAG_CONCURRENT_SIZES)
    ctx.match_batch_raw(table, 2, pr, sw.make_params(p=0.65), ref, ws=ws)
    torch.cuda.synchronize()
    ctx.match_batch_raw(table, 2, pr, p_con, con, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(con, ref)
    for rep in range(3):
        gra.zero_()
        ctx.match_batch_raw(table, 2, pr, p_con, gra, ws=ws, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(gra, ref), rep
    r = sw.parse_records(ref)
    assert bool((r["n"].cpu() == torch.tensor(ns, dtype=torch.int32)).all())
    assert float(r["snr"].min()) > 0


def test_graph_cache_keys(ctx):
    """Different outputs or parameters make different graphs; each stays
    correct after the others have run."""
    import paper_1612_04787_amd as sw
    from datagen import make_section_pair
    print("case graph keys", flush=True)
    a, b, _, _ = make_section_pair(900, 900, 61, 661, device=dev(), max_shift=3.0)
    rng = np.random.default_rng(8)
    ns = [128] * 4 + [256] * 4
    th = np.array([[rng.uniform(200, 700), rng.uniform(200, 700), 1, 0, 0, 0, 1, 0] for _ in ns], np.float32)
    t = torch.from_numpy(th).to(dev())
    z = torch.zeros(len(ns), dtype=torch.int32, device=dev())
    prep = ctx.prepare([a, b], ns, z, z + 1, t, t.clone())
    outs = {}
    for p in (0.0, 0.65, 1.0):
        params = sw.make_params(p=p)
        ref = torch.empty((len(ns), 64), dtype=torch.uint8, device=dev())
        ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, ref)
        g = torch.empty_like(ref)
        ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, g, graph=True)
        outs[p] = (ref, g, params)
    for p, (ref, g, params) in outs.items():
        g.zero_()
        ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, g, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(g, ref), p
