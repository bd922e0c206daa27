"""Host logic of the search driver on the CPU: rounds, candidate offsets,
lookahead bookkeeping and per-candidate batch sizes, through a stand-in for
the library whose gather and keep follow swift_search_next and
swift_search_keep as include/swift.h documents them, and whose match scores
window w at candidate k from a table.  The expected selection is the
oracle's search rule."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_04787_amd.search import search_offsets, spiral_offsets


class TableSwift:
    device = torch.device("cpu")

    def __init__(self, snr, offs):
        self.snr = snr  # [K, P]
        self.offs = offs.numpy()
        self.matches = 0

    def image_table(self, images):
        return None

    @staticmethod
    def make_pairs(n_list, img_a, img_b, theta_a, theta_b):
        return dict(n=len(n_list), ta=theta_a, tb=theta_b)

    def search_next(self, done, ox, oy, img_a, img_b, theta_a, theta_b, idx, ia, ib, ta, tb, count):
        keep = torch.nonzero(done == 0).flatten()
        n = keep.numel()
        idx[:n] = keep.to(torch.int32)
        ia[:n], ib[:n] = img_a[keep], img_b[keep]
        t = theta_a[keep].clone()
        t[:, 4] += ox
        t[:, 7] += oy
        ta[:n], tb[:n] = t, theta_b[keep]
        count[0] = n

    def match_batch_raw(self, table, n_imgs, pr, params, out):
        n = pr["n"]
        ta, tb = pr["ta"][:n], pr["tb"][:n]
        w = tb[:, 0].long().numpy()  # the window's id rides in window B's centre
        o = np.stack([(ta[:, 4] - tb[:, 4]).numpy(), (ta[:, 7] - tb[:, 7]).numpy()], 1)
        k = np.array([int(np.flatnonzero((self.offs == oi).all(1))[0]) for oi in o])
        out.zero_()
        f = out.view(torch.float32).view(-1, 16)
        f[:n, 5] = torch.from_numpy(self.snr[k, w].astype(np.float32))
        f[:n, 0] = torch.from_numpy(k.astype(np.float32))
        self.matches += n

    def search_keep(self, P, idx, recs, cand, accept, best, best_cand, done):
        s = recs.view(torch.float32).view(-1, 16)[:, 5]
        bs = best.view(torch.float32).view(P, 16)[:, 5]
        for i, w in enumerate(idx.tolist()):
            if w < 0 or w >= P or done[w]:
                continue
            if best_cand[w] < 0 or s[i] > bs[w]:
                best[w] = recs[i]
                best_cand[w] = cand
            if bs[w] >= accept:
                done[w] = 1


def _windows(P):
    th = torch.zeros((P, 8))
    th[:, 2] = th[:, 6] = 1.0
    tb = th.clone()
    tb[:, 0] = torch.arange(P, dtype=torch.float32)
    z = torch.zeros(P, dtype=torch.int32)
    return z, z + 1, th, tb


@pytest.mark.parametrize("ahead", [1, 2, 3, 25, 40])
@pytest.mark.parametrize("accept", [15.0, float("inf"), 0.0])
def test_search_driver_rounds(ahead, accept):
    rng = np.random.default_rng(int(ahead * 7 + (0 if accept == np.inf else accept)))
    offs = spiral_offsets(10.0, 2)
    K, P = offs.shape[0], 40
    snr = rng.uniform(0, 20, (K, P))
    snr[:, 3] = 9.0  # equal SNRs: the first candidate is kept
    sw = TableSwift(snr, offs)
    ia, ib, ta, tb = _windows(P)
    got = search_offsets(sw, [None, None], [128] * P, ia, ib, ta, tb, None, offs, accept=accept, lookahead=ahead)
    counts = []
    for w in range(P):
        arg, cnt = O.search_select(snr[:, w].astype(np.float32).tolist(), accept)
        counts.append(cnt)
        assert got["cand"][w] == arg, (w, got["cand"][w], arg)
        rec = got["best"][w].view(torch.float32)
        assert rec[0] == arg and rec[5] == np.float32(snr[arg, w])
        assert got["done"][w] == (1 if snr[arg, w].astype(np.float32) >= accept else 0)
    counts = np.array(counts)
    want, k = [], 0
    while k < K:
        n = int((counts > k).sum())
        if n == 0:
            want += [0] * (K - k)
            break
        b = min(ahead, K - k)
        want += [n] * b
        k += b
    assert got["matched"] == want
    assert sw.matches == sum(want)


def test_search_driver_edges():
    offs = spiral_offsets(10.0, 1)
    sw = TableSwift(np.zeros((9, 4)), offs)
    ia, ib, ta, tb = _windows(4)
    # several window edges cannot be matched ahead (the repeated batch would
    # not be sorted)
    with pytest.raises(ValueError):
        search_offsets(sw, [None, None], [64, 64, 128, 128], ia, ib, ta, tb, None, offs, lookahead=2)
    # no windows: nothing matched
    e = torch.zeros(0, dtype=torch.int32)
    got = search_offsets(sw, [None, None], [], e, e, torch.zeros((0, 8)), torch.zeros((0, 8)), None, offs)
    assert got["matched"] == [0] * 9 and got["cand"].numel() == 0
