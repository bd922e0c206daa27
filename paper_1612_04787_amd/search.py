"""Search with an SNR stop (Section III, SNR paragraph: an SNR above 15 marks a
correct match, so a search for better matches can end there).

A window whose placement is off by more than a window match can capture is
matched at candidate translations in a fixed order (offsets[k] moves window
A's translation).  Every round matches only the windows still searching, and
swift_search_keep keeps each window's best (highest SNR) match and marks it
done once that SNR reaches `accept`.  swift_search_next gathers the windows
still searching; the only host synchronisation per round is reading their
count (it sizes the next batch).

With candidates spaced `step` apart, give params a search radius (max_shift)
of about step / 2: a window then scores each candidate only within that
candidate's cell.  Without it, a candidate whose content only partly overlaps
(a residual between n/2 and n px) can still reach the threshold with its peak
wrapped around the window, which gives a wrong offset.
"""
from __future__ import annotations

import torch

from .swift import REC_BYTES


def spiral_offsets(step: float, rings: int):
    """Candidate translations ordered by ring: the origin, then the 8 cells of
    ring 1, ... on a square grid of `step` px, each ring row-major.  Returns a
    float32 host tensor [(2 rings + 1)^2, 2]."""
    out = [(0.0, 0.0)]
    for r in range(1, rings + 1):
        for j in range(-r, r + 1):
            for i in range(-r, r + 1):
                if max(abs(i), abs(j)) == r:
                    out.append((i * step, j * step))
    return torch.tensor(out, dtype=torch.float32)


def search_offsets(sw, images, n_list, img_a, img_b, theta_a, theta_b, params, offsets, accept=15.0, lookahead=1):
    """Returns dict(best [P, 64] uint8 records, cand [P] int32 kept candidate,
    done [P] uint8, matched [K] windows matched per candidate).  n_list must be
    sorted (any subset of the windows then is too).  Each round is
    swift_search_next (gather the windows still searching), one match of that
    batch, and swift_search_keep; the host reads the batch size in between.
    lookahead B > 1 (one window edge only) matches the windows still searching
    at the next B candidates in one batch and keeps them candidate by
    candidate: the result is the same, with fewer rounds and some matches
    past a window's stop (counted in `matched`)."""
    dev = sw.device
    P = len(n_list)
    K = int(offsets.shape[0])
    n_host = [int(n) for n in n_list]
    mixed = len(set(n_host)) > 1
    B = max(1, int(lookahead))
    if mixed and B > 1:
        raise ValueError("lookahead > 1 needs a single window edge (a repeated ragged batch is not sorted)")
    img_a = img_a.to(dev, torch.int32).contiguous()
    img_b = img_b.to(dev, torch.int32).contiguous()
    theta_a = theta_a.to(dev, torch.float32).contiguous()
    theta_b = theta_b.to(dev, torch.float32).contiguous()
    best = torch.zeros((P, REC_BYTES), dtype=torch.uint8, device=dev)
    cand = torch.full((P,), -1, dtype=torch.int32, device=dev)
    done = torch.zeros(P, dtype=torch.uint8, device=dev)
    idx = torch.empty(B * P, dtype=torch.int32, device=dev)
    ia = torch.empty(B * P, dtype=torch.int32, device=dev)
    ib = torch.empty(B * P, dtype=torch.int32, device=dev)
    ta = torch.empty((B * P, 8), dtype=torch.float32, device=dev)
    tb = torch.empty((B * P, 8), dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    recs = torch.empty((B * P, REC_BYTES), dtype=torch.uint8, device=dev)
    table = sw.image_table(images)
    offs = offsets.tolist()
    matched = []
    k = 0
    while k < K:
        if P == 0:
            matched.append(0)
            k += 1
            continue
        sw.search_next(done, offs[k][0], offs[k][1], img_a, img_b, theta_a, theta_b, idx, ia, ib, ta, tb, count)
        n = int(count.item())
        if n == 0:
            matched.extend([0] * (K - k))
            break
        b = min(B, K - k)
        for c in range(1, b):  # the same windows (done is unchanged) at the next candidates
            sw.search_next(done, offs[k + c][0], offs[k + c][1], img_a, img_b, theta_a, theta_b, idx[c * n:],
                           ia[c * n:], ib[c * n:], ta[c * n:], tb[c * n:], count)
        sub = [n_host[i] for i in idx[:n].tolist()] if mixed else [n_host[0]] * n
        pr = sw.make_pairs(sub * b, ia, ib, ta, tb)
        sw.match_batch_raw(table, len(images), pr, params, recs[:b * n])
        for c in range(b):
            sw.search_keep(P, idx[c * n:(c + 1) * n], recs[c * n:(c + 1) * n], k + c, accept, best, cand, done)
            matched.append(n)
        k += b
    return dict(best=best, cand=cand, done=done, matched=matched)
