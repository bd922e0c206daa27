"""Iterative stack alignment: global section affines, then a local-affine mesh (Sections III-IV).

Each pass works at one pyramid level (iscale), coarse to fine:

  1. render every raw section by its current affine (mir);
  2. build each section's model as the z-projection of its rendered
     neighbours, self excluded (remod);
  3. match a grid of windows of each raw section, read through its affine,
     against the model (swim), and refine them to the 0.01 px level (plain
     centroid iteration or Newton steps from the adjoint Jacobian);
  4. refit each section's affine to the window correspondences, weighted by
     SNR (mir's least squares, global affine).

A pass can repeat steps 1-4 (the paper iterates until the SNR scores settle).
align_mesh then replaces the section affines by a triangulated mesh of local
affines (Section IV): the window centres are the mesh nodes and every
triangle's affine is the least-squares fit of the matches in its band.
repair_jumps mends breaks at abrupt content or magnification changes with
one-sided models (Section III, model paragraphs).
Every step is a library call on the current stream; Python only sequences
them and reads a few scalars for reporting.
"""
from __future__ import annotations

import time

import torch

from .refine import refine_adjoint, refine_plain
from .swift import REC_BYTES, make_params, parse_records


def build_pyramid(sw, stack, max_level):
    """[level 0 = stack, level 1, ...] as [S, H_l, W_l] uint8 device stacks."""
    levels = [stack]
    for _ in range(max_level):
        prev = levels[-1]
        S, h, w = prev.shape
        nxt = torch.empty((S, h // 2, w // 2), dtype=torch.uint8, device=stack.device)
        for s in range(S):
            sw.pyramid(prev[s], out=nxt[s])
        levels.append(nxt)
    return levels


def _match_windows(sw, images, ia, ib, ta, tb, n, params, refine, tol, stop_frac):
    """swim with refinement; returns (theta_a, records, iterations)."""
    P = ta.shape[0]
    n_list = [n] * P
    it = 0
    if refine == "adjoint":
        ta, it, _ = refine_adjoint(sw, images, n_list, ia, ib, ta, tb, params, tol=tol, stop_frac=stop_frac)
    elif refine == "plain":
        ta, it, _ = refine_plain(sw, images, n_list, ia, ib, ta, tb, params, tol=tol, stop_frac=stop_frac)
    prep = sw.prepare(images, n_list, ia, ib, ta, tb)
    out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=ta.device)
    sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out)
    return ta, out, it


def _search_start(sw, images, ia, ib, ta, tb, n, p, rings, accept, lookahead=1):
    """Window A parameters moved to each window's kept candidate of a search
    with an SNR stop (Section III): candidates n/2 apart in a square spiral,
    each scored within radius n/4 + 4 px (its own cell).  Returns (theta_a,
    matches run)."""
    from .search import search_offsets, spiral_offsets
    offs = spiral_offsets(n / 2.0, rings)
    got = search_offsets(sw, images, [n] * ta.shape[0], ia, ib, ta, tb, make_params(p=p, max_shift=n // 4 + 4), offs,
                         accept=accept, lookahead=lookahead)
    o = offs.to(ta.device)[got["cand"].long().clamp(min=0)]
    ta = ta.clone()
    ta[:, 4] += o[:, 0]
    ta[:, 7] += o[:, 1]
    return ta, int(sum(got["matched"]))


def align_stack(sw, raw, levels=(2, 1, 0), ns=(128, 256, 512), iters=(2, 1, 1), ks=(3, 3, 3), grid=8, p=0.65,
                refine="adjoint", min_snr=6.0, tol=0.005, stop_frac=0.01, aff=None, on_pass=None, search=None):
    """Aligns a [S, H, W] uint8 device stack.  Returns (affines [S, 6] float64
    device, level-0 aligned frame -> raw section, and a list of per-pass
    reports).  ks: model half-span per level (wider models at coarse levels
    smooth the alignment globally, Section III).  refine: "adjoint", "plain"
    or None (one match, no refinement);
    the refinement of a pass stops when at most stop_frac of the windows still
    step by tol px or more (windows on damaged or featureless content may never
    settle).
    on_pass(report, aff), if given, is called after every pass.
    search: None, or a dict (rings, accept, lookahead) for a search with an SNR stop in
    the first pass (Section III: early stages of an alignment): every window
    first searches candidate offsets (search.search_offsets) and refines from
    its kept one, so sections misplaced beyond one window's capture are
    found.  lookahead (default 1) candidates are matched per round."""
    S, H, W = raw.shape
    dev = raw.device
    pyr = build_pyramid(sw, raw, max(levels))
    if aff is None:
        aff = torch.zeros((S, 6), dtype=torch.float64, device=dev)
        aff[:, 0] = 1.0
        aff[:, 4] = 1.0
    params = make_params(p=p)
    reports = []
    for level, n, reps, k in zip(levels, ns, iters, ks):
        src = pyr[level]
        _, hl, wl = src.shape
        for rep in range(reps):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            rendered = sw.render(src, aff, level)
            model = sw.project(rendered, k=k)
            images = [src[s] for s in range(S)] + [model[s] for s in range(S)]
            ia, ib, ta, tb = sw.stack_windows(aff, level, grid, hl, wl, 0, S)
            P = ta.shape[0]
            searched = 0
            if search is not None and not reports:
                ta, searched = _search_start(sw, images, ia, ib, ta, tb, n, p, int(search.get("rings", 2)),
                                             float(search.get("accept", 15.0)), int(search.get("lookahead", 1)))
            ta, out, it = _match_windows(sw, images, ia, ib, ta, tb, n, params, refine, tol, stop_frac)
            status = sw.fit_sections(ta, tb, out, grid * grid, level, aff, min_snr=min_snr)
            torch.cuda.synchronize(dev)
            el = time.perf_counter() - t0
            rec = parse_records(out)
            snr = rec["snr"].float()
            rep_d = dict(level=level, n=n, k=k, repeat=rep, pairs=P, search_matches=searched, refine_iters=it, ms=el * 1e3,
                         median_snr=float(snr.median()), frac_snr_gt_15=float((snr > 15).float().mean()),
                         frac_weighted=float((snr >= min_snr).float().mean()),
                         singular_sections=int((status != 0).sum()))
            reports.append(rep_d)
            if on_pass is not None:
                on_pass(rep_d, aff)
    return aff, reports


def align_mesh(sw, raw, aff, level=0, n=256, grid=16, k=3, passes=2, p=0.65, refine="adjoint", min_snr=6.0,
               tol=0.005, stop_frac=0.01, pyr=None, on_pass=None):
    """Local-affine alignment of a globally aligned [S, H, W] uint8 device
    stack at one pyramid level (Section IV).  aff [S, 6] float64 (device):
    the section affines, the starting point and the fallback of triangles
    without enough weighted matches.  Each pass renders the stack (through
    the mesh after the first pass), builds the models, matches a grid x grid
    window layout at the mesh nodes (window A read through its node's
    triangle) with refinement, and fits every triangle's affine.  Returns
    (tri_aff [S, 2 (grid-1)^2, 6] float64 device, reports)."""
    S, H, W = raw.shape
    if pyr is None:
        pyr = build_pyramid(sw, raw, level)
    src = pyr[level]
    _, hl, wl = src.shape
    params = make_params(p=p)
    tri = None
    reports = []
    for rep in range(passes):
        torch.cuda.synchronize(raw.device)
        t0 = time.perf_counter()
        if tri is None:
            rendered = sw.render(src, aff, level)
            ia, ib, ta, tb = sw.stack_windows(aff, level, grid, hl, wl, 0, S)
        else:
            rendered = sw.render_mesh(src, tri, grid, level)
            ia, ib, ta, tb = sw.mesh_windows(tri, level, grid, hl, wl, 0, S)
        model = sw.project(rendered, k=k)
        images = [src[s] for s in range(S)] + [model[s] for s in range(S)]
        ta, out, it = _match_windows(sw, images, ia, ib, ta, tb, n, params, refine, tol, stop_frac)
        tri, status = sw.fit_mesh(ta, tb, out, grid, level, aff, min_snr=min_snr)
        torch.cuda.synchronize(raw.device)
        el = time.perf_counter() - t0
        snr = parse_records(out)["snr"].float()
        rep_d = dict(level=level, n=n, grid=grid, k=k, repeat=rep, pairs=ta.shape[0], refine_iters=it,
                     ms=el * 1e3, median_snr=float(snr.median()),
                     frac_weighted=float((snr >= min_snr).float().mean()),
                     singular_triangles=int((status != 0).sum()))
        reports.append(rep_d)
        if on_pass is not None:
            on_pass(rep_d, tri)
    return tri, reports


def _spans(bad):
    """Maximal runs [a, b] of True in a host list."""
    spans, s = [], 0
    while s < len(bad):
        if bad[s]:
            e = s
            while e + 1 < len(bad) and bad[e + 1]:
                e += 1
            spans.append((s, e))
            s = e + 1
        else:
            s += 1
    return spans


def _fit_against(sw, src, models, aff, level, grid, n, params, refine, tol, stop_frac, min_snr, idx=None):
    """Windows of every section (or of the sections idx) through aff,
    matched against models[s] with refinement; returns (fitted affines [S, 6]
    (aff where not fitted), window theta_b, records)."""
    S = src.shape[0]
    g2 = grid * grid
    _, hl, wl = src.shape
    images = [src[s] for s in range(S)] + [models[s] for s in range(S)]
    ia, ib, ta, tb = sw.stack_windows(aff, level, grid, hl, wl, 0, S)
    if idx is not None:
        sel = lambda t: t.view(S, g2, *t.shape[1:])[idx].reshape(-1, *t.shape[1:]).contiguous()  # noqa: E731
        ia, ib, ta, tb = sel(ia), sel(ib), sel(ta), sel(tb)
    ta, out, _ = _match_windows(sw, images, ia, ib, ta, tb, n, params, refine, tol, stop_frac)
    fit = aff.clone()
    if idx is None:
        sw.fit_sections(ta, tb, out, g2, level, fit, min_snr=min_snr)
    else:
        part = aff[idx].contiguous()
        sw.fit_sections(ta, tb, out, g2, level, part, min_snr=min_snr)
        fit[idx] = part
    return fit, tb, out


def repair_jumps(sw, raw, aff, level=0, n=512, grid=8, k=3, break_px=2.0, frac=0.75, p=0.65, refine="adjoint",
                 min_snr=6.0, tol=0.005, stop_frac=0.01, max_breaks=4, pyr=None):
    """Jump repair (Section III, model paragraphs) of an aligned [S, H, W]
    uint8 device stack with section affines aff [S, 6] (float64 device;
    returns the repaired affines and a report).

    1. Breaks: every section is matched (windows through its affine,
       refined) against its left one-sided model and an affine is fitted.
       The first section whose fit moves its window centres by more than
       break_px (RMS, level-0 px) starts a break: the sections from it on are
       joined to the frame before it (swift_join_break).  Repeated, left to
       right, until no break is left (at most max_breaks).
    2. Failed spans: runs of sections whose median window SNR against the
       two-sided model is below frac times the stack median are matched
       against the models on either side (offending sections omitted from
       both) and fitted, and each span gets the Bezier blend from the left
       fit to the right fit (swift_blend_span)."""
    S, H, W = raw.shape
    if pyr is None:
        pyr = build_pyramid(sw, raw, level)
    src = pyr[level]
    params = make_params(p=p)
    g2 = grid * grid
    sc, hf = float(1 << level), (float(1 << level) - 1.0) / 2.0
    torch.cuda.synchronize(raw.device)
    t0 = time.perf_counter()
    breaks, rounds = [], []
    centres = None
    for _ in range(max_breaks):
        rendered = sw.render(src, aff, level)
        left = sw.project_side(rendered, k, -1)
        fit, tb, _ = _fit_against(sw, src, left, aff, level, grid, n, params, refine, tol, stop_frac, min_snr)
        # level-0 window centres and how far the left fit moves them (RMS)
        c = tb.view(S, g2, 8)[:, :, 0:2].double() * sc + hf
        def move(a):
            return torch.stack([a[:, None, 0] * c[..., 0] + a[:, None, 1] * c[..., 1] + a[:, None, 2],
                                a[:, None, 3] * c[..., 0] + a[:, None, 4] * c[..., 1] + a[:, None, 5]], -1)
        score = (move(fit) - move(aff)).square().sum(-1).mean(-1).sqrt().cpu().tolist()
        if centres is None:
            centres = c.cpu().numpy()
        rounds.append(dict(aff=aff.cpu().numpy(), fit=fit.cpu().numpy(), scores=score))
        j = next((s for s in range(1, S) if score[s] > break_px), None)
        if j is None:
            break
        breaks.append(dict(section=j, rms_px=score[j]))
        aff = sw.join_break(j, aff, fit)
    rendered = sw.render(src, aff, level)
    model = sw.project(rendered, k=k)
    _, _, out = _fit_against(sw, src, model, aff, level, grid, n, params, None, tol, stop_frac, min_snr)
    # medians as the midpoint of the two middle values for even counts
    snr = torch.quantile(parse_records(out)["snr"].double().view(S, g2), 0.5, dim=1)
    bad = (snr < frac * torch.quantile(snr, 0.5)).cpu().tolist()
    spans = _spans(bad)
    fits = {}
    if spans:
        idx = torch.tensor([s for s in range(S) if bad[s]], dtype=torch.long, device=raw.device)
        excl = torch.tensor(bad, dtype=torch.uint8, device=raw.device)
        fits = {}
        for side in (-1, 1):
            one = sw.project_side(rendered, k, side, exclude=excl)
            fits[side], _, _ = _fit_against(sw, src, one, aff, level, grid, n, params, refine, tol, stop_frac,
                                            min_snr, idx=idx)
        aff = aff.clone()
        for (a, b) in spans:
            sw.blend_span(a, b, fits[-1], fits[1], aff)
    torch.cuda.synchronize(raw.device)
    report = dict(breaks=breaks, spans=spans, section_snr=snr.cpu().tolist(), ms=(time.perf_counter() - t0) * 1e3,
                  rounds=rounds, centres=centres, side_fits={sd: f.cpu().numpy() for sd, f in fits.items()})
    return aff, report
