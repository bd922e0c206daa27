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


def align_stack(sw, raw, levels=(2, 1, 0), ns=(128, 256, 512), iters=(2, 1, 1), ks=(3, 3, 3), grid=8, p=0.65,
                refine="adjoint", min_snr=6.0, tol=0.005, stop_frac=0.01, aff=None, on_pass=None):
    """Aligns a [S, H, W] uint8 device stack.  Returns (affines [S, 6] float64
    device, level-0 aligned frame -> raw section, and a list of per-pass
    reports).  ks: model half-span per level (wider models at coarse levels
    smooth the alignment globally, Section III).  refine: "adjoint", "plain"
    or None (one match, no refinement);
    the refinement of a pass stops when at most stop_frac of the windows still
    step by tol px or more (windows on damaged or featureless content may never
    settle).
    on_pass(report, aff), if given, is called after every pass."""
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
            ta, out, it = _match_windows(sw, images, ia, ib, ta, tb, n, params, refine, tol, stop_frac)
            status = sw.fit_sections(ta, tb, out, grid * grid, level, aff, min_snr=min_snr)
            torch.cuda.synchronize(dev)
            el = time.perf_counter() - t0
            rec = parse_records(out)
            snr = rec["snr"].float()
            rep_d = dict(level=level, n=n, k=k, repeat=rep, pairs=P, refine_iters=it, ms=el * 1e3,
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
