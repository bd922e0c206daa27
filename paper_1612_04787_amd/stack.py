"""Iterative stack alignment with global section affines (Sections III-IV).

Each pass works at one pyramid level (iscale), coarse to fine:

  1. render every raw section by its current affine (mir);
  2. build each section's model as the z-projection of its rendered
     neighbours, self excluded (remod);
  3. match a grid of windows of each raw section, read through its affine,
     against the model (swim), and refine them to the 0.01 px level (plain
     centroid iteration or Newton steps from the adjoint Jacobian);
  4. refit each section's affine to the window correspondences, weighted by
     SNR (mir's least squares, global affine only).

A pass can repeat steps 1-4 (the paper iterates until the SNR scores settle).
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
            n_list = [n] * P
            it = 0
            if refine == "adjoint":
                ta, it, _ = refine_adjoint(sw, images, n_list, ia, ib, ta, tb, params, tol=tol,
                                           stop_frac=stop_frac)
            elif refine == "plain":
                ta, it, _ = refine_plain(sw, images, n_list, ia, ib, ta, tb, params, tol=tol, stop_frac=stop_frac)
            prep = sw.prepare(images, n_list, ia, ib, ta, tb)
            out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=dev)
            sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out)
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
