"""Iterative sub-pixel refinement of window matches (Section IV: the matching
is repeated, each time from the updated alignment, until the scores settle).

Two drivers over the same library calls:
  refine_plain    match, then move each window A by its centroid shift;
  refine_adjoint  centroid steps while the batch's longest step is at least
                  `newton_below` px, by default the step clamp (half a pixel)
                  (far from the solution the centroid step is cheap and halves
                  the error, and the Jacobian measured there does not hold at
                  the solution; once no step is clamped it does), then match + one
                  adjoint pass for the Jacobian J of the centroid shift d with
                  respect to the translation of window A and a Newton step
                  t <- t - J^-1 d on d(t) = 0 (centroid step while the integer
                  peak is not yet at the origin).
The centroid of a bilinearly resampled window underestimates the shift (its
slope J is well below 1), so the plain iteration contracts the error by only
|1 - J| per step, while Newton's reaches the 0.01 px level in a few steps.
Both stop when the longest step of the batch is below `tol` pixels.  Each
iteration is a fixed sequence of launches on the current stream; the only
host synchronisation is reading the longest step.  params may carry a search
radius (max_shift): every match of the driver then uses the pruned inverse,
which finds the full search's peaks while the shifts stay inside it.
"""
from __future__ import annotations

import torch

from .swift import REC_BYTES

CENTROID, NEWTON = 0, 1


def _state(sw, images, n_list, img_a, img_b, theta_a, theta_b):
    prep = sw.prepare(images, n_list, img_a, img_b, theta_a, theta_b)
    return prep, prep["keep"][2]  # device theta_a updated in place


def _done(step, tol, stop_frac):
    """Longest step of the batch (for the history) and whether to stop: every
    step below tol, or (stop_frac > 0) at most that fraction of them not."""
    if step.numel() == 0:
        return 0.0, True
    if stop_frac > 0.0:
        m, frac = torch.stack([step.max(), (step >= tol).float().mean()]).tolist()
        return m, frac <= stop_frac
    m = float(step.max())
    return m, m < tol


def refine_plain(sw, images, n_list, img_a, img_b, theta_a, theta_b, params, tol=0.005, max_iter=60,
                 max_step=0.5, stop_frac=0.0):
    """Returns (theta_a [P, 8], iterations, list of longest steps)."""
    prep, th = _state(sw, images, n_list, img_a, img_b, theta_a.clone(), theta_b)
    P = prep["pairs"].n_pairs
    out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=sw.device)
    step = torch.empty(P, dtype=torch.float32, device=sw.device)
    hist = []
    for it in range(1, max_iter + 1):
        sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out)
        sw.refine_update(out, th, CENTROID, None, max_step, step)
        m, stop = _done(step, tol, stop_frac)
        hist.append(m)
        if stop:
            return th, it, hist
    return th, max_iter, hist


def refine_adjoint(sw, images, n_list, img_a, img_b, theta_a, theta_b, params, tol=0.005, max_iter=20,
                   max_step=0.5, stop_frac=0.0, newton_below=None):
    """Returns (theta_a [P, 8], iterations, list of longest steps).  Centroid
    steps until the longest step of the batch is below newton_below px (None:
    max_step, i.e. until no step is clamped), Newton
    steps from then on.  The Jacobian is recomputed every Newton iteration: it
    changes across a pixel cell (bilinear sampling), and reusing an earlier
    one (chord steps) stalls.  Only its translation columns are computed (the
    Newton step uses no others)."""
    from .swift import FLAG_JAC_TRANSLATION, make_params
    if newton_below is None:
        newton_below = max_step
    jparams = make_params(params.p, params.eps_rel, params.taper_frac, params.centroid_r,
                          params.flags | FLAG_JAC_TRANSLATION, params.max_shift)
    prep, th = _state(sw, images, n_list, img_a, img_b, theta_a.clone(), theta_b)
    P = prep["pairs"].n_pairs
    out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=sw.device)
    _, sv = sw.workspace_size(prep["pairs"], params)
    saved = torch.empty(max(sv, 256), dtype=torch.uint8, device=sw.device)
    jac = torch.empty((P, 2, 6), dtype=torch.float32, device=sw.device)
    step = torch.empty(P, dtype=torch.float32, device=sw.device)
    hist = []
    newton = False
    for it in range(1, max_iter + 1):
        if newton:
            sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out, saved=saved)
            sw.centroid_jacobian_raw(prep["table"], prep["n_imgs"], prep["pairs"], jparams, saved, jac)
            sw.refine_update(out, th, NEWTON, jac, max_step, step)
        else:
            sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out)
            sw.refine_update(out, th, CENTROID, None, max_step, step)
        m, stop = _done(step, tol, stop_frac)
        hist.append(m)
        if stop and newton:
            return th, it, hist
        if not newton:
            # switch when the steps are small; with stop_frac, up to that
            # fraction of windows may still step further (as in _done)
            newton = _done(step, newton_below, stop_frac)[1]
    return th, max_iter, hist


def refine_adjoint_graph(sw, images, n_list, img_a, img_b, theta_a, theta_b, params, tol=0.005, max_iter=20,
                         max_step=0.5, newton_below=None, theta_trace=None):
    """refine_adjoint with every iteration one replayed graph: the match of the
    whole (ragged) batch, for Newton iterations the centroid Jacobian, the
    update of theta_a, and the copy of the per-window steps into pinned host
    memory, from which the host reads the stop test (one synchronisation per
    iteration, no host-side launches).  Two graphs are captured once per call:
    the centroid iteration and the Newton iteration.  theta_trace, if given
    ([max_iter, P, 8] device), receives theta_a after each iteration.
    Returns (theta_a [P, 8], iterations, list of longest steps, list of host
    times in seconds after each iteration, measured from the first replay)."""
    import time

    from .swift import FLAG_JAC_TRANSLATION, make_params
    if newton_below is None:
        newton_below = max_step
    jparams = make_params(params.p, params.eps_rel, params.taper_frac, params.centroid_r,
                          params.flags | FLAG_JAC_TRANSLATION, params.max_shift)
    prep, th = _state(sw, images, n_list, img_a, img_b, theta_a.clone(), theta_b)
    P = prep["pairs"].n_pairs
    dev = sw.device
    out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=dev)
    need, sv = sw.workspace_size(prep["pairs"], params)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    saved = torch.empty(max(sv, 256), dtype=torch.uint8, device=dev)
    jac = torch.empty((P, 2, 6), dtype=torch.float32, device=dev)
    step = torch.empty(P, dtype=torch.float32, device=dev)
    host_step = torch.empty(P, dtype=torch.float32, pin_memory=True)

    def body(newton):
        if newton:
            sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out, saved=saved, ws=ws)
            sw.centroid_jacobian_raw(prep["table"], prep["n_imgs"], prep["pairs"], jparams, saved, jac, ws=ws)
            sw.refine_update(out, th, NEWTON, jac, max_step, step)
        else:
            sw.match_batch_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, out, ws=ws)
            sw.refine_update(out, th, CENTROID, None, max_step, step)
        host_step.copy_(step, non_blocking=True)

    # capture on a side stream (theta is restored after the warm-up runs that
    # precede each capture; a capture itself executes nothing)
    th0 = th.clone()
    graphs = {}
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for newton in (False, True):
            body(newton)
            torch.cuda.current_stream(dev).synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                body(newton)
            graphs[newton] = g
    torch.cuda.current_stream(dev).wait_stream(side)
    th.copy_(th0)
    torch.cuda.synchronize(dev)

    hist, times = [], []
    newton = False
    t0 = time.perf_counter()
    for it in range(1, max_iter + 1):
        graphs[newton].replay()
        if theta_trace is not None:
            theta_trace[it - 1].copy_(th)
        torch.cuda.current_stream(dev).synchronize()
        m = float(host_step.max()) if P else 0.0
        hist.append(m)
        times.append(time.perf_counter() - t0)
        if newton and m < tol:
            return th, it, hist, times
        if not newton:
            newton = m < newton_below
    return th, max_iter, hist, times
