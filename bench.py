"""Throughput of the whitened FFT window-matching hot path on one MI355X.

Workload (512^2 headline batch): 64 synthetic 4096^2 uint8 sections with
accumulated drift and per-section affine distortion; the reference of every
section is its +-3 z-projection; an 8 x 8 grid of 512^2 windows per section
gives 4096 window pairs.  One step = projection of the whole stack plus the
whitened match of all 4096 pairs (gather, taper + mean, forward FFTs,
whitening, inverse FFT, peak / SNR / centroid).  Inputs are resident in HBM
before the timed region.

Prints one JSON line (metric, value in pairs/s, roofline of the dominant
kernel from live HIP-event timing, and the FP64 oracle's throughput on a
bounded sample of the same pairs on the host cores).  Further blocks of the
line: the same step with a pruned inverse (search radius 64 px), the same
pairs scored by Pearson-normalised correlation, plain vs
adjoint refinement to 0.01 px, the iterative stack loop, jump repair on a
stack with a magnification change, the local-affine mesh on a bent stack,
and ragged multi-level batches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "512² window-pair matches/sec + HBM GB/s; plain vs batched+adjoint at 0.01px"
HBM_PEAK_GBS = 8000.0
S_SECTIONS, SIZE, N, GRID, K_PROJ, P_WHITEN = 64, 4096, 512, 8, 3, 0.65
PRUNE_R = N // 8  # search radius of the pruned-inverse variant (64 px at 512^2)
REFINE_R = 8      # search radius of the pruned refinement (its shifts stay below a pixel)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_match_512_headline.txt")
CONFIG2_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_section_pair_1024.txt")
LDS_FILE = os.path.join(ROOT, "profiles", "lds_match_512_headline.txt")
# LDS peak: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4


def kernel_bytes(name: str, n: int, pairs: int, sections: int, size: int) -> float:
    """Algorithmic HBM bytes of one launch of a kernel over the whole batch:
    what the kernel must read and write at least (inputs once, exchange
    buffers once each way), not what the caches end up doing."""
    nn = float(n) * n
    half = 8.0 * n * (n // 2 + 1)  # one complex64 half spectrum
    if name.startswith("k_row_fwd"):
        per = 2 * nn + 8 * nn          # two uint8 windows in, packed complex row spectra out
    elif name.startswith("k_col"):
        per = 8 * nn + half            # packed spectra in, inverse-column half spectrum out
    elif name.startswith("k_row_inv"):
        per = half                     # half spectrum in (surface statistics out are tiny)
    elif name.startswith("k_finalize"):
        per = 24.0 * (n // 2 + 1) + 64  # three spectrum rows re-read + record
    elif name.startswith("k_pair_stats"):
        per = 64
    elif name.startswith("k_project"):
        return 2.0 * sections * size * size  # every section read once, every model written once
    else:
        per = 0.0
    return per * pairs


def kept_rows(n: int, radius: int, inv_rows: int) -> int:
    """Surface rows the pruned column pass writes back for a search radius:
    |y| <= radius + 1, rounded out to whole inverse row blocks (the library's
    rule; every row when the blocks would overlap)."""
    rr, blocks = radius + 1, n // inv_rows
    lo, hs = rr // inv_rows + 1, (n - rr) // inv_rows
    return n if lo >= hs else (lo + blocks - hs) * inv_rows


def variant_bytes(name: str, n: int, pairs: int, rows: int, pearson: bool) -> float:
    """Algorithmic HBM bytes of one launch of a kernel of the pruned or
    Pearson step: as kernel_bytes, with rows surface rows written back by the
    column pass and read by the inverse row pass, and the Pearson row sums
    (f', f'^2 per row and placement) and patch energies."""
    nn = float(n) * n
    npl = n // 2 + 1
    if name.startswith("k_row_fwd"):
        per = 2 * nn + 8 * nn + (8.0 * n * npl if pearson else 0.0)
    elif name.startswith("k_col"):
        per = 8 * nn + 8.0 * rows * npl
    elif name.startswith("k_row_inv"):
        per = 8.0 * rows * npl + (4.0 * npl * npl if pearson else 0.0)
    elif name.startswith("k_ncc_energy"):
        per = 8.0 * n * npl + 4.0 * npl * npl
    else:
        return kernel_bytes(name, n, pairs, S_SECTIONS, SIZE)
    return per * pairs


def variant_kernels(prof, n, pairs, rows, pearson, traffic_file=None, steps=None):
    """Per-kernel launches, average ms, algorithmic bytes per launch and GB/s
    of a step variant, and the HBM roofline of its longest kernel (with the
    measured traffic of traffic_file when it belongs to the current kernel
    sources).  `pairs` per step; with `steps` profiled steps a kernel launched
    cnt times covers pairs * steps / cnt pairs per launch."""
    kernels = {}
    for name, (cnt, tot) in prof.items():
        avg = tot / cnt
        per_launch = pairs * steps / cnt if steps else pairs
        b = variant_bytes(name, n, per_launch, rows, pearson)
        kernels[name] = dict(launches=cnt, avg_ms=avg, bytes=b, gbs=b / (avg / 1e3) / 1e9)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    d = kernels[dom]
    traffic = None
    if traffic_file is not None:
        from paper_1612_04787_amd.counters import read_traffic, source_digest
        # the library timer names the Pearson row pass k_row_fwd<N>; its
        # rocprofv3 summary names the instance apart
        name = dom.replace("k_row_fwd", "k_row_fwd_pearson") if pearson else dom
        traffic, digest = read_traffic(traffic_file, name)
        if digest != source_digest():
            traffic = None
    roof = dict(bound="hbm", kernel=dom, achieved=d["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=d["gbs"] / HBM_PEAK_GBS, traffic=traffic, bytes_per_launch=d["bytes"], avg_ms=d["avg_ms"])
    return kernels, roof


def pair_bytes(n: int) -> float:
    """Algorithmic bytes per pair of the whole match path: uint8 inputs, the
    record, and one write + read of each exchanged spectrum."""
    return 2.0 * n * n + 64 + 48.0 * n * (n // 2 + 1)


FP32_PEAK_TFLOPS = 157.3


def path_roofline(pairs_per_s: float, n: int) -> dict:
    """Achieved pairs/s against min(HBM bound, ALU bound) of the per-pair
    model, and against the input-only bound (2 N^2 + 64 bytes per pair, or the
    ALU bound if that is lower)."""
    hbm = HBM_PEAK_GBS * 1e9 / pair_bytes(n)
    alu = FP32_PEAK_TFLOPS * 1e12 / pair_flops(n)
    inp = min(HBM_PEAK_GBS * 1e9 / (2.0 * n * n + 64), alu)
    bound = min(hbm, alu)
    return dict(bound="hbm" if hbm <= alu else "alu", bound_pairs_per_s=bound, frac=pairs_per_s / bound,
                input_only_bound_pairs_per_s=inp, input_only_frac=pairs_per_s / inp)


def hbm_reference(dev, reps: int = 20) -> dict:
    """Bandwidth a plain streaming kernel reaches on this GPU: torch's
    elementwise FP32 multiply reading and writing 1 GiB each, median of `reps`
    runs timed with HIP events on the current stream.  The practical
    counterpart of the 8 TB/s peak for kernels that read and write."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(x, 1.0, out=y)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    ms = ts[len(ts) // 2]
    nbytes = 2 * x.numel() * x.element_size()
    del x, y
    return dict(elementwise_rw_gbs=nbytes / (ms / 1e3) / 1e9, ms=ms, bytes=nbytes,
                note="torch.mul(x, 1.0, out=y), 1 GiB read + 1 GiB written, FP32")


def pair_flops(n: int) -> float:
    import math
    return 7.5 * n * n * math.log2(n * n) + 40.0 * n * n


class one_chunk:
    """Context in which the listed window sizes run as one chunk (their tuned
    row variants kept): each kernel launch then covers the whole batch with
    nothing else on the GPU, which is how the per-kernel timing is taken."""

    def __init__(self, ctx, sizes):
        self.ctx, self.sizes = ctx, list(sizes)

    def __enter__(self):
        self.keep = {n: self.ctx.plan(n, full=True)[2] for n in self.sizes}
        for n in self.sizes:
            self.ctx.plan(n, -1, -1, 1)
        return self

    def __exit__(self, *exc):
        for n, c in self.keep.items():
            self.ctx.plan(n, -1, -1, c)
        return False


def median_event_ms(fn, reps, warm=2):
    """Median over `reps` calls of fn, each bracketed by HIP events on the
    current stream (the stream the library launches on)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


# --------------------------------------------------------------------------- CPU oracle leg
def _oracle_worker(job):
    import numpy as np

    import oracle as O
    t0 = time.perf_counter()
    out = []
    for (wa, wb, tha, thb, n, p) in job:
        r = O.match_pair(wa, wb, tha, thb, n, O.Params(p=p))
        out.append((r["ix"], r["iy"], r["snr"]))
    return out, time.perf_counter() - t0


def host_cores():
    """(cores used, cores this process may run on, logical CPUs of the host).
    The CPU legs use every core the process may run on, at most 16 (the host
    share of one GPU on the benchmark machines)."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return min(16, aff), aff, os.cpu_count() or 1


def _fp32_worker(job):
    from oracle import cpu_fp32
    t0 = time.perf_counter()
    out = []
    # every pair is its own crop, so each is a batch of one
    for (a, b, tha, thb, n, p) in job:
        r = cpu_fp32.match_batch(a, b, tha[None], thb[None], n, p=p, workers=1)
        out.append((int(r["ix"][0]), int(r["iy"][0]), float(r["snr"][0])))
    return out, time.perf_counter() - t0


def _sample_jobs(stack_cpu, refs_cpu, centres, n_sample_sections, per_section, seed=0):
    """Pairs of the benchmark batch cropped with a margin (so clamped reads at
    the section border are reproduced exactly), with their crop-relative
    affines."""
    import numpy as np
    rng = np.random.default_rng(seed)
    jobs = []
    H = stack_cpu.shape[1]
    m = 4
    for s in range(min(n_sample_sections, stack_cpu.shape[0])):
        for w in rng.choice(len(centres), per_section, replace=False):
            cx, cy = centres[w]
            x0, y0 = int(max(cx - N // 2 - m, 0)), int(max(cy - N // 2 - m, 0))
            x1, y1 = int(min(cx + N // 2 + m, H)), int(min(cy + N // 2 + m, H))
            th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
            jobs.append((stack_cpu[s, y0:y1, x0:x1].copy(), refs_cpu[s, y0:y1, x0:x1].copy(), th, th, N, P_WHITEN))
    return jobs


def _pool_time(worker, jobs, cores):
    import multiprocessing as mp
    chunks = [jobs[i::cores] for i in range(cores)]
    ctx = mp.get_context("spawn")
    env_keep = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with ctx.Pool(cores) as pool:
            pool.map(worker, [c[:1] for c in chunks])  # warm the workers (imports)
            t0 = time.perf_counter()
            res = pool.map(worker, chunks)
            wall = time.perf_counter() - t0
    finally:
        if env_keep is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_keep
    return wall, sum(r[1] for r in res)


def cpu_fp32_baseline(stack_cpu, refs_cpu, centres, n_sample_sections=64, per_section=16):
    """The same pairs through the CPU FP32 implementation (SciPy pocketfft in
    single precision, one process per core): the fast CPU reference point."""
    cores, aff, logical = host_cores()
    jobs = _sample_jobs(stack_cpu, refs_cpu, centres, n_sample_sections, per_section, seed=1)
    wall, cpu_s = _pool_time(_fp32_worker, jobs, cores)
    return dict(value=len(jobs) / wall, unit="pairs/s", cores=cores, kind="scipy_fp32",
                sample="%d pairs of %d^2 of the benchmark batch, FP32 SciPy pocketfft, one process per core; "
                       "%.1f s of CPU work" % (len(jobs), N, cpu_s), cpu_seconds=cpu_s)


def cpu_baseline(stack_cpu, refs_cpu, centres, n_sample_sections=64, per_section=8):
    """Times the FP64 oracle (one process per core) on a bounded sample of the
    same pairs."""
    cores, aff, logical = host_cores()
    jobs = _sample_jobs(stack_cpu, refs_cpu, centres, n_sample_sections, per_section, seed=0)
    wall, cpu_s = _pool_time(_oracle_worker, jobs, cores)
    return dict(value=len(jobs) / wall, unit="pairs/s", cores=cores, kind="oracle",
                sample="%d pairs of %d^2 (%d sections x %d windows) of the benchmark batch, FP64 NumPy, "
                       "one process per core; %.1f s of CPU work" % (len(jobs), N, n_sample_sections,
                                                                     per_section, cpu_s),
                cpu_seconds=cpu_s, mpx_per_s_per_core=len(jobs) * N * N / cpu_s / 1e6,
                host={"cores_allowed": aff, "logical_cpus": logical,
                      "note": "every allowed core up to 16, the host share of one GPU"})


# --------------------------------------------------------------------------- refinement comparison
def refine_comparison(ctx, sw, stack, cen, dev, tol=0.005, target=0.01, seed=9, max_shift=0):
    """Plain (centroid) vs batched + adjoint (Newton on the centroid) window
    refinement to a known sub-pixel truth, over the benchmark's 4096 window
    positions: window B samples section s at a fractional translation t*
    (U(-0.5, 0.5)^2), window A samples the same section starting U(-0.5,
    0.5)^2 px away from t*, so the aligned translation of A is exactly t*
    (bilinear sampling on both sides).  Both drivers stop when the longest
    step of the batch is below `tol` px.  Reports wall time, iterations, the
    final RMS / max error, and the iteration and time at which the RMS error
    first reaches `target`.  max_shift > 0 runs every match of both drivers
    with the pruned inverse (peak searched within that radius; the
    refinement's shifts stay below a pixel)."""
    import numpy as np
    import torch

    from paper_1612_04787_amd.refine import refine_adjoint, refine_plain
    S = stack.shape[0]
    rng = np.random.default_rng(seed)
    P = S * len(cen)
    tb = np.zeros((P, 8), np.float32)
    k = 0
    for s in range(S):
        for (cx, cy) in cen:
            tb[k] = [cx, cy, 1, 0, rng.uniform(-0.5, 0.5), 0, 1, rng.uniform(-0.5, 0.5)]
            k += 1
    ta = tb.copy()
    ta[:, 4] += rng.uniform(-0.5, 0.5, P).astype(np.float32)
    ta[:, 7] += rng.uniform(-0.5, 0.5, P).astype(np.float32)
    images = [stack[s] for s in range(S)]
    idx = torch.arange(S, device=dev, dtype=torch.int32).repeat_interleave(len(cen))
    tha, thb = torch.from_numpy(ta).to(dev), torch.from_numpy(tb).to(dev)
    truth = thb[:, [4, 7]].clone()
    params = sw.make_params(p=P_WHITEN, max_shift=max_shift)
    n_list = [N] * P

    def rms_max(th):
        e = (th[:, [4, 7]] - truth).norm(dim=1)
        return float(e.pow(2).mean().sqrt()), float(e.max())

    out = {}
    for name, fn, cap in (("plain", refine_plain, 80), ("adjoint", refine_adjoint, 20)):
        fn(ctx, images, n_list, idx, idx, tha, thb, params, tol=tol, max_iter=2)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th, iters, _ = fn(ctx, images, n_list, idx, idx, tha, thb, params, tol=tol, max_iter=cap)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r, mx = rms_max(th)
        # the first iteration count whose RMS error reaches the target, and the
        # wall time of a run of exactly that many iterations (iterations differ
        # in cost: the adjoint driver starts with centroid steps)
        hit, hit_ms = None, None
        for it in range(1, iters + 1):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            thi, _, _ = fn(ctx, images, n_list, idx, idx, tha, thb, params, tol=0.0, max_iter=it)
            torch.cuda.synchronize()
            t_it = time.perf_counter() - t1
            if rms_max(thi)[0] <= target:
                hit, hit_ms = it, t_it * 1e3
                break
        out[name] = dict(iterations=iters, wall_ms=wall * 1e3, rms_px=r, max_px=mx,
                         iters_to_target=hit, ms_to_target=hit_ms, windows_per_s=P / wall)
    r0 = rms_max(tha)[0]
    return dict(note="adjoint: centroid steps until the longest step is below the 0.5 px clamp, then Newton steps on the "
                     "centroid shift with the Jacobian (translation columns) from one adjoint pass per iteration",
                workload="%d windows of %d^2 (the benchmark's window grid), truth = fractional translation of "
                         "window B, start U(-0.5, 0.5)^2 px away" % (P, N),
                search_radius_px=max_shift, start_rms_px=r0, tol_px=tol, target_rms_px=target, **out)


# --------------------------------------------------------------------------- ragged levels
def config3_images(ctx, dev, sections=32, size=8192):
    """The multi-level input: a 32 x 8192^2 stack, its x2 pyramid (4 levels)
    and the +-3 projections of every level.  Image table layout: level l's
    sections at 2 S l + s, their references at 2 S l + S + s."""
    from datagen.workloads import level_stack
    from paper_1612_04787_amd.stack import build_pyramid
    stack = level_stack(sections, size, seed=3, device=dev)
    pyr = build_pyramid(ctx, stack, 3)
    images = []
    for lv in pyr:
        ref = ctx.project(lv, k=K_PROJ)
        images += [lv[s] for s in range(sections)] + [ref[s] for s in range(sections)]
    return images


def ragged_levels(ctx, sw, dev, images, sections=32, size=8192, reps=20):
    """Every pyramid level of a 32 x 8192^2 stack at once: 8 x 8 windows per
    section and level (1024^2 at level 0 down to 128^2 at level 3), 8192
    pairs against +-3 projections of each level.  Compares four plain calls
    (one per level, in sequence) with one call for the whole ragged batch
    (size groups concurrent) and with the same batch as one replayed hipGraph.
    Median of `reps` runs each."""
    import torch

    from datagen.workloads import ragged_level_pairs
    n_list, ia, ib, ta, tb = ragged_level_pairs(sections, size, 4, 8, dev)
    P = len(n_list)
    params = sw.make_params(p=P_WHITEN, flags=sw.FLAG_CONCURRENT_SIZES)
    params_seq = sw.make_params(p=P_WHITEN)
    prep = ctx.prepare(images, n_list, ia, ib, ta, tb)
    need, _ = ctx.workspace_size(prep["pairs"], params)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev)
    # per-level descriptors over the same arrays (pairs are sorted by size)
    levels = []
    off = 0
    for n in sorted(set(n_list)):
        c = n_list.count(n)
        sl = slice(off, off + c)
        pr = ctx.make_pairs(n_list[sl], prep["keep"][0][sl], prep["keep"][1][sl], prep["keep"][2][sl],
                            prep["keep"][3][sl])
        levels.append((pr, out[sl]))
        off += c

    def per_level():
        for pr, o in levels:
            ctx.match_batch_raw(prep["table"], len(images), pr, params_seq, o, ws=ws)

    def one_call():
        ctx.match_batch_raw(prep["table"], len(images), prep["pairs"], params, out, ws=ws)

    def graph():
        ctx.match_batch_raw(prep["table"], len(images), prep["pairs"], params, out, ws=ws, graph=True)

    # per-size kernel time of the sequential calls (HIP events on the launch
    # stream) against each size's bound: the FP32 vector ALUs for 64 / 128
    # (the one-workgroup kernel keeps spectra in LDS), HBM for >= 256
    per_level()
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(5):
        per_level()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    sizes = {}
    for name, (cnt, tot) in prof.items():
        nn = int(name.split("<")[1].rstrip(">")) if "<" in name else 0
        if nn:
            d = sizes.setdefault(nn, dict(kernels={}, ms=0.0))
            d["kernels"][name] = tot / 5
            d["ms"] += tot / 5
    for nn, d in sizes.items():
        cnt = n_list.count(nn)
        d["pairs"] = cnt
        d["pairs_per_s"] = cnt / (d["ms"] / 1e3)
        d["plan"] = dict(zip(("fwd_rows", "inv_rows", "chunks"), ctx.plan(nn, full=True)))
        if nn <= 128:
            tf = cnt * pair_flops(nn) / (d["ms"] / 1e3) / 1e12
            d["roofline"] = dict(bound="alu", achieved=tf, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                 frac=tf / FP32_PEAK_TFLOPS)
        else:
            gbs = cnt * pair_bytes(nn) / (d["ms"] / 1e3) / 1e9
            d["roofline"] = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS)

    res = {"per_size": {str(k): v for k, v in sorted(sizes.items())}}
    for name, fn in (("per_level_calls", per_level), ("one_call_concurrent", one_call), ("graph", graph)):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        times.sort()
        med = times[len(times) // 2]
        res[name] = dict(ms=med * 1e3, pairs_per_s=P / med)
    r = sw.parse_records(out)
    res["workload"] = ("%d sections of %d^2, 4 pyramid levels, 8x8 windows per level: %s pairs of 128/256/512/1024"
                       % (sections, size, "/".join(str(n_list.count(n)) for n in sorted(set(n_list)))))
    res["median_snr"] = float(r["snr"].float().median())
    res["graph_speedup_vs_per_level"] = res["per_level_calls"]["ms"] / res["graph"]["ms"]

    # The same levels with a small batch (the first `k` windows of every size):
    # four per-level calls are then bound by their launches and host calls,
    # which one replayed graph of the whole ragged batch removes.
    k = 16
    sel, off = [], 0
    for n in sorted(set(n_list)):
        sel.extend(range(off, off + k))
        off += n_list.count(n)
    idx = torch.tensor(sel, device=dev)
    keep = [prep["keep"][i][idx].contiguous() for i in range(4)]  # alive while the descriptors are used
    n_small = [n_list[i] for i in sel]
    small_pairs = ctx.make_pairs(n_small, *keep)
    small_levels, off = [], 0
    for n in sorted(set(n_small)):
        sl = slice(off, off + k)
        small_levels.append((ctx.make_pairs(n_small[sl], keep[0][sl], keep[1][sl], keep[2][sl], keep[3][sl]),
                             out[sl]))
        off += k

    def small_per_level():
        for pr, o in small_levels:
            ctx.match_batch_raw(prep["table"], len(images), pr, params_seq, o, ws=ws)

    def small_graph():
        ctx.match_batch_raw(prep["table"], len(images), small_pairs, params, out[:len(sel)], ws=ws, graph=True)

    small = {}
    for name, fn in (("per_level_calls", small_per_level), ("graph", small_graph)):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(5 * reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        times.sort()
        med = times[len(times) // 2]
        small[name] = dict(ms=med * 1e3, pairs_per_s=len(sel) / med)
    small["workload"] = "%d pairs of each of 128/256/512/1024 from the same levels" % k
    small["graph_speedup_vs_per_level"] = small["per_level_calls"]["ms"] / small["graph"]["ms"]
    res["small_batch"] = small
    return res


# --------------------------------------------------------------------------- config 2: 1024^2 windows
def config2_block(ctx, sw, dev, reps=20):
    """A 16384^2 section pair (B = bilinear affine warp of A about the centre,
    rotation <= 0.5 deg, scale 1 +- 0.002, shift <= 40 px, plus noise sigma 8)
    and a 16 x 16 grid of 1024^2 windows at identity affines: 256 pairs,
    p = 0.65.  Median of `reps` replays of the batch as one hipGraph, the
    per-kernel HIP-event timing with the HBM roofline of the longest kernel,
    the whole-path roofline, and the shifts against the generator's warp at
    the window centres."""
    import numpy as np
    import torch

    from datagen.workloads import section_pair_1024
    n = 1024
    a, b, m, bv, n_list, ia, ib, ta, tb = section_pair_1024(16384, dev)
    P = len(n_list)
    prep = ctx.prepare([a, b], n_list, ia, ib, ta, tb)
    params = sw.make_params(p=P_WHITEN)
    need, _ = ctx.workspace_size(prep["pairs"], params)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev)
    ms = median_event_ms(lambda: ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, out, None, ws,
                                                     graph=True), reps)
    ctx.profile(True)
    with one_chunk(ctx, [n]):
        for _ in range(5):
            ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, out, None, ws)
        torch.cuda.synchronize()
    kernels, roof = variant_kernels(ctx.profile_read(), n, P, n, False, traffic_file=CONFIG2_TRAFFIC_FILE, steps=5)
    ctx.profile(False)
    r = sw.parse_records(out)
    # B(q) = A(M q + b): window B's content at centre q sits at M q + b in A,
    # so the match shift is q - (M q + b)
    cen = ta[:, :2].double().cpu().numpy()
    mm, bb = np.asarray(m, np.float64), np.asarray(bv, np.float64)
    expect = cen - (cen @ mm.T + bb)
    got = np.stack([r["dx"].double().cpu().numpy(), r["dy"].double().cpu().numpy()], 1)
    err = np.linalg.norm(got - expect, axis=1)
    rate = P / (ms / 1e3)
    del ws, a, b
    return dict(workload="256 pairs of 1024^2: 16 x 16 windows of a 16384^2 uint8 section pair (B = bilinear affine "
                         "warp of A plus noise), identity affines, p = 0.65",
                replays=reps, median_ms=ms, pairs_per_s=rate, kernels=kernels, roofline=roof,
                path_roofline=path_roofline(rate, n), hbm_floor_ms=P * pair_bytes(n) / (HBM_PEAK_GBS * 1e9) * 1e3,
                shift_error_px={"median": float(np.median(err)), "p90": float(np.quantile(err, 0.9)),
                                "max": float(err.max()),
                                "note": "against the warp's displacement at the window centre; the warp's rotation "
                                        "moves the window's far corners up to ~4 px more, so this is not the "
                                        "sub-pixel parity bound"},
                median_snr=float(r["snr"].median()))


# --------------------------------------------------------------------------- per-size rooflines
def size_rooflines(ctx, sw, dev, pairs_per_size=2048, reps=20):
    """Each window size alone, as in the multi-level workload (2048 pairs per
    size): windows on a regular grid over an 8192^2 section pair (B = bilinear
    affine warp of A plus noise), identity affines, p = 0.65, the plan the
    tuner chose.  Median of `reps` graph replays per size, per-kernel HIP-event
    timing, and the size's bound: the FP32 vector ALUs for n <= 128 (the
    one-workgroup kernel keeps the spectra in LDS; 7.5 n^2 log2 n^2 + 40 n^2
    flop per pair), HBM for n >= 256 (inputs, record and one write + read of
    each exchanged spectrum per pair)."""
    import numpy as np
    import torch

    from datagen import make_section_pair
    a, b, _, _ = make_section_pair(8192, 8192, 3, 303, device=dev)
    out_all = {}
    for n in sw.SIZES:
        g = int(np.ceil(np.sqrt(pairs_per_size)))
        xs = np.linspace(n / 2 + 2, 8192 - n / 2 - 2, g)
        cx, cy = np.meshgrid(xs, xs)
        th = np.zeros((g * g, 8), np.float32)
        th[:, 0], th[:, 1], th[:, 2], th[:, 6] = cx.ravel(), cy.ravel(), 1, 1
        th = th[:pairs_per_size]
        P = th.shape[0]
        t = torch.from_numpy(th).to(dev)
        z = torch.zeros(P, dtype=torch.int32, device=dev)
        prep = ctx.prepare([a, b], [n] * P, z, z + 1, t, t.clone())
        params = sw.make_params(p=P_WHITEN)
        need, _ = ctx.workspace_size(prep["pairs"], params)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev)
        ms = median_event_ms(lambda: ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, out, None, ws,
                                                         graph=True), reps)
        ctx.profile(True)
        with one_chunk(ctx, [n]):
            for _ in range(5):
                ctx.match_batch_raw(prep["table"], 2, prep["pairs"], params, out, None, ws)
            torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        d = dict(pairs=P, median_ms=ms, pairs_per_s=P / (ms / 1e3),
                 kernels_one_chunk_ms={k: v[1] / v[0] for k, v in prof.items()},
                 plan=dict(zip(("fwd_rows", "inv_rows", "chunks"), ctx.plan(n, full=True))))
        if n <= 128:
            tf = P * pair_flops(n) / (ms / 1e3) / 1e12
            d["roofline"] = dict(bound="alu", achieved=tf, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                 frac=tf / FP32_PEAK_TFLOPS, flop_per_pair=pair_flops(n))
        else:
            gbs = P * pair_bytes(n) / (ms / 1e3) / 1e9
            d["roofline"] = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                                 bytes_per_pair=pair_bytes(n))
        out_all[str(n)] = d
        del ws
    return out_all


# --------------------------------------------------------------------------- refinement on the ragged levels
def refine_levels(ctx, sw, dev, images, sections=32, size=8192, tol=0.005, target=0.01, seed=9, max_plain=80,
                  max_adjoint=20):
    """Refinement of the 8192 ragged windows of the multi-level input to a
    known sub-pixel truth: window B samples its level image at a fractional
    translation t* (U(-0.5, 0.5)^2), window A the same image starting
    U(-0.5, 0.5)^2 px away from t*, so A's aligned translation is t*.
      plain    per iteration one call per level (four sizes in sequence) and
               a centroid update per level; the host reads the longest step.
      batched+adjoint  per iteration one replayed graph of the whole ragged
               batch (match, centroid Jacobian on Newton iterations, update,
               the steps copied to pinned host memory); centroid steps until
               the longest is below 0.25 px, then Newton steps.
    Both stop when the longest step is below `tol`.  Reports wall time,
    iterations, final RMS / max error, and the iteration and wall time at
    which the RMS error over all windows first reaches `target` (from theta
    recorded after every iteration), with windows/s to that point."""
    import numpy as np
    import torch

    from datagen.workloads import ragged_level_pairs
    from paper_1612_04787_amd.refine import CENTROID, refine_adjoint_graph
    n_list, ia, _, _, tb = ragged_level_pairs(sections, size, 4, 8, dev)
    P = len(n_list)
    rng = np.random.default_rng(seed)
    tbn = tb.cpu().numpy().copy()
    tbn[:, 4] = rng.uniform(-0.5, 0.5, P)
    tbn[:, 7] = rng.uniform(-0.5, 0.5, P)
    tan = tbn.copy()
    tan[:, 4] += rng.uniform(-0.5, 0.5, P)
    tan[:, 7] += rng.uniform(-0.5, 0.5, P)
    tha0 = torch.from_numpy(tan.astype(np.float32)).to(dev)
    thb = torch.from_numpy(tbn.astype(np.float32)).to(dev)
    truth = thb[:, [4, 7]].clone()
    ib = ia.clone()  # both windows on the same level image

    def rms_of(trace_rows):
        e = (trace_rows[..., [4, 7]] - truth).norm(dim=-1)
        return e.pow(2).mean(-1).sqrt().cpu().numpy(), e.max(-1).values.cpu().numpy()

    res = {}
    # plain: one call per level per iteration
    params = sw.make_params(p=P_WHITEN)
    prep = ctx.prepare(images, n_list, ia, ib, tha0.clone(), thb)
    th = prep["keep"][2]
    need, _ = ctx.workspace_size(prep["pairs"], params)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev)
    step = torch.empty(P, dtype=torch.float32, device=dev)
    lv = []
    off = 0
    for n in sorted(set(n_list)):
        c = n_list.count(n)
        sl = slice(off, off + c)
        lv.append((sl, ctx.make_pairs(n_list[sl], prep["keep"][0][sl], prep["keep"][1][sl], th[sl],
                                      prep["keep"][3][sl])))
        off += c

    def plain_iter():
        for sl, pr in lv:
            ctx.match_batch_raw(prep["table"], len(images), pr, params, out[sl], ws=ws)
            ctx.refine_update(out[sl], th[sl], CENTROID, None, 0.5, step[sl])

    plain_iter()  # warm-up
    torch.cuda.synchronize()
    th.copy_(tha0)
    trace = torch.empty((max_plain, P, 8), dtype=torch.float32, device=dev)
    times = []
    t0 = time.perf_counter()
    iters = max_plain
    for it in range(1, max_plain + 1):
        plain_iter()
        trace[it - 1].copy_(th)
        m = float(step.max())
        times.append(time.perf_counter() - t0)
        if m < tol:
            iters = it
            break
    rms, mx = rms_of(trace[:iters])
    res["plain"] = _refine_summary(P, iters, times, rms, mx, target)
    del trace, ws
    # batched + adjoint: one replayed graph of the ragged batch per iteration
    pc = sw.make_params(p=P_WHITEN, flags=sw.FLAG_CONCURRENT_SIZES)
    trace = torch.empty((max_adjoint, P, 8), dtype=torch.float32, device=dev)
    _, iters, hist, times = refine_adjoint_graph(ctx, images, n_list, ia, ib, tha0, thb, pc, tol=tol,
                                                 max_iter=max_adjoint, theta_trace=trace)
    rms, mx = rms_of(trace[:iters])
    res["batched_adjoint"] = _refine_summary(P, iters, times, rms, mx, target)
    del trace
    res["iteration_kernels"] = iteration_kernels(ctx, sw, images, n_list, ia, ib, tha0, thb, pc)
    res["workload"] = ("%d windows of the multi-level input (2048 each of 128/256/512/1024), truth = fractional "
                       "translation of window B, start U(-0.5, 0.5)^2 px away" % P)
    r0 = float((tha0[:, [4, 7]] - truth).norm(dim=1).pow(2).mean().sqrt())
    res.update(start_rms_px=r0, tol_px=tol, target_rms_px=target)
    a, b = res["plain"], res["batched_adjoint"]
    if a["ms_to_target"] and b["ms_to_target"]:
        res["speedup_to_target"] = a["ms_to_target"] / b["ms_to_target"]
    return res


def iteration_kernels(ctx, sw, images, n_list, ia, ib, tha, thb, params, reps=5):
    """Per-kernel HIP-event times (ms per iteration, mean of `reps` eager
    runs on the launch stream) of the two iterations of the adjoint driver
    over the whole batch: the centroid iteration's match, and the Newton
    iteration's match with saved state plus the centroid-Jacobian pass."""
    import torch
    jp = sw.make_params(params.p, params.eps_rel, params.taper_frac, params.centroid_r,
                        params.flags | sw.FLAG_JAC_TRANSLATION, params.max_shift)
    plain = sw.make_params(params.p, params.eps_rel, params.taper_frac, params.centroid_r, 0, params.max_shift)
    prep = ctx.prepare(images, n_list, ia, ib, tha.clone(), thb)
    P = prep["pairs"].n_pairs
    need, sv = ctx.workspace_size(prep["pairs"], plain)
    ws = torch.empty(need, dtype=torch.uint8, device=ctx.device)
    saved = torch.empty(sv, dtype=torch.uint8, device=ctx.device)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=ctx.device)
    jac = torch.empty((P, 2, 6), dtype=torch.float32, device=ctx.device)
    calls = {
        "match": lambda: ctx.match_batch_raw(prep["table"], len(images), prep["pairs"], plain, out, ws=ws),
        "match_saved": lambda: ctx.match_batch_raw(prep["table"], len(images), prep["pairs"], plain, out,
                                                   saved=saved, ws=ws),
        "jacobian": lambda: ctx.centroid_jacobian_raw(prep["table"], len(images), prep["pairs"], jp, saved, jac,
                                                      ws=ws),
    }
    res = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        ks = {k: round(v[1] / reps, 4) for k, v in sorted(prof.items(), key=lambda x: -x[1][1])}
        res[name] = {"ms": round(sum(ks.values()), 3), "kernels": ks}
    res["centroid_iteration_ms"] = res["match"]["ms"]
    res["newton_iteration_ms"] = round(res["match_saved"]["ms"] + res["jacobian"]["ms"], 3)
    res["note"] = ("kernel times only, size groups in sequence; the refinement's graphs run the groups "
                   "concurrently and add the update and the step copy")
    del ws, saved
    return res


def refine_generator_bias(ctx, sw, dev, size=2048, n=512, seed=21,
                          shifts=((0.31, -0.22), (-0.44, 0.17), (0.12, 0.41), (-0.27, -0.36))):
    """Sensitivity of the refinement's fixed point to how the sub-pixel truth
    is generated: image B is image A (a 2048^2 section) moved by a fractional
    shift d, B(q) = A(q - d), resampled by SciPy as a cubic B-spline
    (ndimage.shift, order 3) or bilinearly (order 1, the gather's own
    convention), both kept in FP32.  A 3 x 3 grid of 512^2 windows per shift
    and generator, window B at identity, window A starting U(-0.5, 0.5)^2 px
    from its aligned translation -d; the adjoint driver runs until its longest
    step is below 1e-4 px.  Reports the converged error |t + d| per generator."""
    import numpy as np
    import torch
    from scipy import ndimage

    from datagen import make_section
    from paper_1612_04787_amd.refine import refine_adjoint
    a = make_section(size, size, seed).numpy().astype(np.float64)
    images = [torch.from_numpy(a.astype(np.float32)).to(dev)]
    rng = np.random.default_rng(seed)
    cs = [size / 2 - 600, size / 2, size / 2 + 600]
    ta, tb, ia, ib, gen, dd = [], [], [], [], [], []
    for (dx, dy) in shifts:
        for order in (3, 1):
            b = ndimage.shift(a, (dy, dx), order=order, mode="nearest")
            images.append(torch.from_numpy(b.astype(np.float32)).to(dev))
            for cy in cs:
                for cx in cs:
                    tb.append([cx, cy, 1, 0, 0, 0, 1, 0])
                    ta.append([cx, cy, 1, 0, -dx + rng.uniform(-0.5, 0.5), 0, 1, -dy + rng.uniform(-0.5, 0.5)])
                    ia.append(0)
                    ib.append(len(images) - 1)
                    gen.append(order)
                    dd.append((dx, dy))
    P = len(ta)
    tha = torch.tensor(ta, dtype=torch.float32, device=dev)
    thb = torch.tensor(tb, dtype=torch.float32, device=dev)
    ia_t = torch.tensor(ia, dtype=torch.int32, device=dev)
    ib_t = torch.tensor(ib, dtype=torch.int32, device=dev)
    th, iters, _ = refine_adjoint(ctx, images, [n] * P, ia_t, ib_t, tha, thb, sw.make_params(p=P_WHITEN),
                                  tol=1e-4, max_iter=30)
    t = th[:, [4, 7]].double().cpu().numpy()
    err = np.linalg.norm(t + np.asarray(dd, np.float64), axis=1)
    gen = np.asarray(gen)
    out = {}
    for order, name in ((3, "cubic"), (1, "bilinear")):
        e = err[gen == order]
        out[name] = dict(mean_px=float(e.mean()), max_px=float(e.max()), windows=int(e.size))
    return dict(workload="%d windows of %d^2 on a %d^2 section moved by %d fractional shifts, p = %.2f"
                         % (P, n, size, len(shifts), P_WHITEN), iterations=iters, **out)


def _refine_summary(P, iters, times, rms, mx, target):
    hit = next((i for i in range(iters) if rms[i] <= target), None)
    ms_hit = times[hit] * 1e3 if hit is not None else None
    return dict(iterations=iters, wall_ms=times[iters - 1] * 1e3, rms_px=float(rms[iters - 1]),
                max_px=float(mx[iters - 1]), rms_by_iteration=[float(v) for v in rms],
                iters_to_target=(hit + 1) if hit is not None else None, ms_to_target=ms_hit,
                windows_per_s_to_target=(P / (ms_hit / 1e3)) if ms_hit else None)


# --------------------------------------------------------------------------- stack loop
def stack_loop(ctx, stack, warps, refine="adjoint"):
    """The iterative stack alignment on the benchmark stack: passes at pyramid
    levels 2, 1, 0 (4, 2 and 1 of them) with 8 x 8 windows of 128^2, 256^2,
    512^2 per section (render, project over +-8 / +-4 / +-3 sections, match +
    refine, per-section affine fit).
    Residuals against the generator's section warps: RMS about the best global
    affine (gauge removed) and between neighbouring sections."""
    import numpy as np
    import torch

    from datagen.evaluate import residuals
    from paper_1612_04787_amd.stack import align_stack
    S, H, W = stack.shape
    pts = np.array([(W // 16 + W // 8 * i, H // 16 + H // 8 * j) for j in range(8) for i in range(8)], np.float64)
    g0, n0 = residuals(np.tile([1.0, 0, 0, 0, 1.0, 0], (S, 1)), warps, pts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    aff, rep = align_stack(ctx, stack, levels=(2, 1, 0), ns=(128, 256, 512), iters=(4, 2, 1), ks=(8, 4, 3),
                           refine=refine)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g1, n1 = residuals(aff.cpu().numpy(), warps, pts)
    return dict(workload="%d sections of %d^2: levels 2/1/0 x 4/2/1 passes, 8x8 windows of 128/256/512, "
                         "models +-8/+-4/+-3, refine=%s" % (S, H, refine),
                wall_ms=wall * 1e3, passes=rep, residual_px={"global_before": g0, "global_after": g1,
                                                             "neighbour_before": n0, "neighbour_after": n1})


# --------------------------------------------------------------------------- Pearson-normalised correlation
def pearson_block(ctx, sw, stack, refs, table, images, pairs, res_w, args, prof_steps):
    """The headline batch scored by Pearson-normalised correlation (the
    central 256^2 template of each raw window against every placement within
    +-128 px in the model window; FFT correlation plus the cumulative-area
    correction).  Timed like the headline step (projection included); match
    quality set against the whitened records of the same pairs."""
    import torch
    P = pairs.n_pairs
    prm = sw.make_params(flags=sw.FLAG_PEARSON)
    need, _ = ctx.workspace_size(pairs, prm)
    ws = ctx.workspace(need)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=stack.device)

    def step():
        ctx.project(stack, k=K_PROJ, out=refs)
        ctx.match_batch_raw(table, len(images), pairs, prm, out, None, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.profile(True)
    with one_chunk(ctx, [N]):
        for _ in range(prof_steps):
            step()
        torch.cuda.synchronize()
    rows = kept_rows(N, N // 4, ctx.plan(N)[1])
    kp, roof = variant_kernels(ctx.profile_read(), N, P, rows, True,
                               os.path.join(ROOT, "profiles", "hbm_traffic_match_512_pearson.txt"), steps=prof_steps)
    ctx.profile(False)
    r = sw.parse_records(out)
    same = (r["ix"] == res_w["ix"]) & (r["iy"] == res_w["iy"])
    dd = torch.maximum((r["dx"] - res_w["dx"]).abs(), (r["dy"] - res_w["dy"]).abs())
    del ws
    # single-shot shifts of both scores sit near whole pixels (3 x 3 centroid),
    # so they are compared within one pixel; the SNR is the paper's comparison
    return dict(template_px=N // 2, range_px=N // 4, ms_per_step=ms, pairs_per_s=P / (ms / 1e3),
                workspace_gb=need / 1e9, kernels=kp, roofline=roof, same_peak_frac=float(same.float().mean()),
                frac_shift_within_1px=float((dd <= 1.0).float().mean()),
                median_abs_shift_diff_px=float(dd.median()), median_peak_coefficient=float(r["peak"].median()),
                median_snr=float(r["snr"].median()), median_snr_whitened=float(res_w["snr"].median()))


# --------------------------------------------------------------------------- local-affine mesh
MESH_SECTIONS, MESH_GRID, MESH_N, MESH_BEND = 16, 16, 256, 3.0
# FP64 operations per rendered pixel in the render definition (contraction
# off, so no FMA): level -> base 4, affine 8, base -> level 4, floor and
# fraction 4, bilinear weights and blend 11, rounding and clamp 4.
RENDER_FP64_OPS = 35
# non-FMA FP64 vector rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
FP64_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def mesh_block(ctx, dev, sections=MESH_SECTIONS, size=SIZE, grid=MESH_GRID, n=MESH_N, reps=10):
    """Local-affine triangle mesh (mir, Section IV) on a stack with nonlinear
    section warps: global affines first (levels 2/1/0), then two mesh passes
    at level 0 (grid x grid nodes at the window centres, n^2 windows).
    Residuals against the generator's warps at the triangle centroids; the
    mesh render timed per launch with HIP events over the whole stack."""
    import torch

    from datagen.evaluate import mesh_centroids, residuals
    from datagen.workloads import bent_stack
    from paper_1612_04787_amd.stack import align_mesh, align_stack, build_pyramid
    stack, warps = bent_stack(sections, size, seed=11, bend=MESH_BEND, device=dev)
    pyr = build_pyramid(ctx, stack, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    aff, _ = align_stack(ctx, stack, levels=(2, 1, 0), ns=(128, 256, 512), iters=(2, 1, 1), ks=(4, 3, 3), grid=8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tri, mrep = align_mesh(ctx, stack, aff, level=0, n=n, grid=grid, k=3, passes=2, pyr=pyr)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cen = mesh_centroids(grid, size, size)
    g0, n0 = residuals(aff.cpu().numpy(), warps, cen)
    g1, n1 = residuals(tri.cpu().numpy(), warps, cen)
    out = torch.empty_like(stack)
    ctx.render_mesh(stack, tri, grid, 0, out=out)
    ctx.render(stack, aff, 0, out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        ctx.render_mesh(stack, tri, grid, 0, out=out)
        ctx.render(stack, aff, 0, out=out)
    prof = ctx.profile_read()
    ctx.profile(False)
    px = float(sections) * size * size

    def rate(name):
        cnt, tot = prof[name]
        ms = tot / cnt
        return dict(ms=ms, gpix_s=px / (ms / 1e3) / 1e9, hbm_gbs=2.0 * px / (ms / 1e3) / 1e9,
                    fp64_tops=RENDER_FP64_OPS * px / (ms / 1e3) / 1e12)

    rm, rg = rate("k_render_mesh<0>"), rate("k_render<0>")
    from paper_1612_04787_amd.counters import read_traffic, source_digest
    traffic, digest = read_traffic(os.path.join(ROOT, "profiles", "hbm_traffic_mesh_render_16x4096.txt"),
                                   "k_render_mesh")
    if digest != source_digest():
        traffic = None
    roof = {"bound": "alu", "achieved": rm["fp64_tops"], "peak": FP64_VALU_PEAK_TOPS, "unit": "TFLOP/s",
            "frac": rm["fp64_tops"] / FP64_VALU_PEAK_TOPS, "traffic": traffic}
    res = dict(workload="%d sections of %d^2 with drift, affine distortion and a smooth bend of up to %.0f px; "
                        "global affines (levels 2/1/0), then 2 mesh passes at level 0 with %d x %d nodes and "
                        "%d^2 windows" % (sections, size, MESH_BEND, grid, grid, n),
               affine_ms=(t1 - t0) * 1e3, mesh_ms=(t2 - t1) * 1e3, passes=mrep,
               residual_px={"neighbour_affine": n0, "neighbour_mesh": n1, "global_affine": g0, "global_mesh": g1},
               render_mesh=dict(rm, roofline=roof), render_affine=rg,
               note="render roofline: %d FP64 operations per pixel of the definition against the non-FMA FP64 "
                    "vector rate; HBM bytes 2 per pixel (uint8 in and out)" % RENDER_FP64_OPS)
    sample = (stack[0].cpu().numpy(), tri[0].cpu().numpy(), grid)
    del stack, pyr, out
    torch.cuda.empty_cache()
    return res, sample


def cpu_baseline_variants(stack_cpu, refs_cpu, centres, n_pruned=32):
    """The oracle on the pruned and Pearson variants of the benchmark pairs,
    one process: n_pruned pairs with the search radius (the oracle computes
    the whole surface either way), and one pair scored by Pearson
    coefficients at every placement (direct per-placement sums)."""
    import numpy as np

    import oracle as O
    rng = np.random.default_rng(3)
    H = stack_cpu.shape[1]
    m = 4
    crops = []
    for _ in range(n_pruned):
        s = int(rng.integers(0, stack_cpu.shape[0]))
        cx, cy = centres[int(rng.integers(0, len(centres)))]
        x0, y0 = int(max(cx - N // 2 - m, 0)), int(max(cy - N // 2 - m, 0))
        x1, y1 = int(min(cx + N // 2 + m, H)), int(min(cy + N // 2 + m, H))
        th = np.array([cx - x0, cy - y0, 1, 0, 0, 0, 1, 0], np.float64)
        crops.append((stack_cpu[s, y0:y1, x0:x1].copy(), refs_cpu[s, y0:y1, x0:x1].copy(), th))
    t0 = time.perf_counter()
    for (wa, wb, th) in crops:
        O.match_pair(wa, wb, th, th, N, O.Params(p=P_WHITEN, max_shift=PRUNE_R))
    tp = time.perf_counter() - t0
    wa, wb, th = crops[0]
    t0 = time.perf_counter()
    O.pearson_pair(wa, wb, th, th, N)
    tq = time.perf_counter() - t0
    return dict(pruned=dict(value=n_pruned / tp, unit="pairs/s", cores=1, kind="oracle",
                            sample="%d pairs of %d^2 of the benchmark batch, radius %d, FP64 NumPy, one process; "
                                   "%.1f s" % (n_pruned, N, PRUNE_R, tp)),
                pearson=dict(value=1.0 / tq, unit="pairs/s", cores=1, kind="oracle",
                             sample="1 pair of %d^2 of the benchmark batch, Pearson coefficient at each of the "
                                    "%d placements, FP64 NumPy, one process; %.1f s" % (N, (N // 2 + 1) ** 2, tq)))


def cpu_baseline_jump(sample):
    """The oracle's one-sided models (left and right, k = 3) of every section
    of a crop of the jump stack (the top eighth of each section), one
    process, in Mpixel/s of models."""
    import oracle as O
    S = sample.shape[0]
    t0 = time.perf_counter()
    for side in (-1, 1):
        for s in range(S):
            O.project_side(sample, s, 3, side)
    el = time.perf_counter() - t0
    px = 2.0 * S * sample.shape[1] * sample.shape[2]
    return dict(value=px / el / 1e6, unit="Mpixel/s", cores=1, kind="oracle",
                sample="left and right models (k = 3) of %d sections of %d x %d px, integer NumPy, one "
                       "process; %.1f s" % (S, sample.shape[1], sample.shape[2], el))


def cpu_baseline_mesh(sample, n_px=1 << 23):
    """The oracle's mesh render on a bounded sample of pixels of one section
    (one process, FP64 NumPy), in Mpixel/s."""
    import numpy as np

    import oracle as O
    img, tri, grid = sample
    H, W = img.shape
    rng = np.random.default_rng(1)
    xs = rng.integers(0, W, n_px)
    ys = rng.integers(0, H, n_px)
    t0 = time.perf_counter()
    O.render_mesh_at(img, tri, 0, grid, H, W, xs, ys)
    el = time.perf_counter() - t0
    return dict(value=n_px / el / 1e6, unit="Mpixel/s", cores=1, kind="oracle",
                sample="%d random pixels of one %d^2 section through its %d x %d mesh, FP64 NumPy; %.1f s"
                       % (n_px, H, grid, grid, el))


# --------------------------------------------------------------------------- jump repair
def jump_block(ctx, dev, sections=16, size=SIZE, j0=8, mag=0.02):
    """Jump repair (Section III, model paragraphs) on a stack with a
    magnification change: the section-affine loop (levels 2/1/0), then
    repair_jumps at level 0 (512^2 windows, 8 x 8 per section).  Residuals
    between neighbouring sections against the generator's warps, per pair."""
    import numpy as np
    import torch

    from datagen.evaluate import composed_points
    from datagen.workloads import jump_stack
    from paper_1612_04787_amd.stack import align_stack, build_pyramid, repair_jumps
    stack, warps = jump_stack(sections, size, seed=13, j0=j0, mag=mag, device=dev)
    pyr = build_pyramid(ctx, stack, 2)
    aff, _ = align_stack(ctx, stack, levels=(2, 1, 0), ns=(128, 256, 512), iters=(2, 1, 1), ks=(4, 3, 3), grid=8)
    pts = np.array([(size // 16 + size // 8 * i, size // 16 + size // 8 * j) for j in range(8) for i in range(8)],
                   np.float64)

    def pair_res(a):
        c = composed_points(a.cpu().numpy(), warps, pts)
        return np.sqrt(np.mean(np.sum((c[1:] - c[:-1]) ** 2, 2), 1))

    r0 = pair_res(aff)
    torch.cuda.synchronize()
    ctx.profile(True)
    aff2, rep = repair_jumps(ctx, stack, aff.clone(), level=0, n=512, grid=8, k=3, pyr=pyr)
    prof = ctx.profile_read()
    ctx.profile(False)
    r1 = pair_res(aff2)
    kernels = {}
    for name, (cnt, tot) in prof.items():
        kernels[name] = dict(launches=cnt, avg_ms=tot / cnt)
        if name.startswith("k_project"):  # every section read once, every model written once
            kernels[name]["gbs"] = 2.0 * sections * size * size / (tot / cnt / 1e3) / 1e9
    sample = stack[:, : size // 8].cpu().numpy()
    del stack, pyr
    torch.cuda.empty_cache()
    return dict(workload="%d sections of %d^2 with drift and section affines, magnification change of %.0f%% at "
                         "section %d; section-affine loop at levels 2/1/0, then repair at level 0 (512^2 windows)"
                         % (sections, size, 100 * mag, j0),
                breaks=rep["breaks"], spans=rep["spans"], repair_ms=rep["ms"], kernels=kernels,
                pair_residual_px={"max_before": float(r0.max()), "at_jump_before": float(r0[j0 - 1]),
                                  "max_after": float(r1.max()), "at_jump_after": float(r1[j0 - 1]),
                                  "median_after": float(np.median(r1))}), sample


# --------------------------------------------------------------------------- search with an SNR stop
def search_block(ctx, sw, dev, size=8192, n=256, grid=24, step=128.0, rings=2, accept=15.0, reps=3):
    """Search with an SNR stop (Section III, SNR paragraph) on a section pair
    misplaced by about a window edge and rotated 1 degree: 25 candidate
    offsets (spiral, n/2 apart), each window leaving at its first candidate
    with SNR >= 15, against the same driver searching every candidate.
    Found offsets against the generator's displacement."""
    import numpy as np
    import torch

    from datagen.workloads import search_pair
    from paper_1612_04787_amd.search import search_offsets, spiral_offsets
    a, b, m, bv, nl, ia, ib, ta, tb, cen = search_pair(size, n, grid, device=dev)
    radius = int(step // 2) + 4  # each candidate owns its cell of the spiral
    params = sw.make_params(p=0.65, max_shift=radius)
    offs = spiral_offsets(step, rings)
    P, K = len(nl), offs.shape[0]

    def run(acc, ahead=1):
        search_offsets(ctx, [a, b], nl, ia, ib, ta, tb, params, offs, accept=acc, lookahead=ahead)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            got = search_offsets(ctx, [a, b], nl, ia, ib, ta, tb, params, offs, accept=acc, lookahead=ahead)
        torch.cuda.synchronize()
        return got, (time.perf_counter() - t0) / reps * 1e3

    got, ms = run(accept)
    full, ms_full = run(float("inf"))
    ahead = {}
    for B in (2, 4):
        g2, ms2 = run(accept, B)
        same = bool(torch.equal(g2["best"], got["best"]) and torch.equal(g2["cand"], got["cand"]))
        ahead[str(B)] = dict(ms=ms2, matches=int(sum(g2["matched"])), same_result=same)
    ctx.profile(True)
    search_offsets(ctx, [a, b], nl, ia, ib, ta, tb, params, offs, accept=accept)
    prof = ctx.profile_read()
    ctx.profile(False)
    # launches shrink round by round, so each kernel is priced over the whole
    # search: algorithmic bytes of every match it ran over its total time
    m_prof = int(sum(got["matched"]))
    rows = kept_rows(n, radius, ctx.plan(n)[1])
    kernels = {}
    for name, (cnt, tot) in prof.items():
        byt = variant_bytes(name, n, m_prof, rows, False)
        kernels[name] = dict(launches=cnt, avg_ms=tot / cnt, total_ms=tot, bytes=byt, gbs=byt / (tot / 1e3) / 1e9)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    roof = dict(bound="hbm", kernel=dom, achieved=kernels[dom]["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=kernels[dom]["gbs"] / HBM_PEAK_GBS, traffic=None, matches=m_prof,
                total_ms=kernels[dom]["total_ms"])
    rec = sw.parse_records(got["best"])
    cand = got["cand"].cpu().numpy()
    done = got["done"].cpu().numpy().astype(bool)
    def found(g):
        r = sw.parse_records(g["best"])
        d = np.stack([r["dx"].cpu().numpy(), r["dy"].cpu().numpy()], 1)
        return offs.numpy().astype(np.float64)[g["cand"].cpu().numpy()] - d

    est = found(got)
    err = np.abs(est - (cen @ m.T + bv - cen)).max(1)
    agree = np.abs(est - found(full)).max(1) <= 1.0
    sample = (a.cpu().numpy(), b.cpu().numpy(), ta.cpu().numpy(), offs.numpy(), accept, radius)
    del a, b
    torch.cuda.empty_cache()
    return dict(workload="%d^2 section pair misplaced by (230, -150) px and rotated 1 degree; %d windows of %d^2, "
                         "%d candidate offsets %g px apart, each matched within radius %d (pruned inverse), stop at "
                         "SNR >= %g" % (size, P, n, K, step, radius, accept),
                ms=ms, windows_per_s=P / (ms / 1e3), matches=int(sum(got["matched"])),
                exhaustive=dict(ms=ms_full, matches=P * K), speedup=ms_full / ms,
                done_frac=float(done.mean()), max_err_px_done=float(err[done].max()) if done.any() else None,
                max_err_px_all=float(err.max()), same_offset_as_exhaustive=float(agree.mean()), lookahead=ahead,
                kernels=kernels, roofline=roof), sample


def search_stack_block(ctx, dev, sections=12, size=2048, j=6, move=(150.0, -110.0)):
    """The stack loop with and without a search in its first pass, on
    sections with drift and section affines where section j is moved a further
    `move` px (beyond a 64^2 window's capture at level 2).  Neighbour
    residuals against the generator's warps."""
    import numpy as np
    import torch

    from datagen.evaluate import composed_points
    from datagen.synth import make_stack
    from datagen.workloads import stack_warps
    from paper_1612_04787_amd.stack import align_stack
    warps = stack_warps(sections, size, size, 41)
    m, b = warps[j]
    warps[j] = (m, b + np.asarray(move))
    raw = make_stack(sections, size, size, 41, device=dev, warps=warps)
    pts = np.array([(size // 16 + size // 8 * i, size // 16 + size // 8 * k) for k in range(8) for i in range(8)],
                   np.float64)

    def pair_res(a):
        c = composed_points(a.cpu().numpy(), warps, pts)
        return np.sqrt(np.mean(np.sum((c[1:] - c[:-1]) ** 2, 2), 1))

    kw = dict(levels=(2, 1, 0), ns=(64, 128, 256), iters=(2, 1, 1), ks=(3, 3, 3))
    align_stack(ctx, raw, search=dict(rings=2, accept=15.0), **kw)  # warm-up (first calls at these sizes)
    out = {}
    for name, srch in (("with_search", dict(rings=2, accept=15.0)), ("with_search_lookahead4",
                                                                     dict(rings=2, accept=15.0, lookahead=4)),
                       ("without", None)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        aff, rep = align_stack(ctx, raw, search=srch, **kw)
        torch.cuda.synchronize()
        r = pair_res(aff)
        out[name] = dict(wall_ms=(time.perf_counter() - t0) * 1e3, search_matches=rep[0]["search_matches"],
                         first_pass_ms=rep[0]["ms"], max_pair_px=float(r.max()), at_section_px=float(r[j - 1]))
    del raw
    torch.cuda.empty_cache()
    out["workload"] = ("%d sections of %d^2 (drift, section affines), section %d moved a further (%g, %g) px; "
                       "levels 2/1/0 with 64/128/256 windows, 8 x 8 per section" % (sections, size, j, move[0], move[1]))
    return out


def cpu_baseline_search(sample, n=256, windows=range(0, 576, 16)):
    """The oracle's search (FP64 matches over the candidate list, stopping at
    the threshold) for a few windows of the search pair, one process, in
    windows/s."""
    import oracle as O
    a, b, ta, offs, accept, radius = sample
    t0 = time.perf_counter()
    matches = 0
    for w in windows:
        snrs = []
        for k in range(offs.shape[0]):
            th = ta[w].astype("float64").copy()
            th[4] += offs[k, 0]
            th[7] += offs[k, 1]
            snrs.append(O.match_pair(a, b, th, ta[w].astype("float64"), n, O.Params(p=0.65, max_shift=radius))["snr"])
            matches += 1
            if snrs[-1] >= accept:
                break
        O.search_select(snrs, accept)
    el = time.perf_counter() - t0
    return dict(value=len(windows) / el, unit="windows/s", cores=1, kind="oracle",
                sample="search of %d windows (%d FP64 matches of %d^2), one process; %.1f s"
                       % (len(windows), matches, n, el))


# --------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-refine", action="store_true", help="skip the plain vs adjoint refinement comparison")
    ap.add_argument("--no-stack", action="store_true", help="skip the iterative stack-alignment run")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the multi-level ragged batch comparison and the refinement on it")
    ap.add_argument("--ragged-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-sizes", action="store_true", help="skip the per-size roofline block")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default row-count plan (no tuning launches)")
    ap.add_argument("--no-mesh", action="store_true", help="skip the local-affine mesh run")
    ap.add_argument("--no-prune", action="store_true", help="skip the pruned-inverse (search radius) variant")
    ap.add_argument("--no-pearson", action="store_true", help="skip the Pearson-normalised correlation variant")
    ap.add_argument("--no-jump", action="store_true", help="skip the jump-repair run")
    ap.add_argument("--no-search", action="store_true", help="skip the SNR-stop search run")
    ap.add_argument("--no-config2", action="store_true", help="skip the 256 x 1024^2 section-pair batch")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration under a profiler)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    if args.ragged_child:
        ragged_main(args)
        return

    import torch

    import paper_1612_04787_amd as sw
    from datagen.workloads import distorted_stack, section_grid_pairs

    dev = torch.device("cuda", 0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.time()
    stack, warps = distorted_stack(S_SECTIONS, SIZE, seed=5, device=dev)
    torch.cuda.synchronize()
    log("workload: %d x %d^2 stack generated in %.1f s" % (S_SECTIONS, SIZE, time.time() - t0))

    ctx = sw.Swift(0)
    refs = torch.empty_like(stack)
    images = [stack[s] for s in range(S_SECTIONS)] + [refs[s] for s in range(S_SECTIONS)]
    table = ctx.image_table(images)
    n_list, ia, ib, ta, tb, cen = section_grid_pairs(S_SECTIONS, SIZE, N, GRID, dev)
    pairs = ctx.make_pairs(n_list, ia, ib, ta, tb)
    P = pairs.n_pairs
    params = sw.make_params(p=P_WHITEN)
    need, _ = ctx.workspace_size(pairs, params)
    ws = ctx.workspace(need)
    out = torch.empty((P, sw.swift.REC_BYTES), dtype=torch.uint8, device=dev)
    log("pairs: %d of %d^2, workspace %.2f GB" % (P, N, need / 1e9))
    # row-count variants chosen on the device (synthetic batch, untimed set-up)
    if args.no_autotune:
        tuned = {n: ([], ctx.plan(n, full=True)) for n in sw.SIZES}
    else:
        tuned = ctx.autotune(sw.SIZES, pairs_per_size=2048)
    log("plan: " + ", ".join("%d: (fwd rows, inv rows, chunks) %s" % (n, v[1]) for n, v in tuned.items()))

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB device-to-device")

    def step():
        ctx.project(stack, k=K_PROJ, out=refs)
        ctx.match_batch_raw(table, len(images), pairs, params, out, None, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / args.steps * 1e3
    value = P / (ms / 1e3)
    log("timed: %d steps, %.3f ms/step, %.0f pairs/s" % (args.steps, ms, value))

    # the same step with the match as one replayed hipGraph: each of 20
    # replays timed on its own (HIP events on the launch stream), median
    def step_graph():
        ctx.project(stack, k=K_PROJ, out=refs)
        ctx.match_batch_raw(table, len(images), pairs, params, out, None, ws, graph=True)

    graph_rep = median_event_ms(step_graph, 20)
    log("graph replays: median %.3f ms/step, %.0f pairs/s" % (graph_rep, P / (graph_rep / 1e3)))

    # live per-kernel timing (HIP events on the launch stream), same work
    ctx.profile(True)
    prof_steps = max(3, min(args.steps, 10))
    with one_chunk(ctx, [N]):
        for _ in range(prof_steps):
            step()
        torch.cuda.synchronize()
    kt = ctx.profile_read()
    ctx.profile(False)
    kernels = {}
    for name, (cnt, tot) in kt.items():
        b = kernel_bytes(name, N, P * prof_steps / cnt, S_SECTIONS, SIZE)
        avg = tot / cnt
        kernels[name] = dict(launches=cnt, avg_ms=avg, bytes=b, gbs=b / (avg / 1e3) / 1e9)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    d = kernels[dom]
    # measured HBM bytes per launch of the dominant kernel (rocprofv3 FETCH_SIZE +
    # WRITE_SIZE, copy-calibrated), valid only for the kernel sources it was taken on
    from paper_1612_04787_amd.counters import read_traffic, source_digest
    traffic, digest = read_traffic(TRAFFIC_FILE, dom)
    digest_now = source_digest()
    if digest != digest_now:
        traffic = None
    roof = dict(bound="hbm", kernel=dom, achieved=d["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=d["gbs"] / HBM_PEAK_GBS, traffic=traffic,
                bytes_per_launch=d["bytes"], avg_ms=d["avg_ms"],
                timing="HIP events on the launch stream over %d steps, the batch as one chunk (every launch covers "
                       "all %d pairs)" % (prof_steps, P))
    # LDS bytes per launch of the three passes (rocprofv3 LDS load/store
    # bandwidth counters, valid for the kernel sources they were taken on)
    # over the live launch times
    from paper_1612_04787_amd.counters import read_lds
    lds_rate = {}
    for kname, kv in kernels.items():
        if not kname.startswith(("k_row_fwd", "k_col", "k_row_inv")):
            continue
        # the library's timer names the column pass k_col<N>; rocprofv3 sees
        # the kernel, k_col_pair<N>
        lname = kname.replace("k_col<", "k_col_pair<")
        b, busy, dg = read_lds(LDS_FILE, lname)
        if b is None or dg != digest_now:
            continue
        gbs = b / (kv["avg_ms"] / 1e3) / 1e9
        lds_rate[kname] = dict(bytes_per_launch=b, gbs=gbs, peak_gbs=LDS_PEAK_GBS, frac=gbs / LDS_PEAK_GBS,
                               busy_frac_counter=busy)
    res = sw.parse_records(out)
    snr = res["snr"].float()
    step_bytes = P * pair_bytes(N) + kernel_bytes("k_project", N, P, S_SECTIONS, SIZE)

    pruned = None
    if not args.no_prune:
        # the same step with the pruned inverse: peak searched within +-PRUNE_R
        # px, only the surface rows near the origin transformed back
        prm_p = sw.make_params(p=P_WHITEN, max_shift=PRUNE_R)
        out_p = torch.empty_like(out)

        def step_p():
            ctx.project(stack, k=K_PROJ, out=refs)
            ctx.match_batch_raw(table, len(images), pairs, prm_p, out_p, None, ws)

        for _ in range(args.warmup):
            step_p()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_p()
        torch.cuda.synchronize()
        ms_p = (time.perf_counter() - t0) / args.steps * 1e3
        ctx.profile(True)
        with one_chunk(ctx, [N]):
            for _ in range(prof_steps):
                step_p()
            torch.cuda.synchronize()
        rows_p = kept_rows(N, PRUNE_R, ctx.plan(N)[1])
        kp, roof_p = variant_kernels(ctx.profile_read(), N, P, rows_p, False,
                                     TRAFFIC_FILE,
                                     steps=prof_steps)
        ctx.profile(False)
        rp = sw.parse_records(out_p)
        same = (rp["ix"] == res["ix"]) & (rp["iy"] == res["iy"])
        dd = torch.maximum((rp["dx"] - res["dx"]).abs(), (rp["dy"] - res["dy"]).abs())[same]
        pruned = dict(radius_px=PRUNE_R, rows_kept=rows_p, ms_per_step=ms_p, pairs_per_s=P / (ms_p / 1e3),
                      speedup=ms / ms_p, kernels=kp, roofline=roof_p, same_peak_frac=float(same.float().mean()),
                      max_subpixel_diff_px=float(dd.max()) if dd.numel() else None,
                      max_snr_rel_diff=float(((rp["snr"] - res["snr"]).abs() / res["snr"].abs()).max()))
        log("pruned (r=%d): %.3f ms/step (%.2fx), same peak %.4f" % (PRUNE_R, ms_p, ms / ms_p,
                                                                     pruned["same_peak_frac"]))
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^2 window pairs: 64 sections of 4096^2 uint8 (drift + affine distortion), "
                               "references = +-3 z-projections, 8x8 windows per section",
                   "window": N, "pairs": P, "sections": S_SECTIONS, "section_px": SIZE, "p": P_WHITEN,
                   "eps_rel": 1e-4, "taper_frac": 0.25, "projection_k": K_PROJ},
        "hbm_gbs": step_bytes / (ms / 1e3) / 1e9,
        "alu_tflops": P * pair_flops(N) / (ms / 1e3) / 1e12,
        "roofline": roof,
        # whole path against its traffic / flop model (uint8 inputs, the
        # record and one write + read of each exchanged spectrum per pair):
        # the binding bound, and the stricter bound of the inputs alone
        "path_roofline": path_roofline(value, N),
        "kernels": kernels,
        "lds": lds_rate or None,
        "plan": {str(n): {"fwd_rows": v[1][0], "inv_rows": v[1][1], "chunks": v[1][2],
                          "one_workgroup": v[1][0] == n, "slot_ms": v[0]} for n, v in tuned.items()},
        "match_quality": {"median_snr": float(snr.median()), "frac_snr_gt_15": float((snr > 15).float().mean())},
        "graph_replays": {"replays": 20, "median_ms_per_step": graph_rep, "pairs_per_s": P / (graph_rep / 1e3),
                          "note": "projection + the match as one replayed hipGraph, each replay timed with HIP "
                                  "events on the launch stream"},
    }
    ref = hbm_reference(dev)
    ref["roofline_kernel_frac_of_reference"] = roof["achieved"] / ref["elementwise_rw_gbs"] if roof else None
    ref["path_frac_of_reference"] = line["hbm_gbs"] / ref["elementwise_rw_gbs"]
    line["hbm_reference"] = ref
    log("HBM reference (elementwise read + write of 1 GiB): %.0f GB/s; headline step %.0f GB/s (%.2f of it)"
        % (ref["elementwise_rw_gbs"], line["hbm_gbs"], ref["path_frac_of_reference"]))
    if pruned is not None:
        line["pruned"] = pruned
    if not args.no_pearson:
        log("pearson: the same batch scored by Pearson-normalised correlation ...")
        line["pearson"] = pearson_block(ctx, sw, stack, refs, table, images, pairs, res, args, prof_steps)
        pb = line["pearson"]
        log("pearson: %.3f ms/step (%.0f pairs/s), shifts within 1 px of the whitened ones %.3f, median SNR %.1f "
            "(whitened %.1f)" % (pb["ms_per_step"], pb["pairs_per_s"], pb["frac_shift_within_1px"], pb["median_snr"],
                                 pb["median_snr_whitened"]))
    if not args.no_refine:
        log("refinement: plain vs batched + adjoint to 0.01 px ...")
        ws = None
        line["refine"] = refine_comparison(ctx, sw, stack, cen, dev)
        line["refine_pruned"] = refine_comparison(ctx, sw, stack, cen, dev, max_shift=REFINE_R)
        line["refine_generator_bias"] = gb = refine_generator_bias(ctx, sw, dev)
        log("refine, truth generator sensitivity: converged error %.4f px mean (%.4f max) with a cubic-spline "
            "shifted image, %.1e px with a bilinear one" % (gb["cubic"]["mean_px"], gb["cubic"]["max_px"],
                                                           gb["bilinear"]["mean_px"]))
        for key in ("refine", "refine_pruned"):
            rf = line[key]
            log("%s: to 0.01 px plain %s it %.1f ms | adjoint %s it %.1f ms; final rms plain %.2e adjoint %.2e"
                % (key, rf["plain"]["iters_to_target"], rf["plain"]["ms_to_target"] or -1,
                   rf["adjoint"]["iters_to_target"], rf["adjoint"]["ms_to_target"] or -1, rf["plain"]["rms_px"],
                   rf["adjoint"]["rms_px"]))
    if not args.no_stack:
        log("stack loop: 3 passes of render / project / match + refine / fit ...")
        line["stack_loop"] = stack_loop(ctx, stack, warps)
        r = line["stack_loop"]["residual_px"]
        log("stack loop: %.0f ms, residual global %.2f -> %.2f px, neighbour %.2f -> %.2f px"
            % (line["stack_loop"]["wall_ms"], r["global_before"], r["global_after"], r["neighbour_before"],
               r["neighbour_after"]))
    jump_sample = None
    if not args.no_jump:
        log("jump repair: a stack with a magnification change ...")
        line["jump_repair"], jump_sample = jump_block(ctx, dev)
        jr = line["jump_repair"]["pair_residual_px"]
        log("jump repair: break %.2f px -> %.2f px (max pair %.2f -> %.2f), %.0f ms"
            % (jr["at_jump_before"], jr["at_jump_after"], jr["max_before"], jr["max_after"],
               line["jump_repair"]["repair_ms"]))
    search_sample = None
    if not args.no_search:
        log("search: candidate offsets with an SNR stop vs every candidate ...")
        line["search"], search_sample = search_block(ctx, sw, dev)
        q = line["search"]
        log("search: %.2f ms (%d matches) vs %.2f ms exhaustive (%d), %.2fx; done %.3f, max err %.3f px, "
            "same offset as exhaustive %.3f" % (q["ms"], q["matches"], q["exhaustive"]["ms"],
                                                q["exhaustive"]["matches"], q["speedup"], q["done_frac"],
                                                q["max_err_px_done"] or -1, q["same_offset_as_exhaustive"]))
        log("search: %s %.1f GB/s over the search (%.2f of HBM peak)"
            % (q["roofline"]["kernel"], q["roofline"]["achieved"], q["roofline"]["frac"]))
        for B, v in q["lookahead"].items():
            log("search, %s candidates per round: %.2f ms (%d matches), same result %s"
                % (B, v["ms"], v["matches"], v["same_result"]))
        log("search in the stack loop: a section moved beyond one window's capture ...")
        q["stack_loop"] = search_stack_block(ctx, dev)
        w1, w0 = q["stack_loop"]["with_search"], q["stack_loop"]["without"]
        w4 = q["stack_loop"]["with_search_lookahead4"]
        log("search in the stack loop: max pair residual %.2f px with (%d search matches, %.0f ms; with 4 "
            "candidates per round %.2f px, %.0f ms), %.1f px without (%.0f ms)"
            % (w1["max_pair_px"], w1["search_matches"], w1["wall_ms"], w4["max_pair_px"], w4["wall_ms"],
               w0["max_pair_px"], w0["wall_ms"]))
    mesh_sample = None
    if not args.no_mesh:
        log("mesh: global affines then two local-affine mesh passes on a bent stack ...")
        line["mesh"], mesh_sample = mesh_block(ctx, dev)
        m = line["mesh"]
        log("mesh: neighbour residual %.3f -> %.3f px; passes %.0f ms; render_mesh %.3f ms (%.0f Gpix/s), "
            "render %.3f ms" % (m["residual_px"]["neighbour_affine"], m["residual_px"]["neighbour_mesh"],
                                m["mesh_ms"], m["render_mesh"]["ms"], m["render_mesh"]["gpix_s"],
                                m["render_affine"]["ms"]))
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the FP64 oracle on a sample ...")
        line["cpu_baseline"] = cpu_baseline(stack.cpu().numpy(), refs.cpu().numpy(), cen)
        log("cpu baseline: %.1f pairs/s on %d cores" % (line["cpu_baseline"]["value"], line["cpu_baseline"]["cores"]))
        line["cpu_baseline"]["fp32_scipy"] = cpu_fp32_baseline(stack.cpu().numpy(), refs.cpu().numpy(), cen)
        log("cpu baseline, FP32 SciPy: %.1f pairs/s on %d cores" % (line["cpu_baseline"]["fp32_scipy"]["value"],
                                                                   line["cpu_baseline"]["fp32_scipy"]["cores"]))
        if mesh_sample is not None:
            line["cpu_baseline"]["mesh_render"] = cpu_baseline_mesh(mesh_sample)
        if jump_sample is not None:
            line["cpu_baseline"]["jump_models"] = cpu_baseline_jump(jump_sample)
        if search_sample is not None:
            line["cpu_baseline"]["search"] = cpu_baseline_search(search_sample)
        if not (args.no_prune and args.no_pearson):
            line["cpu_baseline"].update(cpu_baseline_variants(stack.cpu().numpy(), refs.cpu().numpy(), cen))
    if not args.no_config2:
        log("config 2: 256 pairs of 1024^2 from a 16384^2 section pair ...")
        ws = None
        torch.cuda.empty_cache()
        line["config2_1024"] = config2_block(ctx, sw, dev)
        c2 = line["config2_1024"]
        log("config 2: median %.3f ms (%.0f pairs/s, %.2f of the path's HBM bound); %s %.0f GB/s (%.2f of peak); "
            "median shift error %.3f px" % (c2["median_ms"], c2["pairs_per_s"], c2["path_roofline"]["frac"],
                                            c2["roofline"]["kernel"], c2["roofline"]["achieved"],
                                            c2["roofline"]["frac"], c2["shift_error_px"]["median"]))
        torch.cuda.empty_cache()
    if not args.no_sizes:
        log("per-size rooflines: 2048 pairs of each size on an 8192^2 section pair ...")
        torch.cuda.empty_cache()
        line["sizes"] = size_rooflines(ctx, sw, dev)
        for k, v in line["sizes"].items():
            log("  n=%s: %.3f ms for %d pairs (%.0f pairs/s), %s %.1f %s (%.3f of peak), plan %s"
                % (k, v["median_ms"], v["pairs"], v["pairs_per_s"], v["roofline"]["bound"], v["roofline"]["achieved"],
                   v["roofline"]["unit"], v["roofline"]["frac"], v["plan"]))
        torch.cuda.empty_cache()
    if not args.no_ragged:
        # the multi-level block runs in a child process with the default plan
        # (one chunk per size group): its first run with the tuned plans ended
        # the process with a host segfault whose cause was not found, and a
        # child keeps any such failure from taking the benchmark line with it
        log("ragged levels (child process, default plan): per-level calls vs one concurrent call vs one graph, "
            "and the refinement on them ...")
        del stack, refs, images, table, out
        torch.cuda.empty_cache()
        line.update(ragged_child(args, log))
    ctx.close()
    print(json.dumps(line), flush=True)


def ragged_child(args, log):
    """Runs `bench.py --ragged-child` and returns its blocks, or an error record."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--ragged-child"]
    if args.no_refine:
        cmd.append("--no-refine")
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, timeout=900, text=True)
    except subprocess.TimeoutExpired:
        log("ragged child: timed out")
        return {"ragged": {"error": "timed out after 900 s"}}
    if r.returncode != 0 or not r.stdout.strip():
        log("ragged child: exit status %d" % r.returncode)
        return {"ragged": {"error": "child process exit status %d" % r.returncode}}
    return json.loads(r.stdout.strip().splitlines()[-1])


def ragged_main(args):
    """The multi-level blocks alone, with the default plan; prints one JSON
    object with `ragged` (and `refine_levels`)."""
    import torch

    import paper_1612_04787_amd as sw
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    dev = torch.device("cuda", 0)
    ctx = sw.Swift(0)
    out = {}
    images3 = config3_images(ctx, dev)
    out["ragged"] = ragged_levels(ctx, sw, dev, images3)
    g = out["ragged"]
    log("ragged levels: per-level %.2f ms, one call %.2f ms, graph %.2f ms"
        % (g["per_level_calls"]["ms"], g["one_call_concurrent"]["ms"], g["graph"]["ms"]))
    for k, v in g["per_size"].items():
        log("  n=%s: %.3f ms for %d pairs, %s %.1f %s (%.3f of peak), plan %s"
            % (k, v["ms"], v["pairs"], v["roofline"]["bound"], v["roofline"]["achieved"], v["roofline"]["unit"],
               v["roofline"]["frac"], v["plan"]))
    sb = g["small_batch"]
    log("ragged levels, small batch (%s): per-level %.3f ms, graph %.3f ms (%.2fx)"
        % (sb["workload"], sb["per_level_calls"]["ms"], sb["graph"]["ms"], sb["graph_speedup_vs_per_level"]))
    if not args.no_refine:
        log("refinement on the ragged levels: plain per-level calls vs one graph per iteration + adjoint ...")
        out["refine_levels"] = refine_levels(ctx, sw, dev, images3)
        q = out["refine_levels"]
        log("refine levels: to %.2f px rms plain %s it %s ms | batched+adjoint %s it %s ms"
            % (q["target_rms_px"], q["plain"]["iters_to_target"], q["plain"]["ms_to_target"],
               q["batched_adjoint"]["iters_to_target"], q["batched_adjoint"]["ms_to_target"]))
        ik = q["iteration_kernels"]
        log("refine levels, kernel time per iteration: centroid %.2f ms, Newton %.2f ms (match with saved state "
            "%.2f + Jacobian %.2f)" % (ik["centroid_iteration_ms"], ik["newton_iteration_ms"], ik["match_saved"]["ms"],
                                       ik["jacobian"]["ms"]))
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
