"""ctypes binding of libswift (include/swift.h).

Argument marshalling only: tensors supply device memory and the current HIP
stream; every step of matching runs in the library's HIP kernels.  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswift.so")
SIZES = (64, 128, 256, 512, 1024)

SWIFT_U8, SWIFT_F32 = 0, 1
FLAG_CONCURRENT_SIZES = 1
FLAG_JAC_TRANSLATION = 2
FLAG_PEARSON = 4
ST_NEAR_TIE, ST_DEGENERATE, ST_CLAMPED = 1, 2, 4
ERRORS = {-1: "SWIFT_E_INVAL", -2: "SWIFT_E_UNSUPPORTED", -3: "SWIFT_E_WORKSPACE",
          -4: "SWIFT_E_HIP", -5: "SWIFT_E_CAPTURE"}


class SwiftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch", C.c_int64), ("dtype", C.c_int32), ("reserved", C.c_int32)]


class Pairs(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("size_count", C.c_int32 * 5),
                ("img_a", C.c_void_p), ("img_b", C.c_void_p),
                ("theta_a", C.c_void_p), ("theta_b", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("p", C.c_float), ("eps_rel", C.c_float), ("taper_frac", C.c_float),
                ("centroid_r", C.c_int32), ("flags", C.c_int32), ("max_shift", C.c_int32),
                ("snr_exclude_r", C.c_int32), ("reserved", C.c_int32)]


REC_BYTES = 64
TUNE_SLOTS = 8
assert C.sizeof(Image) == 32 and C.sizeof(Pairs) == 56 and C.sizeof(Params) == 32

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libswift.so and declares its entry points.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libswift.so is not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.swift_create.argtypes = [C.c_int, C.c_char_p, C.POINTER(vp)]
    lib.swift_destroy.argtypes = [vp]
    lib.swift_destroy.restype = None
    lib.swift_workspace_size.argtypes = [vp, C.POINTER(Pairs), C.POINTER(Params), C.POINTER(sz), C.POINTER(sz)]
    lib.swift_match_batch.argtypes = [vp, vp, i32, C.POINTER(Pairs), C.POINTER(Params), vp, vp, vp, vp, sz, vp]
    lib.swift_match_graph.argtypes = [vp, vp, i32, C.POINTER(Pairs), C.POINTER(Params), vp, vp, vp, vp, sz, vp]
    lib.swift_match_batch_noalloc.argtypes = [vp, vp, i32, C.POINTER(Pairs), C.POINTER(Params), vp, vp]
    lib.swift_plan.argtypes = [vp, i32, i32, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.swift_autotune.argtypes = [vp, C.POINTER(i32), i32, i32, C.POINTER(C.c_float)]
    lib.swift_match_backward.argtypes = [vp, vp, i32, C.POINTER(Pairs), C.POINTER(Params), vp, vp, vp, vp, vp,
                                         vp, vp, sz, vp]
    lib.swift_project.argtypes = [vp, vp, i32, i32, i32, i64, i64, vp, i32, vp, i64, i64, vp]
    lib.swift_pyramid.argtypes = [vp, C.POINTER(Image), C.POINTER(Image), vp]
    lib.swift_snr.argtypes = [vp, vp, i32, i32, C.POINTER(Params), vp, vp]
    lib.swift_centroid_jacobian.argtypes = [vp, vp, i32, C.POINTER(Pairs), C.POINTER(Params), vp, vp, vp, sz, vp]
    lib.swift_refine_update.argtypes = [vp, i32, vp, vp, vp, i32, C.c_float, vp, vp]
    lib.swift_render.argtypes = [vp, vp, i32, i32, i32, i64, i64, vp, i32, vp, i32, i32, i64, i64, vp]
    lib.swift_stack_windows.argtypes = [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.swift_fit_sections.argtypes = [vp, i32, i32, vp, vp, vp, i32, C.c_float, vp, vp, vp]
    lib.swift_project_side.argtypes = [vp, vp, i32, i32, i32, i64, i64, vp, i32, i32, vp, i64, i64, vp]
    lib.swift_blend_span.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
    lib.swift_join_break.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.swift_search_keep.argtypes = [vp, i32, i32, vp, vp, i32, C.c_float, vp, vp, vp, vp]
    lib.swift_search_next.argtypes = [vp, i32, vp, C.c_float, C.c_float, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.swift_render_mesh.argtypes = [vp, vp, i32, i32, i32, i64, i64, vp, i32, i32, vp, i32, i32, i64, i64, vp]
    lib.swift_mesh_windows.argtypes = [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.swift_fit_mesh.argtypes = [vp, i32, i32, vp, vp, vp, i32, C.c_float, vp, vp, vp, vp]
    lib.swift_profile_enable.argtypes = [vp, C.c_int]
    lib.swift_profile_read.argtypes = [vp, i32, C.c_char_p, C.POINTER(i32), C.POINTER(C.c_double), C.POINTER(i32)]
    lib.swift_last_error.restype = C.c_char_p
    for f in exported_symbols():
        if f not in ("swift_destroy", "swift_last_error"):
            getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def exported_symbols():
    """Every entry point include/swift.h declares."""
    return ["swift_create", "swift_destroy", "swift_workspace_size", "swift_match_batch", "swift_match_batch_noalloc",
            "swift_match_graph",
            "swift_match_backward", "swift_centroid_jacobian", "swift_project", "swift_project_side",
            "swift_blend_span", "swift_join_break", "swift_search_keep", "swift_search_next", "swift_pyramid",
            "swift_snr", "swift_refine_update", "swift_render", "swift_stack_windows", "swift_fit_sections",
            "swift_render_mesh", "swift_mesh_windows", "swift_fit_mesh", "swift_plan", "swift_autotune",
            "swift_profile_enable", "swift_profile_read", "swift_last_error"]


def _check(rc):
    if rc != 0:
        raise SwiftError(rc, _lib.swift_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def make_params(p=0.65, eps_rel=1e-4, taper_frac=0.25, centroid_r=1, flags=0, max_shift=0, snr_exclude_r=0):
    return Params(float(p), float(eps_rel), float(taper_frac), int(centroid_r), int(flags), int(max_shift),
                  int(snr_exclude_r), 0)


def parse_records(rec: torch.Tensor) -> dict:
    """Splits a [P, 64] uint8 record tensor into named field views."""
    P = rec.shape[0]
    f32 = rec.view(torch.float32).view(P, 16)
    i32 = rec.view(torch.int32).view(P, 16)
    f64 = rec.view(torch.float64).view(P, 8)
    return dict(dx=f32[:, 0], dy=f32[:, 1], ix=i32[:, 2], iy=i32[:, 3], peak=f32[:, 4], snr=f32[:, 5],
                mean=f64[:, 3], std=f64[:, 4], status=i32[:, 10], n=i32[:, 11], hxx=f32[:, 12], hyy=f32[:, 13],
                hxy=f32[:, 14])


class Swift:
    """A libswift context on one GPU."""

    def __init__(self, device: int = 0, tune_cache=None):
        """tune_cache: path of the plan file swift_autotune writes and later
        contexts read (None: no file)."""
        if not torch.cuda.is_available():
            raise RuntimeError("libswift needs a ROCm GPU; none is visible")
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        path = tune_cache.encode() if tune_cache else None
        _check(self.lib.swift_create(device, path, C.byref(h)))
        self.h = h
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.swift_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------------ kernel timing
    def profile(self, enable=True):
        _check(self.lib.swift_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self, max_kernels=64):
        """{kernel name: (launches, total ms)} of the kernels timed since the last read."""
        names = C.create_string_buffer(64 * max_kernels)
        cnt = (C.c_int32 * max_kernels)()
        ms = (C.c_double * max_kernels)()
        nk = C.c_int32()
        _check(self.lib.swift_profile_read(self.h, max_kernels, names, cnt, ms, C.byref(nk)))
        out = {}
        for i in range(min(nk.value, max_kernels)):
            nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (cnt[i], ms[i])
        return out

    # ------------------------------------------------------------------ helpers
    def image_table(self, images):
        """Device table of swift_image descriptors for a list of 2-D uint8 or
        float32 device tensors (row pitch from their strides)."""
        rows = []
        for im in images:
            assert im.dim() == 2 and im.device == self.device and im.stride(1) == 1
            dt = SWIFT_U8 if im.dtype == torch.uint8 else SWIFT_F32
            assert im.dtype in (torch.uint8, torch.float32)
            pitch = im.stride(0) * im.element_size()
            rows.append([im.data_ptr(), (im.shape[1] & 0xFFFFFFFF) | (im.shape[0] << 32), pitch, dt])
        t = torch.tensor(rows, dtype=torch.int64).to(self.device)
        t._swift_keepalive = list(images)
        return t

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    @staticmethod
    def make_pairs(n_list, img_a, img_b, theta_a, theta_b):
        n_list = [int(n) for n in n_list]
        assert all(n_list[i] <= n_list[i + 1] for i in range(len(n_list) - 1)), "pairs must be sorted by n"
        counts = [sum(1 for n in n_list if n == s) for s in SIZES]
        assert sum(counts) == len(n_list), "window edges must be in %s" % (SIZES,)
        pr = Pairs()
        pr.n_pairs = len(n_list)
        for i, c in enumerate(counts):
            pr.size_count[i] = c
        pr.img_a, pr.img_b = img_a.data_ptr(), img_b.data_ptr()
        pr.theta_a, pr.theta_b = theta_a.data_ptr(), theta_b.data_ptr()
        return pr

    def workspace_size(self, pairs, params):
        ws = C.c_size_t()
        sv = C.c_size_t()
        _check(self.lib.swift_workspace_size(self.h, C.byref(pairs), C.byref(params), C.byref(ws), C.byref(sv)))
        return ws.value, sv.value

    # ------------------------------------------------------------------ entry points
    def match_batch_raw(self, table, n_imgs, pairs, params, out, surfaces=None, ws=None, saved=None, graph=False):
        """swift_match_batch, or with graph=True swift_match_graph (captured
        once per argument tuple, then replayed)."""
        need, _ = self.workspace_size(pairs, params)
        if ws is None:
            ws = self.workspace(need)
        fn = self.lib.swift_match_graph if graph else self.lib.swift_match_batch
        _check(fn(self.h, _ptr(table), int(n_imgs), C.byref(pairs), C.byref(params), _ptr(out), _ptr(surfaces),
                  _ptr(saved), _ptr(ws), ws.numel(), self.stream()))

    def match_backward_raw(self, table, n_imgs, pairs, params, saved, g_peak, g_snr, g_theta_a, g_theta_b=None,
                           peak_hess=None, ws=None):
        need, _ = self.workspace_size(pairs, params)
        if ws is None:
            ws = self.workspace(need)
        _check(self.lib.swift_match_backward(self.h, _ptr(table), int(n_imgs), C.byref(pairs), C.byref(params),
                                             _ptr(saved), _ptr(g_peak), _ptr(g_snr), _ptr(g_theta_a),
                                             _ptr(g_theta_b), _ptr(peak_hess), _ptr(ws), ws.numel(), self.stream()))

    def centroid_jacobian_raw(self, table, n_imgs, pairs, params, saved, jac, ws=None):
        need, _ = self.workspace_size(pairs, params)
        if ws is None:
            ws = self.workspace(need)
        _check(self.lib.swift_centroid_jacobian(self.h, _ptr(table), int(n_imgs), C.byref(pairs), C.byref(params),
                                                _ptr(saved), _ptr(jac), _ptr(ws), ws.numel(), self.stream()))

    def prepare(self, images, n_list, img_a, img_b, theta_a, theta_b):
        """Device image table and pair descriptor (tensors kept alive in the dict)."""
        table = self.image_table(images)
        img_a = img_a.to(self.device, torch.int32).contiguous()
        img_b = img_b.to(self.device, torch.int32).contiguous()
        theta_a = theta_a.to(self.device, torch.float32).contiguous()
        theta_b = theta_b.to(self.device, torch.float32).contiguous()
        pr = self.make_pairs(n_list, img_a, img_b, theta_a, theta_b)
        return dict(table=table, n_imgs=len(images), pairs=pr, keep=(img_a, img_b, theta_a, theta_b))

    def match_batch(self, images, n_list, img_a, img_b, theta_a, theta_b, params=None, surfaces=False, save=False):
        """Whitened FFT matching of window pairs.  images: list of device
        tensors; n_list: host list of window edges (sorted); img_a/img_b: int32
        device [P]; theta_a/theta_b: float32 device [P, 8].  Returns a dict of
        device tensors (dx, dy, ix, iy, peak, snr, mean, std, status, n) and,
        with surfaces=True, 'surfaces' as a flat float32 tensor; with save=True,
        'saved' (state for match_backward) and 'prep'."""
        params = params or make_params()
        prep = self.prepare(images, n_list, img_a, img_b, theta_a, theta_b)
        pr = prep["pairs"]
        P = pr.n_pairs
        out = torch.empty((P, REC_BYTES), dtype=torch.uint8, device=self.device)
        surf = None
        if surfaces:
            surf = torch.empty(sum(int(n) * int(n) for n in n_list), dtype=torch.float32, device=self.device)
        saved = None
        if save:
            _, sv = self.workspace_size(pr, params)
            saved = torch.empty(max(sv, 256), dtype=torch.uint8, device=self.device)
        self.match_batch_raw(prep["table"], prep["n_imgs"], pr, params, out, surf, saved=saved)
        res = parse_records(out)
        res["raw"] = out
        if surfaces:
            res["surfaces"] = surf
        if save:
            res["saved"] = saved
            res["prep"] = prep
        return res

    def match_backward(self, fwd, params, g_peak=None, g_snr=None, want_b=True, want_hess=False):
        """Gradients [P, 6] (a11, a12, tx, a21, a22, ty) of sum(g_peak*peak +
        g_snr*snr) for windows A (and B) of a forward run made with save=True;
        with want_hess also the surface Hessian at the peak [P, 3]."""
        prep = fwd["prep"]
        P = prep["pairs"].n_pairs
        ga = torch.empty((P, 6), dtype=torch.float32, device=self.device)
        gb = torch.empty((P, 6), dtype=torch.float32, device=self.device) if want_b else None
        hs = torch.empty((P, 3), dtype=torch.float32, device=self.device) if want_hess else None
        gp = g_peak.to(self.device, torch.float32).contiguous() if g_peak is not None else None
        gs = g_snr.to(self.device, torch.float32).contiguous() if g_snr is not None else None
        self.match_backward_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, fwd["saved"], gp, gs, ga, gb,
                                hs)
        if want_hess:
            return ga, gb, hs
        return ga, gb

    def project(self, stack, k=3, exclude=None, out=None):
        """Z-projection models of every section of a [S, H, W] uint8 device stack."""
        assert stack.dtype == torch.uint8 and stack.dim() == 3 and stack.stride(2) == 1
        S, H, W = stack.shape
        if out is None:
            out = torch.empty_like(stack)
        ex = None
        if exclude is not None:
            ex = torch.as_tensor(exclude, dtype=torch.uint8).to(self.device).contiguous()
        _check(self.lib.swift_project(self.h, _ptr(stack), S, H, W, stack.stride(1), stack.stride(0), _ptr(ex),
                                      int(k), _ptr(out), out.stride(1), out.stride(0), self.stream()))
        return out

    def pyramid(self, img, out=None):
        assert img.dtype == torch.uint8 and img.dim() == 2 and img.stride(1) == 1
        h, w = img.shape
        dst = out if out is not None else torch.empty((h // 2, w // 2), dtype=torch.uint8, device=img.device)
        assert dst.shape == (h // 2, w // 2) and dst.stride(1) == 1
        si = Image(img.data_ptr(), w, h, img.stride(0), SWIFT_U8, 0)
        di = Image(dst.data_ptr(), w // 2, h // 2, dst.stride(0), SWIFT_U8, 0)
        _check(self.lib.swift_pyramid(self.h, C.byref(si), C.byref(di), self.stream()))
        return dst

    def centroid_jacobian(self, fwd, params):
        """[P, 2, 6]: d(dx)/d theta_A and d(dy)/d theta_A for a forward run
        made with save=True."""
        prep = fwd["prep"]
        P = prep["pairs"].n_pairs
        jac = torch.empty((P, 2, 6), dtype=torch.float32, device=self.device)
        self.centroid_jacobian_raw(prep["table"], prep["n_imgs"], prep["pairs"], params, fwd["saved"], jac)
        return jac

    def refine_update(self, recs_raw, theta, mode=0, jac=None, max_step=0.5, step_out=None):
        """One refinement step applied in place to theta [P, 8] (device);
        Newton mode takes jac [P, 2, 6] from centroid_jacobian."""
        P = theta.shape[0]
        _check(self.lib.swift_refine_update(self.h, P, _ptr(recs_raw), _ptr(jac), _ptr(theta), int(mode),
                                            float(max_step), _ptr(step_out), self.stream()))

    # ------------------------------------------------------------------ tuning
    def plan(self, n, fwd_variant=-1, inv_variant=-1, chunks=-1, full=False):
        """Sets (values >= 0) and returns the plan of size n as (forward rows
        per block, inverse rows per block), with full=True also the chunks."""
        fr, ir, ch = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib.swift_plan(self.h, int(n), int(fwd_variant), int(inv_variant), int(chunks), C.byref(fr),
                                   C.byref(ir), C.byref(ch)))
        if full:
            return fr.value, ir.value, ch.value
        return fr.value, ir.value

    def autotune(self, sizes=SIZES, pairs_per_size=512):
        """Times the plan variants of each size and keeps the fastest.
        Returns {n: (times_ms[TUNE_SLOTS], (fwd_rows, inv_rows, chunks))}."""
        sizes = [int(n) for n in sizes]
        arr = (C.c_int32 * len(sizes))(*sizes)
        times = (C.c_float * (TUNE_SLOTS * len(sizes)))()
        _check(self.lib.swift_autotune(self.h, arr, len(sizes), int(pairs_per_size), times))
        return {n: (list(times[TUNE_SLOTS * k:TUNE_SLOTS * k + TUNE_SLOTS]), self.plan(n, full=True))
                for k, n in enumerate(sizes)}

    # ------------------------------------------------------------------ stack loop
    def render(self, src, aff, level, out_hw=None, out=None):
        """mir rendering of a [S, H, W] uint8 device stack (level-l raw
        sections) by level-0 affines aff [S, 6] float64 (device)."""
        assert src.dtype == torch.uint8 and src.dim() == 3 and src.stride(2) == 1
        assert aff.dtype == torch.float64 and aff.is_contiguous() and aff.shape == (src.shape[0], 6)
        S, H, W = src.shape
        if out is None:
            oh, ow = out_hw if out_hw is not None else (H, W)
            out = torch.empty((S, oh, ow), dtype=torch.uint8, device=src.device)
        _check(self.lib.swift_render(self.h, _ptr(src), S, H, W, src.stride(1), src.stride(0), _ptr(aff), int(level),
                                     _ptr(out), out.shape[1], out.shape[2], out.stride(1), out.stride(0),
                                     self.stream()))
        return out

    def stack_windows(self, aff, level, grid, h_l, w_l, img_a0, img_b0):
        """Window pairs of every section: (img_a, img_b [P] int32, theta_a,
        theta_b [P, 8] float32), P = S * grid^2, all on the device."""
        S = aff.shape[0]
        P = S * grid * grid
        ta = torch.empty((P, 8), dtype=torch.float32, device=self.device)
        tb = torch.empty((P, 8), dtype=torch.float32, device=self.device)
        ia = torch.empty(P, dtype=torch.int32, device=self.device)
        ib = torch.empty(P, dtype=torch.int32, device=self.device)
        _check(self.lib.swift_stack_windows(self.h, S, _ptr(aff), int(level), int(grid), int(h_l), int(w_l),
                                            int(img_a0), int(img_b0), _ptr(ta), _ptr(tb), _ptr(ia), _ptr(ib),
                                            self.stream()))
        return ia, ib, ta, tb

    def fit_sections(self, theta_a, theta_b, recs_raw, per_section, level, aff, min_snr=6.0, status=None):
        """Refits aff [S, 6] float64 (device, in place) from the window
        matches; returns the per-section status tensor."""
        S = aff.shape[0]
        if status is None:
            status = torch.empty(S, dtype=torch.int32, device=self.device)
        _check(self.lib.swift_fit_sections(self.h, S, int(per_section), _ptr(theta_a), _ptr(theta_b),
                                           _ptr(recs_raw), int(level), float(min_snr), _ptr(aff), _ptr(status),
                                           self.stream()))
        return status

    # ---- jump repair
    def project_side(self, stack, k, side, exclude=None, out=None):
        """One-sided models (side -1: the k sections before, +1: after) of a
        [S, H, W] uint8 device stack; exclude: [S] uint8 device or None."""
        assert stack.dtype == torch.uint8 and stack.dim() == 3 and stack.stride(2) == 1
        S, H, W = stack.shape
        if out is None:
            out = torch.empty_like(stack)
        ex = None if exclude is None else exclude.to(self.device, torch.uint8).contiguous()
        _check(self.lib.swift_project_side(self.h, _ptr(stack), S, H, W, stack.stride(1), stack.stride(0), _ptr(ex),
                                           int(k), int(side), _ptr(out), out.stride(1), out.stride(0),
                                           self.stream()))
        return out

    def blend_span(self, a, b, aff_left, aff_right, aff):
        """aff[a..b] <- Bezier blend of aff_left and aff_right (all [S, 6]
        float64 device)."""
        S = aff.shape[0]
        for t in (aff_left, aff_right, aff):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.shape == (S, 6)
        _check(self.lib.swift_blend_span(self.h, S, int(a), int(b), _ptr(aff_left), _ptr(aff_right), _ptr(aff),
                                         self.stream()))
        return aff

    def join_break(self, j, aff, aff_left, out=None):
        """Sections from j on composed with D = A_j^-1 L_j ([S, 6] float64
        device; returns out)."""
        S = aff.shape[0]
        if out is None:
            out = torch.empty_like(aff)
        for t in (aff, aff_left, out):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.shape == (S, 6)
        _check(self.lib.swift_join_break(self.h, S, int(j), _ptr(aff), _ptr(aff_left), _ptr(out), self.stream()))
        return out

    def search_next(self, done, ox, oy, img_a, img_b, theta_a, theta_b, idx, ia, ib, ta, tb, count):
        """Gathers the windows not yet done (device tensors: done [P] uint8,
        img_a/img_b [P] int32, theta_a/theta_b [P, 8]; outputs with room for
        P, count [1] int32)."""
        P = done.shape[0]
        assert img_a.shape[0] == P and img_b.shape[0] == P and theta_a.shape[0] == P and theta_b.shape[0] == P
        assert idx.shape[0] >= P and ia.shape[0] >= P and ib.shape[0] >= P and ta.shape[0] >= P and tb.shape[0] >= P
        _check(self.lib.swift_search_next(self.h, int(P), _ptr(done), float(ox), float(oy), _ptr(img_a), _ptr(img_b),
                                          _ptr(theta_a), _ptr(theta_b), _ptr(idx), _ptr(ia), _ptr(ib), _ptr(ta),
                                          _ptr(tb), _ptr(count), self.stream()))

    def search_keep(self, P, idx, recs_raw, cand, accept, best, best_cand, done):
        """One round of the SNR-stop search: idx [n] int32, recs_raw [n, 64]
        uint8, best [P, 64] uint8, best_cand [P] int32, done [P] uint8 (all
        device, updated in place)."""
        n = idx.shape[0]
        assert recs_raw.shape[0] == n and best.shape[0] == P and best_cand.shape[0] == P and done.shape[0] == P
        _check(self.lib.swift_search_keep(self.h, int(P), int(n), _ptr(idx), _ptr(recs_raw), int(cand), float(accept),
                                          _ptr(best), _ptr(best_cand), _ptr(done), self.stream()))

    # ---- local-affine triangle mesh: tri_aff [S, 2 (grid-1)^2, 6] float64 (device)
    @staticmethod
    def mesh_triangles(grid):
        return 2 * (grid - 1) * (grid - 1)

    def render_mesh(self, src, tri_aff, grid, level, out_hw=None, out=None):
        """mir texture mapping of a [S, H, W] uint8 device stack: every output
        pixel through the affine of its triangle in the mesh of the output
        frame."""
        assert src.dtype == torch.uint8 and src.dim() == 3 and src.stride(2) == 1
        S, H, W = src.shape
        assert tri_aff.dtype == torch.float64 and tri_aff.is_contiguous()
        assert tri_aff.shape == (S, self.mesh_triangles(grid), 6)
        if out is None:
            oh, ow = out_hw if out_hw is not None else (H, W)
            out = torch.empty((S, oh, ow), dtype=torch.uint8, device=src.device)
        _check(self.lib.swift_render_mesh(self.h, _ptr(src), S, H, W, src.stride(1), src.stride(0), _ptr(tri_aff),
                                          int(grid), int(level), _ptr(out), out.shape[1], out.shape[2],
                                          out.stride(1), out.stride(0), self.stream()))
        return out

    def mesh_windows(self, tri_aff, level, grid, h_l, w_l, img_a0, img_b0):
        """Window pairs at the mesh nodes, window A through its node's
        triangle: (img_a, img_b [P] int32, theta_a, theta_b [P, 8] float32)."""
        S = tri_aff.shape[0]
        assert tri_aff.dtype == torch.float64 and tri_aff.is_contiguous()
        assert tri_aff.shape == (S, self.mesh_triangles(grid), 6)
        P = S * grid * grid
        ta = torch.empty((P, 8), dtype=torch.float32, device=self.device)
        tb = torch.empty((P, 8), dtype=torch.float32, device=self.device)
        ia = torch.empty(P, dtype=torch.int32, device=self.device)
        ib = torch.empty(P, dtype=torch.int32, device=self.device)
        _check(self.lib.swift_mesh_windows(self.h, S, _ptr(tri_aff), int(level), int(grid), int(h_l), int(w_l),
                                           int(img_a0), int(img_b0), _ptr(ta), _ptr(tb), _ptr(ia), _ptr(ib),
                                           self.stream()))
        return ia, ib, ta, tb

    def fit_mesh(self, theta_a, theta_b, recs_raw, grid, level, aff, min_snr=6.0, tri_aff=None, status=None):
        """Per-triangle affines [S, T, 6] float64 from the node matches (pairs
        s grid^2 + k); singular triangles take their section's affine aff
        [S, 6].  Returns (tri_aff, status [S, T] int32)."""
        S = aff.shape[0]
        T = self.mesh_triangles(grid)
        assert aff.dtype == torch.float64 and aff.is_contiguous() and aff.shape == (S, 6)
        assert theta_a.shape[0] == S * grid * grid and recs_raw.shape[0] == S * grid * grid
        if tri_aff is None:
            tri_aff = torch.empty((S, T, 6), dtype=torch.float64, device=self.device)
        if status is None:
            status = torch.empty((S, T), dtype=torch.int32, device=self.device)
        _check(self.lib.swift_fit_mesh(self.h, S, int(grid), _ptr(theta_a), _ptr(theta_b), _ptr(recs_raw),
                                       int(level), float(min_snr), _ptr(aff), _ptr(tri_aff), _ptr(status),
                                       self.stream()))
        return tri_aff, status

    def snr(self, surfaces, params=None):
        """Peak, SNR and centroid of [B, n, n] float32 device surfaces."""
        params = params or make_params()
        surfaces = surfaces.contiguous()
        B, n, _ = surfaces.shape
        out = torch.empty((B, REC_BYTES), dtype=torch.uint8, device=self.device)
        _check(self.lib.swift_snr(self.h, _ptr(surfaces), n, B, C.byref(params), _ptr(out), self.stream()))
        return parse_records(out)


def theta6_to_theta8(g6):
    """Gradient with respect to (a11, a12, tx, a21, a22, ty) -> with respect to
    the 8-entry window parameter (cx, cy, a11, a12, tx, a21, a22, ty); the
    centre enters the sample position exactly like the translation."""
    return torch.stack([g6[:, 2], g6[:, 5], g6[:, 0], g6[:, 1], g6[:, 2], g6[:, 3], g6[:, 4], g6[:, 5]], dim=1)


class SwiftMatchFn(torch.autograd.Function):
    """(peak, snr) of whitened window matches as a differentiable function of
    the window parameters theta_a, theta_b [P, 8]; the backward runs the
    library's adjoint kernels (the integer peak is held fixed)."""

    @staticmethod
    def forward(fctx, theta_a, theta_b, sw, images, n_list, img_a, img_b, params):
        res = sw.match_batch(images, n_list, img_a, img_b, theta_a.detach(), theta_b.detach(), params, save=True)
        fctx.sw, fctx.res, fctx.params = sw, res, params
        return res["peak"].clone(), res["snr"].clone()

    @staticmethod
    def backward(fctx, g_peak, g_snr):
        ga, gb = fctx.sw.match_backward(fctx.res, fctx.params, g_peak, g_snr, want_b=True)
        return theta6_to_theta8(ga), theta6_to_theta8(gb), None, None, None, None, None, None
