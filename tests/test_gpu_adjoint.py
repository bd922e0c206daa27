"""GPU adjoint (d peak / d affine, d SNR / d affine) against the FP64 oracle's
chain-rule gradient, which the CPU tests pin to central finite differences."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from datagen import config4_thetas, make_section, make_section_pair

pytestmark = pytest.mark.gpu
GRAD_RTOL = 1e-3
TIE_REL = 2e-4


@pytest.fixture(scope="module")
def ctx():
    import paper_1612_04787_amd as sw
    c = sw.Swift(0)
    yield c
    c.close()


def dev():
    return torch.device("cuda", 0)


def normalised(g6, n):
    """Gradient in the parameterisation (a11 n/2, a12 n/2, tx, a21 n/2, a22 n/2, ty),
    in which a unit step moves no window pixel by more than one pixel."""
    s = np.array([2.0 / n, 2.0 / n, 1.0, 2.0 / n, 2.0 / n, 1.0])
    return np.asarray(g6, np.float64) * s


@pytest.fixture(scope="module")
def pair_small():
    a, b, _, _ = make_section_pair(1200, 1200, 41, 441, device="cpu", max_shift=4.0)
    return a, b


def _thetas(rng, k, n, size):
    ta = np.zeros((k, 8), np.float32)
    tb = np.zeros((k, 8), np.float32)
    for i in range(k):
        cx = rng.uniform(n / 2 + 20, size - n / 2 - 20)
        cy = rng.uniform(n / 2 + 20, size - n / 2 - 20)
        e = rng.uniform(-1e-3, 1e-3, 4)
        ta[i] = [cx, cy, 1 + e[0], e[1], rng.uniform(-0.5, 0.5), e[2], 1 + e[3], rng.uniform(-0.5, 0.5)]
        tb[i] = [cx, cy, 1, 0, rng.uniform(-1, 1), 0, 1, rng.uniform(-1, 1)]
    return ta, tb


@pytest.mark.parametrize("n", [64, 128, 256, 512])
@pytest.mark.parametrize("p", [0.65, 0.0, 1.0])
@pytest.mark.parametrize("gpgs", [(0.0, 1.0), (1.0, 0.0), (0.3, -0.7)])
def test_adjoint_matches_oracle(ctx, pair_small, n, p, gpgs):
    _adjoint_case(ctx, pair_small, n, p, gpgs)


@pytest.mark.parametrize("p,gpgs", [(0.65, (0.0, 1.0)), (1.0, (0.3, -0.7)), (0.0, (1.0, 0.0))])
def test_adjoint_matches_oracle_1024(ctx, pair_small, p, gpgs):
    """The plain adjoint (swift_match_backward) at 1024^2."""
    _adjoint_case(ctx, pair_small, 1024, p, gpgs)


def _adjoint_case(ctx, pair_small, n, p, gpgs):
    import paper_1612_04787_amd as sw
    gp, gs = gpgs
    print("case adjoint n=%d p=%g g=(%g,%g)" % (n, p, gp, gs), flush=True)
    a, b = pair_small
    rng = np.random.default_rng(7 * n + int(10 * p))
    k = 3 if n <= 256 else 2
    ta, tb = _thetas(rng, k, n, 1200)
    params = sw.make_params(p=p)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(ta), torch.from_numpy(tb), params,
                          save=True)
    gpk = torch.full((k,), gp, device=dev())
    gsn = torch.full((k,), gs, device=dev())
    ga, gb, hs = ctx.match_backward(res, params, gpk, gsn, want_hess=True)
    torch.cuda.synchronize()
    ga, gb, hs = ga.cpu().numpy(), gb.cpu().numpy(), hs.cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    checked = 0
    for i in range(k):
        rec, ra, rb = O.match_grad(an, bn, ta[i].astype(np.float64), tb[i].astype(np.float64), n,
                                   O.Params(p=p), g_peak=gp, g_snr=gs)
        if (rec["peak"] - rec["second"]) <= TIE_REL * abs(rec["peak"]):
            continue  # near-tie: the held-fixed peak may differ
        assert (int(res["ix"][i]), int(res["iy"][i])) == (rec["ix"], rec["iy"])
        if gpgs == (0.0, 1.0):
            c = O.match_pair(an, bn, ta[i].astype(np.float64), tb[i].astype(np.float64), n, O.Params(p=p),
                             return_surface=True)["surface"]
            href = np.array(O.surface_hessian(c, rec["iy"], rec["ix"]))
            herr = np.abs(hs[i] - href).max() / np.abs(href).max()
            print("    ", i, "hessian rel err %.2e" % herr, flush=True)
            assert herr <= 1e-3, (i, hs[i], href)
        for g_gpu, g_ref, tag in ((ga[i], ra, "A"), (gb[i], rb, "B")):
            x, y = normalised(g_gpu, n), normalised(g_ref, n)
            err = np.linalg.norm(x - y) / np.linalg.norm(y)
            print("   ", i, tag, "rel err %.2e" % err, flush=True)
            assert err <= GRAD_RTOL, (i, tag, err, x, y)
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("p", [0.65, 0.0, 1.0])
def test_centroid_jacobian_matches_oracle(ctx, pair_small, n, p):
    import paper_1612_04787_amd as sw
    print("case centroid jacobian n=%d p=%g" % (n, p), flush=True)
    a, b = pair_small
    rng = np.random.default_rng(5 * n + int(10 * p))
    k = 3 if n <= 256 else 2
    ta, tb = _thetas(rng, k, n, 1200)
    params = sw.make_params(p=p)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(ta), torch.from_numpy(tb), params,
                          save=True)
    jac = ctx.centroid_jacobian(res, params)
    torch.cuda.synchronize()
    jac = jac.cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    checked = 0
    for i in range(k):
        rec, ref = O.centroid_jacobian(an, bn, ta[i].astype(np.float64), tb[i].astype(np.float64), n,
                                       O.Params(p=p))
        if (rec["peak"] - rec["second"]) <= TIE_REL * abs(rec["peak"]):
            continue
        assert (int(res["ix"][i]), int(res["iy"][i])) == (rec["ix"], rec["iy"])
        for row in range(2):
            x, y = normalised(jac[i, row], n), normalised(ref[row], n)
            err = np.linalg.norm(x - y) / np.linalg.norm(y)
            print("   ", i, "d%s rel err %.2e" % ("xy"[row], err), flush=True)
            assert err <= GRAD_RTOL, (i, row, err, x, y)
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("n", [512, 1024])
def test_centroid_jacobian_translation_windows(ctx, pair_small, n):
    """Both windows at identity linear parts (the refinement's case): the
    adjoint's row pass then samples window A with one set of bilinear weights
    from its uint8 source tile (at 1024^2 four rows per workgroup)."""
    import paper_1612_04787_amd as sw
    print("case centroid jacobian, translation windows n=%d" % n, flush=True)
    a, b = pair_small
    rng = np.random.default_rng(17 * n)
    k = 2
    ta, tb = _thetas(rng, k, n, 1200)
    ta[:, [2, 3, 5, 6]] = [1, 0, 0, 1]
    params = sw.make_params(p=0.65)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(ta), torch.from_numpy(tb), params,
                          save=True)
    jac = ctx.centroid_jacobian(res, sw.make_params(p=0.65, flags=sw.FLAG_JAC_TRANSLATION)).cpu().numpy()
    an, bn = a.numpy(), b.numpy()
    checked = 0
    for i in range(k):
        rec, ref = O.centroid_jacobian(an, bn, ta[i].astype(np.float64), tb[i].astype(np.float64), n,
                                       O.Params(p=0.65))
        if (rec["peak"] - rec["second"]) <= TIE_REL * abs(rec["peak"]):
            continue
        assert (int(res["ix"][i]), int(res["iy"][i])) == (rec["ix"], rec["iy"])
        for row in range(2):
            x, y = jac[i, row, [2, 5]], np.asarray(ref[row], np.float64)[[2, 5]]
            err = np.linalg.norm(x - y) / np.linalg.norm(y)
            print("   ", i, "d%s/dt rel err %.2e" % ("xy"[row], err), flush=True)
            assert err <= GRAD_RTOL, (i, row, err, x, y)
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("n", [64, 256, 512, 1024])
def test_centroid_jacobian_translation_only(ctx, pair_small, n):
    """SWIFT_FLAG_JAC_TRANSLATION: the translation columns equal those of the
    full pass (same sums in the same order), the other four are zero; an
    unknown flag bit is refused."""
    import paper_1612_04787_amd as sw
    print("case centroid jacobian translation-only n=%d" % n, flush=True)
    a, b = pair_small
    rng = np.random.default_rng(11 * n)
    k = 3
    ta, tb = _thetas(rng, k, n, 1200)
    params = sw.make_params(p=0.65)
    res = ctx.match_batch([a.to(dev()), b.to(dev())], [n] * k, torch.zeros(k, dtype=torch.int32),
                          torch.ones(k, dtype=torch.int32), torch.from_numpy(ta), torch.from_numpy(tb), params,
                          save=True)
    full = ctx.centroid_jacobian(res, params).cpu().numpy()
    trans = ctx.centroid_jacobian(res, sw.make_params(p=0.65, flags=sw.FLAG_JAC_TRANSLATION)).cpu().numpy()
    np.testing.assert_array_equal(trans[:, :, [2, 5]], full[:, :, [2, 5]])
    assert not trans[:, :, [0, 1, 3, 4]].any()
    assert np.abs(full[:, :, [2, 5]]).max() > 0
    with pytest.raises(sw.SwiftError):
        ctx.centroid_jacobian(res, sw.make_params(p=0.65, flags=4))


def test_autograd_function(ctx, pair_small):
    import paper_1612_04787_amd as sw
    print("case autograd", flush=True)
    a, b = pair_small
    rng = np.random.default_rng(3)
    ta, tb = _thetas(rng, 3, 128, 1200)
    params = sw.make_params(p=0.65)
    tha = torch.from_numpy(ta).to(dev()).requires_grad_(True)
    thb = torch.from_numpy(tb).to(dev()).requires_grad_(True)
    imgs = [a.to(dev()), b.to(dev())]
    z = torch.zeros(3, dtype=torch.int32, device=dev())
    peak, snr = sw.SwiftMatchFn.apply(tha, thb, ctx, imgs, [128] * 3, z, z + 1, params)
    (snr.sum() + 0.5 * peak.sum()).backward()
    res = ctx.match_batch(imgs, [128] * 3, z, z + 1, tha.detach(), thb.detach(), params, save=True)
    ga, gb = ctx.match_backward(res, params, torch.full((3,), 0.5, device=dev()), torch.ones(3, device=dev()))
    torch.cuda.synchronize()
    g8a = tha.grad.cpu().numpy()
    ga = ga.cpu().numpy()
    np.testing.assert_allclose(g8a[:, [2, 3, 4, 5, 6, 7]], ga, rtol=1e-6, atol=0)
    np.testing.assert_allclose(g8a[:, 0], ga[:, 2], rtol=1e-6)
    np.testing.assert_allclose(g8a[:, 1], ga[:, 5], rtol=1e-6)


def test_config4_shape_sampled(ctx):
    """4096 windows of 256^2 on a 64 x 64 grid (256 px spacing) of a 16384^2
    uint8 section, window A at a perturbed affine (sub-pixel shift, |E| <= 1e-3),
    window B at identity; forward SNR + adjoint for all, 12 sampled windows
    checked against the oracle gradient."""
    import paper_1612_04787_amd as sw
    from datagen import window_grid
    print("case config4 generate", flush=True)
    sec = make_section(16384, 16384, 4, device=dev())
    torch.cuda.synchronize()
    cen = window_grid(16384, 16384, 256, 64, spacing=256)
    th = config4_thetas(len(cen))
    ta = np.zeros((len(cen), 8), np.float32)
    tb = np.zeros((len(cen), 8), np.float32)
    ta[:, 0:2] = cen
    ta[:, 2:] = th[:, [0, 1, 2, 3, 4, 5]]
    tb[:, 0:2] = cen
    tb[:, 2:] = [1, 0, 0, 0, 1, 0]
    P = len(cen)
    params = sw.make_params(p=0.65)
    z = torch.zeros(P, dtype=torch.int32, device=dev())
    print("case config4 forward+adjoint P=%d" % P, flush=True)
    res = ctx.match_batch([sec], [256] * P, z, z, torch.from_numpy(ta), torch.from_numpy(tb), params, save=True)
    ga, gb = ctx.match_backward(res, params, None, torch.ones(P, device=dev()))
    torch.cuda.synchronize()
    ga = ga.cpu().numpy()
    rng = np.random.default_rng(0)
    checked = 0
    for i in rng.choice(P, 12, replace=False):
        cx, cy = cen[i]
        x0, y0 = int(cx - 140), int(cy - 140)
        x0c, y0c = max(x0, 0), max(y0, 0)
        crop = sec[y0c:y0c + 280, x0c:x0c + 280].cpu().numpy()
        t_a = ta[i].astype(np.float64).copy()
        t_b = tb[i].astype(np.float64).copy()
        t_a[0] -= x0c
        t_a[1] -= y0c
        t_b[0] -= x0c
        t_b[1] -= y0c
        edge = x0 < 0 or y0 < 0 or x0 + 280 > 16384 or y0 + 280 > 16384
        if edge:
            continue  # the crop would change clamped reads at the section border
        rec, ra, _ = O.match_grad(crop, crop, t_a, t_b, 256, O.Params(p=0.65), g_peak=0.0, g_snr=1.0)
        if (rec["peak"] - rec["second"]) <= TIE_REL * abs(rec["peak"]):
            continue
        assert abs(float(res["snr"][i]) - rec["snr"]) <= 1e-3 * rec["snr"]
        x, y = normalised(ga[i], 256), normalised(ra, 256)
        err = np.linalg.norm(x - y) / np.linalg.norm(y)
        print("   window %d rel err %.2e" % (i, err), flush=True)
        assert err <= GRAD_RTOL, (i, err, x, y)
        checked += 1
    assert checked >= 6


def _fd_eligible(theta, n, h):
    """Every sample position of the window lies more than 2h from integer
    coordinates, so a step of h in the normalised parameters (which moves no
    sample by more than h) crosses no bilinear kink."""
    x, y, _, _ = O.swift_oracle.window_coords(theta, n)
    fx, fy = x - np.floor(x), y - np.floor(y)
    d = np.minimum(np.minimum(fx, 1 - fx), np.minimum(fy, 1 - fy))
    return float(d.min()) > 2 * h


def test_config4_fp32_central_fd(ctx):
    """Config 4 on fp32 windows: 4096 windows of 256^2 on a 64 x 64 grid of
    a 16384^2 fp32 section, window A at a perturbed affine (sub-pixel shift
    U(-0.5, 0.5), |E| <= 1e-3), B at identity; forward SNR and adjoint for the
    whole batch.  On sampled windows whose samples all lie more than 2h from
    integer coordinates, the GPU gradient of the SNR against FP64 central
    differences of the oracle's SNR, h = 1e-3 in the normalised parameters,
    within 1e-3 relative."""
    import paper_1612_04787_amd as sw
    from datagen import window_grid
    print("case config4 fp32 generate", flush=True)
    sec = make_section(16384, 16384, 4, device=dev()).float()
    torch.cuda.synchronize()
    n, h = 256, 1e-3
    cen = window_grid(16384, 16384, n, 64, spacing=256)
    th = config4_thetas(len(cen))
    P = len(cen)
    ta = np.zeros((P, 8), np.float32)
    tb = np.zeros((P, 8), np.float32)
    ta[:, 0:2] = cen
    ta[:, 2:] = th[:, [0, 1, 2, 3, 4, 5]]
    tb[:, 0:2] = cen
    tb[:, 2:] = [1, 0, 0, 0, 1, 0]
    params = sw.make_params(p=0.65)
    z = torch.zeros(P, dtype=torch.int32, device=dev())
    print("case config4 fp32 forward+adjoint P=%d" % P, flush=True)
    res = ctx.match_batch([sec], [n] * P, z, z, torch.from_numpy(ta), torch.from_numpy(tb), params, save=True)
    ga, _ = ctx.match_backward(res, params, None, torch.ones(P, device=dev()), want_b=False)
    torch.cuda.synchronize()
    ga = ga.cpu().numpy()
    step = np.array([2.0 / n, 2.0 / n, 1.0, 2.0 / n, 2.0 / n, 1.0])  # normalised -> raw parameter step
    idx6 = [2, 3, 4, 5, 6, 7]  # (a11, a12, tx, a21, a22, ty) in theta
    rng = np.random.default_rng(1)
    checked = eligible = 0
    for i in rng.permutation(P):
        if checked >= 6:
            break
        cx, cy = cen[i]
        x0, y0 = int(cx - 140), int(cy - 140)
        if x0 < 0 or y0 < 0 or x0 + 280 > 16384 or y0 + 280 > 16384:
            continue
        t_a = ta[i].astype(np.float64).copy()
        t_b = tb[i].astype(np.float64).copy()
        t_a[0:2] -= (x0, y0)
        t_b[0:2] -= (x0, y0)
        if not _fd_eligible(t_a, n, h):
            continue
        eligible += 1
        crop = sec[y0:y0 + 280, x0:x0 + 280].double().cpu().numpy()
        base = O.match_pair(crop, crop, t_a, t_b, n, O.Params(p=0.65))
        if (base["peak"] - base["second"]) <= TIE_REL * abs(base["peak"]):
            continue
        fd = np.zeros(6)
        for j in range(6):
            tp, tm = t_a.copy(), t_a.copy()
            tp[idx6[j]] += h * step[j]
            tm[idx6[j]] -= h * step[j]
            rp = O.match_pair(crop, crop, tp, t_b, n, O.Params(p=0.65))
            rm = O.match_pair(crop, crop, tm, t_b, n, O.Params(p=0.65))
            assert (rp["ix"], rp["iy"]) == (rm["ix"], rm["iy"]) == (base["ix"], base["iy"])
            fd[j] = (rp["snr"] - rm["snr"]) / (2 * h)
        g = normalised(ga[i], n)
        err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
        print("   window %d |fd| %.4g rel err %.2e" % (i, np.linalg.norm(fd), err), flush=True)
        assert err <= GRAD_RTOL, (i, err, g, fd)
        checked += 1
    print("   eligible windows visited", eligible, flush=True)
    assert checked >= 6


@pytest.mark.parametrize("p", [0.65, 1.0])
def test_adjoint_scale_invariance_fp32(ctx, p):
    """fp32 sources and the same sources times 1e3: the SNR gradient is
    unchanged (the SNR is invariant to intensity scale) and the peak gradient
    scales by 1e3^(2 - 2p)."""
    import paper_1612_04787_amd as sw
    print("case adjoint fp32 scale p=%g" % p, flush=True)
    a = make_section(700, 700, 81).float()
    b = torch.roll(a, shifts=(2, -3), dims=(0, 1)) + 3.0 * torch.randn((700, 700),
                                                                       generator=torch.Generator().manual_seed(8))
    rng = np.random.default_rng(5)
    ta, tb = _thetas(rng, 3, 256, 700)
    params = sw.make_params(p=p)
    z = torch.zeros(3, dtype=torch.int32)
    out = {}
    for scale in (1.0, 1e3):
        imgs = [(a * scale).to(dev()), (b * scale).to(dev())]
        res = ctx.match_batch(imgs, [256] * 3, z, z + 1, torch.from_numpy(ta), torch.from_numpy(tb), params,
                              save=True)
        g_snr, _ = ctx.match_backward(res, params, None, torch.ones(3, device=dev()), want_b=False)
        g_peak, _ = ctx.match_backward(res, params, torch.ones(3, device=dev()), None, want_b=False)
        torch.cuda.synchronize()
        out[scale] = (g_snr.cpu().numpy().astype(np.float64), g_peak.cpu().numpy().astype(np.float64))
    for i in range(3):
        s1, s2 = normalised(out[1.0][0][i], 256), normalised(out[1e3][0][i], 256)
        assert np.linalg.norm(s1 - s2) <= 1e-3 * np.linalg.norm(s1), (i, s1, s2)
        p1, p2 = normalised(out[1.0][1][i], 256), normalised(out[1e3][1][i], 256) / 1e3 ** (2 - 2 * p)
        assert np.linalg.norm(p1 - p2) <= 1e-3 * np.linalg.norm(p1), (i, p1, p2)
