"""Helpers shared by the GPU parity tests: the tolerances of the match path and
the comparison of GPU records with oracle records."""
import numpy as np

import oracle as O

# Tolerances (floating point): surface within 1e-4 of the peak value, sub-pixel
# shift within 0.01 px, SNR within 1e-3 relative.  Integer peaks are bit-exact
# unless the oracle's best and second-best values are within 2e-4 relative,
# where either index is a correct answer (repeating content has several).
SURF_TOL = 1e-4
SUBPIX_TOL = 0.01
SNR_RTOL = 1e-3
TIE_REL = 2e-4


def gpu_record(res, k):
    return {key: (res[key][k].item()) for key in ("dx", "dy", "ix", "iy", "peak", "snr", "mean", "std", "status", "n")}


def oracle_record(imgA, imgB, thA, thB, n, params, surface=False):
    return O.match_pair(imgA, imgB, np.asarray(thA, np.float64), np.asarray(thB, np.float64), n, params,
                        return_surface=surface)


def compare(g, r, n, surf_gpu=None, tag=""):
    """Asserts the GPU record g matches the oracle record r.  Returns a dict of
    the observed errors."""
    peak = r["peak"]
    margin = (peak - r["second"]) / max(abs(peak), 1e-30)
    tie = margin <= TIE_REL
    out = {"tie": tie}
    if r["std"] == 0.0:
        assert g["status"] & O.swift_oracle.STATUS_DEGENERATE, (tag, g)
        assert g["snr"] == 0.0, (tag, g)
        return out
    if not tie:
        assert (g["ix"], g["iy"]) == (r["ix"], r["iy"]), (tag, g, r["ix"], r["iy"], margin)
        out["ddx"] = abs(g["dx"] - r["dx"])
        out["ddy"] = abs(g["dy"] - r["dy"])
        assert out["ddx"] <= SUBPIX_TOL and out["ddy"] <= SUBPIX_TOL, (tag, g, r["dx"], r["dy"])
    else:
        # either index is correct: it must be one of the near-maximal positions
        c = r.get("surface")
        if c is not None:
            assert c[g["iy"], g["ix"]] >= peak - 2 * TIE_REL * abs(peak) - SURF_TOL * abs(peak), (tag, g)
    out["snr_rel"] = abs(g["snr"] - r["snr"]) / max(abs(r["snr"]), 1e-12)
    assert out["snr_rel"] <= SNR_RTOL, (tag, g["snr"], r["snr"])
    assert abs(g["mean"] - r["mean"]) <= SURF_TOL * abs(peak), (tag, g["mean"], r["mean"])
    assert abs(g["std"] - r["std"]) <= SNR_RTOL * r["std"], (tag, g["std"], r["std"])
    assert (g["status"] & O.swift_oracle.STATUS_CLAMPED) == (r["status"] & O.swift_oracle.STATUS_CLAMPED), (tag,)
    if surf_gpu is not None and "surface" in r:
        err = np.abs(surf_gpu.astype(np.float64) - r["surface"]).max() / abs(peak)
        out["surf"] = err
        assert err <= SURF_TOL, (tag, err)
    return out
