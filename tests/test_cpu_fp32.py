"""The CPU FP32 baseline (oracle/cpu_fp32.py) against the FP64 oracle: the
same records within single-precision tolerances, on affine windows (one
partly outside the image) at three whitening exponents."""
import numpy as np
import pytest

import oracle as O
from oracle import cpu_fp32


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("p", [0.65, 1.0, 0.0])
def test_fp32_batch_matches_oracle(n, p):
    rng = np.random.default_rng(31 + n)
    base = rng.normal(0, 1, (420, 420))
    for _ in range(3):  # smooth the noise so windows have structure at several scales
        base = (base + np.roll(base, 1, 0) + np.roll(base, 1, 1) + np.roll(base, (1, 1), (0, 1))) / 4
    img_a = np.clip(128 + 400 * base, 0, 255).astype(np.uint8)
    img_b = np.roll(img_a, (3, -5), (0, 1))
    k = 5
    th = np.zeros((k, 8))
    for i in range(k):
        th[i] = [rng.uniform(n / 2 + 10, 410 - n / 2), rng.uniform(n / 2 + 10, 410 - n / 2),
                 1 + rng.uniform(-2e-3, 2e-3), rng.uniform(-2e-3, 2e-3), rng.uniform(-0.5, 0.5),
                 rng.uniform(-2e-3, 2e-3), 1 + rng.uniform(-2e-3, 2e-3), rng.uniform(-0.5, 0.5)]
    th[-1, :2] = [n / 2 - 3.5, 420 - n / 2 + 2.25]
    thb = th.copy()
    rec = cpu_fp32.match_batch(img_a, img_b, th, thb, n, p=p, workers=2)
    for i in range(k):
        r = O.match_pair(img_a.astype(np.float64), img_b.astype(np.float64), th[i], thb[i], n, O.Params(p=p))
        assert (rec["ix"][i], rec["iy"][i]) == (r["ix"], r["iy"]), (i, rec["ix"][i], rec["iy"][i], r["ix"], r["iy"])
        assert abs(rec["snr"][i] - r["snr"]) <= 1e-3 * abs(r["snr"]), (i, rec["snr"][i], r["snr"])
        assert abs(rec["dx"][i] - r["dx"]) <= 0.01 and abs(rec["dy"][i] - r["dy"]) <= 0.01, i
        assert abs(rec["peak"][i] - r["peak"]) <= 1e-4 * abs(r["peak"]), (i, rec["peak"][i], r["peak"])
