"""Error bounds of the scaled two-way fp16 split that the MFMA passes use for every
float32 product (checked on the host with NumPy's round-to-nearest-even float16).

A value x of a scale group whose largest magnitude is mx is scaled by 2^s, with
s = 15 - e for mx = m 2^e, m in [0.5, 1), so the group's largest scaled magnitude lies in
[2^14, 2^15); then hi = fp16(y), lo = fp16(y - hi).  Claims (stated where the kernels
define the split): |y - hi - lo| <= 2^-22 |y| for |y| >= 2^-3, an absolute error below
2^-25 otherwise, and a product formed from hi*hi + hi*lo + lo*hi within 3 * 2^-22 of the
exact one for operands in the full-accuracy window.
"""

import numpy as np


def _scale_exp(mx):
    if not mx > 0:
        return 0
    _, e = np.frexp(np.float32(mx))
    return int(min(126, max(-113, 15 - e)))


def _split(y32):
    hi = y32.astype(np.float16)
    lo = (y32 - hi.astype(np.float32)).astype(np.float16)
    return hi, lo


def _group(rng, n, spread):
    """float32 values whose magnitudes spread over 2^-spread .. 1 of their maximum."""
    mag = np.exp2(-rng.uniform(0, spread, n)) * np.exp2(rng.uniform(-40, 40))
    return (mag * rng.uniform(0.5, 1.0, n)).astype(np.float32)


def test_scaled_group_maximum_lies_in_window():
    rng = np.random.default_rng(1)
    for _ in range(200):
        x = _group(rng, 64, 10)
        s = _scale_exp(float(x.max()))
        y = x.astype(np.float64) * 2.0 ** s
        assert 2.0 ** 14 <= y.max() < 2.0 ** 15
        assert np.isfinite(y.astype(np.float32).astype(np.float16)).all()  # no fp16 overflow


def test_representation_error_bounds():
    rng = np.random.default_rng(2)
    for _ in range(200):
        x = _group(rng, 256, 30)  # spans the full-accuracy window and below it
        s = _scale_exp(float(x.max()))
        y = (x.astype(np.float64) * 2.0 ** s).astype(np.float32)  # exact: a power of two
        hi, lo = _split(y)
        err = np.abs(y.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
        big = np.abs(y) >= 2.0 ** -3
        assert np.all(err[big] <= 2.0 ** -22 * np.abs(y[big].astype(np.float64)))
        assert np.all(err[~big] <= 2.0 ** -25)


def test_three_product_form_is_float32_accurate():
    rng = np.random.default_rng(3)
    for _ in range(100):
        a = _group(rng, 512, 16)
        b = _group(rng, 512, 16)
        ya = (a.astype(np.float64) * 2.0 ** _scale_exp(float(a.max()))).astype(np.float32)
        yb = (b.astype(np.float64) * 2.0 ** _scale_exp(float(b.max()))).astype(np.float32)
        ah, al = (t.astype(np.float64) for t in _split(ya))
        bh, bl = (t.astype(np.float64) for t in _split(yb))
        approx = ah * bh + ah * bl + al * bh  # each piece product is exact in float32
        exact = ya.astype(np.float64) * yb.astype(np.float64)
        ok = (np.abs(ya) >= 2.0 ** -3) & (np.abs(yb) >= 2.0 ** -3)
        assert np.all(np.abs(approx - exact)[ok] <= 3 * 2.0 ** -22 * np.abs(exact[ok]))
        # the piece products are exact in float32 (11 x 11 significant bits)
        for p in (ah * bh, ah * bl, al * bh):
            assert np.array_equal(p.astype(np.float32).astype(np.float64), p)
