"""The FP16 split behind the default C64 scan, checked on the CPU with numpy's IEEE binary16.

An FP32 operand x (after the exact power-of-two scaling that puts it in [2^-1, 2^13] in magnitude,
as the eigen kernel does for B and the steering table for a) is split as hi = fp16(x),
lo = fp16(x - hi); the matrix cores then form a b as hi_a hi_b + hi_a lo_b + lo_a hi_b.  The
header of the library states the bounds |x - hi - lo| <= 2^-22 |x| + 2^-25 and a neglected part
below 2^-20 |a b| + 2^-25 (|a| + |b|); this test checks them, and that the split dot product of a
real-embedded steering vector with a unit-norm B column is as accurate as the FP32 dot product.
"""

import numpy as np


def _split(x):
    hi = x.astype(np.float16).astype(np.float64)
    lo = (x - hi).astype(np.float16).astype(np.float64)
    return hi, lo


def test_split_residual_bound():
    rng = np.random.default_rng(20071413)
    # FP32 values over the scaled range of the operands
    x = (rng.uniform(0.5, 1.0, 200000) * 2.0 ** rng.integers(-30, 13, 200000)).astype(np.float32).astype(np.float64)
    x *= rng.choice([-1.0, 1.0], x.size)
    hi, lo = _split(x)
    r = np.abs(x - hi - lo)
    assert np.all(r <= 2.0 ** -22 * np.abs(x) + 2.0 ** -25)
    # above the FP16 normal range of lo the bound is relative alone
    big = np.abs(x) >= 2.0 ** -2
    assert np.all(r[big] <= 2.0 ** -22 * np.abs(x[big]))


def test_three_product_bound():
    rng = np.random.default_rng(7)
    a = (rng.uniform(-1, 1, 100000) * 8192.0).astype(np.float32).astype(np.float64)
    b = (rng.uniform(-1, 1, 100000) * 8192.0).astype(np.float32).astype(np.float64)
    ha, la = _split(a)
    hb, lb = _split(b)
    p3 = ha * hb + ha * lb + la * hb            # each product exact in FP64
    assert np.all(np.abs(a * b - p3) <= 2.0 ** -20 * np.abs(a * b) + 2.0 ** -25 * (np.abs(a) + np.abs(b)))


def test_split_dot_matches_fp32_accuracy():
    rng = np.random.default_rng(11)
    M = 16
    errs_split, errs_f32 = [], []
    for _ in range(2000):
        th = rng.uniform(-np.pi / 2, np.pi / 2)
        ph = np.pi * np.arange(M) * np.sin(th)
        a = np.concatenate([np.cos(ph), np.sin(ph)]).astype(np.float32).astype(np.float64)
        bc = rng.standard_normal(M) + 1j * rng.standard_normal(M)
        bc /= np.linalg.norm(bc)
        brow = np.concatenate([bc.real, bc.imag])
        exact = float(np.dot(brow, a))
        # split: steering scaled by 2^13, B by 2^e with its largest entry in [2^12, 2^13)
        sb = 2.0 ** (12 - np.floor(np.log2(np.abs(brow).max())))
        ha, la = _split(a * 8192.0)
        hb, lb = _split(brow * sb)
        acc = np.float32(0.0)
        for k0 in range(0, 2 * M, 16):            # FP32 accumulation per 16-deep step
            sl = slice(k0, k0 + 16)
            acc = np.float32(acc + np.float32(np.sum(hb[sl] * ha[sl] + hb[sl] * la[sl] + lb[sl] * ha[sl])))
        errs_split.append(abs(float(acc) / (8192.0 * sb) - exact))
        acc32 = np.float32(0.0)
        b32, a32 = brow.astype(np.float32), a.astype(np.float32)
        for k in range(2 * M):
            acc32 = np.float32(acc32 + b32[k] * a32[k])
        errs_f32.append(abs(float(acc32) - exact))
    # same order of error as FP32 operands (absolute, |b| = 1, |a_k| <= 1)
    assert max(errs_split) < 4.0 * max(errs_f32)
    assert max(errs_split) < 1e-6


def test_unit_roundoffs_of_the_16_bit_formats():
    # The 16-bit scan bounds use u = 2^-8 for bfloat16 (8 significant bits) and 2^-11 for IEEE
    # half (11 significant bits): the largest relative rounding error of FP32 values reaches each
    # (just above a power of two) and never exceeds it.  Conversions: torch's bfloat16 and numpy's
    # binary16, both round to nearest even.
    import torch
    rng = np.random.default_rng(7)
    x = (rng.uniform(1.0, 2.0, 400000) * 2.0 ** rng.integers(-10, 10, 400000)).astype(np.float32)
    xb = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    rb = np.abs(xb - x) / np.abs(x)
    assert rb.max() <= 2.0 ** -8 and rb.max() > 0.99 * 2.0 ** -8
    xh = x.astype(np.float16).astype(np.float64)
    rh = np.abs(xh - x) / np.abs(x)
    assert rh.max() <= 2.0 ** -11 and rh.max() > 0.99 * 2.0 ** -11


def _split3(x):
    parts = []
    r = np.asarray(x, dtype=np.float64)
    for _ in range(3):
        p = r.astype(np.float16).astype(np.float64)
        parts.append(p)
        r = r - p                                 # exact in FP64
    return parts


def test_three_part_split_reproduces_fp32_operands():
    # Steering values: FP32 v scaled by 2^13.  Three FP16 parts hold 33 significant bits, so every
    # scaled FP32 value of magnitude >= 1/2 is reproduced exactly; below, the remainder is under half
    # the FP16 subnormal spacing, 2^-25.  B from FP64: residual <= 2^-33 |x| + 2^-25.
    rng = np.random.default_rng(20071413)
    v = (rng.uniform(0.5, 1.0, 300000) * 2.0 ** rng.integers(-40, 1, 300000)).astype(np.float32)
    v *= rng.choice(np.array([-1.0, 1.0], dtype=np.float32), v.size)
    x = v.astype(np.float64) * 8192.0
    h, m, l = _split3(x)
    r = np.abs(x - h - m - l)
    big = np.abs(x) >= 0.5
    assert np.all(r[big] == 0.0)
    assert np.all(r <= 2.0 ** -25)
    # from FP64 values in the scaled range of B
    y = rng.uniform(0.5, 1.0, 300000) * 2.0 ** rng.integers(-30, 13, 300000) * rng.choice([-1.0, 1.0], 300000)
    h, m, l = _split3(y)
    assert np.all(np.abs(y - h - m - l) <= 2.0 ** -33 * np.abs(y) + 2.0 ** -25)
    # at the scale of a B column (largest component in [2^12, 2^13)) that is far below the FP32
    # rounding the FP32-operand kernel applies to the same values: worst residual 2^-20 against
    # FP32's 2^-13 near the top of the range, and a mean 100 times smaller
    f32err = np.abs(y.astype(np.float32).astype(np.float64) - y)
    res = np.abs(y - h - m - l)
    assert res.max() <= 2.0 ** -20 and f32err.max() >= 2.0 ** -14
    assert res.mean() < 1e-2 * f32err.mean()


def test_six_product_bound():
    # products of the parts whose orders add up to at most two; the dropped ones are below
    # 2^-33 |a b| plus the subnormal terms 2^-25 (|a| + |b|)
    rng = np.random.default_rng(9)
    a = (rng.uniform(-1, 1, 200000) * 8192.0).astype(np.float32).astype(np.float64)
    b = rng.uniform(-1, 1, 200000) * 8192.0
    pa, pb = _split3(a), _split3(b)
    p6 = sum(pa[i] * pb[j] for i in range(3) for j in range(3) if i + j <= 2)
    exact = np.array([float(np.longdouble(ai) * np.longdouble(bi)) for ai, bi in zip(a[:2000], b[:2000])])
    bound = 2.0 ** -33 * np.abs(a * b) + 2.0 ** -25 * (np.abs(a) + np.abs(b))
    assert np.all(np.abs(exact - p6[:2000]) <= bound[:2000] + 2.0 ** -52 * np.abs(exact))
    # a b reconstructed from the kept products is as close to a b as FP32 can represent it
    assert np.all(np.abs(a * b - p6) <= 2.0 ** -30 * np.abs(a * b) + 2.0 ** -24 * (np.abs(a) + np.abs(b)))


def test_three_part_split_dot_at_least_fp32_accurate():
    # the scan's dot product on three-part operands (six products per step, FP32 accumulation of
    # 16-deep steps) against FP32 operands, on real-embedded steering vectors and unit B columns
    rng = np.random.default_rng(13)
    M = 16
    e6, e32 = [], []
    for _ in range(2000):
        th = rng.uniform(-np.pi / 2, np.pi / 2)
        ph = np.pi * np.arange(M) * np.sin(th)
        a = np.concatenate([np.cos(ph), np.sin(ph)]).astype(np.float32).astype(np.float64)
        bc = rng.standard_normal(M) + 1j * rng.standard_normal(M)
        bc /= np.linalg.norm(bc)
        brow = np.concatenate([bc.real, bc.imag])
        exact = float(np.dot(brow, a))
        sb = 2.0 ** (12 - np.floor(np.log2(np.abs(brow).max())))
        pa, pb = _split3(a * 8192.0), _split3(brow * sb)
        acc = np.float32(0.0)
        for k0 in range(0, 2 * M, 16):
            sl = slice(k0, k0 + 16)
            for i in range(3):
                for j in range(3):
                    if i + j <= 2:
                        acc = np.float32(acc + np.float32(np.sum(pb[i][sl] * pa[j][sl])))
        e6.append(abs(float(acc) / (8192.0 * sb) - exact))
        acc32 = np.float32(0.0)
        b32, a32 = brow.astype(np.float32), a.astype(np.float32)
        for k in range(2 * M):
            acc32 = np.float32(acc32 + b32[k] * a32[k])
        e32.append(abs(float(acc32) - exact))
    assert max(e6) <= 1.5 * max(e32) and np.mean(e6) <= 1.5 * np.mean(e32)
