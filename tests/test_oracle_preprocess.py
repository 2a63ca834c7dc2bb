"""Pins of the oracle's pre-processing (Sec. 2: high-pass background
removal, then contrast-limited adaptive histogram equalisation): scipy box
sums for the high-pass, textbook global histogram equalisation as the
unclipped one-tile case of CLAHE, closed forms for constant images, and a
vectorised numpy restatement of the whole CLAHE."""
import numpy as np
import pytest
from scipy.ndimage import convolve

import oracle


def hp_brute(I, r):
    I = np.asarray(I, np.int64)
    k = np.ones((2 * r + 1, 2 * r + 1), np.int64)
    S = convolve(I, k, mode="constant", cval=0)
    C = convolve(np.ones_like(I), k, mode="constant", cval=0)
    return np.maximum(I - S // C, 0)


@pytest.mark.parametrize("shape,r", [((37, 53), 3), ((64, 64), 7), ((5, 9), 6)])
def test_highpass_vs_scipy_box_sums(shape, r):
    I = np.random.default_rng(11).integers(0, 4096, shape)
    assert np.array_equal(oracle.highpass(I, r), hp_brute(I, r))


def test_highpass_removes_constant_and_ramp_background():
    assert (oracle.highpass(np.full((20, 30), 173), 4) == 0).all()
    # a particle on a constant background keeps its height above the local mean
    I = np.full((21, 21), 40)
    I[10, 10] = 240
    out = oracle.highpass(I, 3)
    assert out[10, 10] == 240 - (40 * 48 + 240) // 49
    assert out.sum() == out[10, 10]


def clahe_brute(I, bits, tx, ty, cf):
    I = np.asarray(I, np.int64)
    H, W = I.shape
    lb = min(bits, 12)
    nb, sh, mx = 1 << lb, bits - lb, (1 << bits) - 1
    xe = [(j * W) // tx for j in range(tx + 1)]
    ye = [(j * H) // ty for j in range(ty + 1)]
    luts = np.zeros((ty, tx, nb), np.int64)
    for j in range(ty):
        for i in range(tx):
            t = I[ye[j]:ye[j + 1], xe[i]:xe[i + 1]] >> sh
            n = t.size
            h = np.bincount(t.ravel(), minlength=nb).astype(np.int64)
            clip = max(1, int(np.floor(cf * n / nb)))
            ex = np.maximum(h - clip, 0).sum()
            h = np.minimum(h, clip) + ex // nb
            rest = ex % nb
            if rest:
                st = max(nb // rest, 1)
                h[np.arange(0, nb, st)[:rest]] += 1
            luts[j, i] = (np.cumsum(h) * mx + n // 2) // n
    cx = np.array([xe[i] + xe[i + 1] - 1 for i in range(tx)])
    cy = np.array([ye[j] + ye[j + 1] - 1 for j in range(ty)])

    def axis(X, c):
        a = np.clip(np.searchsorted(c, X, side="right") - 1, 0, len(c) - 1)
        inner = (X >= c[0]) & (a < len(c) - 1)
        b = np.where(inner, a + 1, a)
        w = np.where(inner, X - c[a], 0)
        d = np.where(inner, c[b] - c[a], 1)
        return a, b, w, d

    ys, xs = np.mgrid[0:H, 0:W]
    ia, ib, wx, dx = axis(2 * xs, cx)
    ja, jb, wy, dy = axis(2 * ys, cy)
    v = I >> sh
    L = lambda j, i: luts[j, i, v]
    num = (dy - wy) * ((dx - wx) * L(ja, ia) + wx * L(ja, ib)) + wy * ((dx - wx) * L(jb, ia) + wx * L(jb, ib))
    den = dx * dy
    return (num + den // 2) // den


@pytest.mark.parametrize("shape,bits,tx,ty,cf", [((64, 64), 8, 4, 4, 2.0), ((70, 90), 8, 8, 3, 1.5),
                                                  ((48, 40), 12, 3, 2, 2.5), ((33, 47), 16, 2, 3, 4.0),
                                                  ((32, 32), 8, 1, 1, 0.2)])
def test_clahe_vs_numpy_restatement(shape, bits, tx, ty, cf):
    rng = np.random.default_rng(12)
    # particle-like: mostly dark with bright spots (so clipping matters)
    I = rng.integers(0, 1 << min(bits, 6), shape)
    spots = rng.random(shape) < 0.05
    I[spots] = rng.integers(0, 1 << bits, int(spots.sum()))
    assert np.array_equal(oracle.clahe(I, bits, tx, ty, cf), clahe_brute(I, bits, tx, ty, cf))


def test_clahe_unclipped_single_tile_is_histogram_equalisation():
    """One tile and a clip limit above every bin: textbook histogram
    equalisation, out = round(cdf(v) * maxval / npix)."""
    I = np.random.default_rng(13).integers(0, 256, (50, 60))
    n = I.size
    cdf = np.cumsum(np.bincount(I.ravel(), minlength=256))
    expect = (cdf[I] * 255 + n // 2) // n
    assert np.array_equal(oracle.clahe(I, 8, 1, 1, 1e9), expect)


def test_clahe_constant_image_closed_form():
    """A constant tile: one bin holds every pixel; it is clipped to the limit
    c, the excess n - c is spread evenly, so the value's cdf is c +
    (v + 1) * ((n - c) // 256) plus the spread remainder bins at or below
    it; every tile is the same, so every pixel takes that one value."""
    v, n = 100, 32 * 32
    I = np.full((64, 64), v)
    c = oracle.clahe_clip(n, 256, 2.0)
    assert c == 8
    ex = n - c
    each, rest = ex // 256, ex % 256
    st = max(256 // rest, 1) if rest else 1
    extra = len([b for b in range(0, 256, st)][:rest]) if rest else 0
    extra_le = len([b for b in list(range(0, 256, st))[:rest] if b <= v]) if rest else 0
    cdf_v = c + each * (v + 1) + extra_le
    out = oracle.clahe(I, 8, 2, 2, 2.0)
    assert (out == (cdf_v * 255 + n // 2) // n).all()
    assert extra == rest


def test_clahe_is_monotone_in_the_input():
    """Within one tile, equalisation never reverses the order of values."""
    I = np.random.default_rng(14).integers(0, 256, (40, 40))
    out = oracle.clahe(I, 8, 1, 1, 2.0)
    o = np.argsort(I.ravel(), kind="stable")
    assert (np.diff(out.ravel()[o]) >= 0).all()
