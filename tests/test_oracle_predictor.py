"""Pins of the oracle's predictor (pyramid, integer SAD search, median,
coarse-to-fine propagation) against closed forms and brute force."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2504_17987_amd import synth


def rand_img(rng, H, W, hi=256):
    return rng.integers(0, hi, (H, W)).astype(np.int32)


def shifted(A, dx, dy):
    """B(p) = A(p - d): content moved by d, zero where it enters."""
    H, W = A.shape
    B = np.zeros_like(A)
    ys, xs = np.mgrid[0:H, 0:W]
    sy, sx = ys - dy, xs - dx
    ok = (sy >= 0) & (sy < H) & (sx >= 0) & (sx < W)
    B[ok] = A[sy[ok], sx[ok]]
    return B


def test_pyramid_constant_and_brute():
    rng = np.random.default_rng(1)
    c = np.full((16, 20), 77, np.int32)
    assert (oracle.pyr_down(c) == 77).all()
    for H, W in [(13, 17), (8, 8), (1, 5), (31, 2)]:
        I = rand_img(rng, H, W)
        assert np.array_equal(oracle.pyr_down(I), brute.pyr_down(I))
    # u16 12-bit values
    I = rand_img(rng, 11, 9, 4096)
    assert np.array_equal(oracle.pyr_down(I), brute.pyr_down(I))
    # rounding: 1+1+1+2 = 5 -> floor(7/4) = 1 ; 1+2+2+2 = 7 -> floor(9/4) = 2
    assert oracle.pyr_down(np.array([[1, 1], [1, 2]]))[0, 0] == 1
    assert oracle.pyr_down(np.array([[1, 2], [2, 2]]))[0, 0] == 2


def test_sad_equal_images_give_zero():
    rng = np.random.default_rng(2)
    A = rand_img(rng, 64, 64)
    for levels in (1, 3):
        p = oracle.predict(A, A, 8, 16, levels, 4, 2)
        assert (p == 0).all()


@pytest.mark.parametrize("d", [(3, -2), (-5, 4), (0, 7)])
def test_sad_integer_shift_single_level(d):
    rng = np.random.default_rng(3)
    A = rand_img(rng, 64, 64)
    B = shifted(A, *d)
    p = oracle.predict(A, B, 8, 16, 1, 8, 0, median=False)
    # interior nodes: block and its shifted copy inside the image
    inner = (slice(2, 6), slice(2, 6))
    assert (p[0][inner] == d[0]).all() and (p[1][inner] == d[1]).all()


def test_sad_integer_shift_three_levels():
    rng = np.random.default_rng(4)
    # smooth-ish random texture so coarse levels keep structure
    from scipy.ndimage import gaussian_filter
    A = np.clip(gaussian_filter(rng.normal(128, 60, (128, 128)), 1.0), 0, 255).astype(np.int32)
    d = (9, -6)
    B = shifted(A, *d)
    p = oracle.predict(A, B, 8, 16, 3, 3, 2, median=True)
    # nodes whose coarse-level ancestors (block + search) stay inside the image
    inner = (slice(3, 13), slice(3, 11))
    assert (p[0][inner] == d[0]).all() and (p[1][inner] == d[1]).all()


def test_sad_tie_break():
    # A flat zero image: every candidate has SAD 0 against a zero B -> (0, 0)
    Z = np.zeros((32, 32), np.int32)
    assert (oracle.sad_level(Z, Z, 4, 4, 8, 8, 3) == 0).all()
    # two exact matches at equal |dx|+|dy|: a periodic pattern with period 2
    # in x gives SAD 0 at dx = -2, 0, +2 ... with cand (1, 0): candidates dx in
    # [-2, 4]; zero-SAD shifts dx = 0, 2 (and -2, 4); smallest L1 is dx = 0.
    A = np.tile(np.array([[10, 200]], np.int32), (32, 16))
    cand = np.zeros((2, 4, 4), np.int32)
    cand[0] = 1
    d = oracle.sad_level(A, A, 4, 4, 8, 8, 3, cand)
    inner = (slice(1, 3), slice(1, 3))
    assert (d[0][inner] == 0).all() and (d[1][inner] == 0).all()
    # candidates only at odd dx in [1, 3] (cand 2, R 1): dx=1 and 3 never
    # match; the ordering (SAD, L1, dy, dx) is checked against brute force
    cand[0] = 2
    assert np.array_equal(oracle.sad_level(A, A, 4, 4, 8, 8, 1, cand),
                          brute.sad_level(A, A, 4, 4, 8, 8, 1, cand))


def test_sad_vs_brute_random():
    rng = np.random.default_rng(5)
    for trial in range(3):
        A = rand_img(rng, 32, 32)
        B = shifted(A, int(rng.integers(-3, 4)), int(rng.integers(-3, 4)))
        B = np.clip(B + rng.integers(-20, 21, B.shape), 0, 255).astype(np.int32)
        for step, block, R in [(8, 8, 2), (4, 8, 3), (8, 16, 1)]:
            nx, ny = 32 // step, 32 // step
            cand = rng.integers(-2, 3, (2, ny, nx)).astype(np.int32)
            assert np.array_equal(oracle.sad_level(A, B, nx, ny, step, block, R, cand),
                                  brute.sad_level(A, B, nx, ny, step, block, R, cand))
            assert np.array_equal(oracle.sad_level(A, B, nx, ny, step, block, R),
                                  brute.sad_level(A, B, nx, ny, step, block, R))


def test_median_vs_brute():
    rng = np.random.default_rng(6)
    for ny, nx in [(5, 7), (1, 1), (2, 3), (4, 4)]:
        d = rng.integers(-9, 10, (2, ny, nx)).astype(np.int32)
        assert np.array_equal(oracle.median3_int(d), brute.median3_int(d))
    # a lone spike is removed by the 3x3 median
    d = np.zeros((2, 5, 5), np.int32)
    d[0, 2, 2] = 11
    assert (oracle.median3_int(d) == 0).all()


def test_predict_vs_brute_two_levels():
    A, B = synth.make_pair(32, 32, synth.Uniform(2.0, -1.0), 0.06, seed=9)
    for median in (True, False):
        a = oracle.predict(A, B, 4, 8, 2, 2, 1, median)
        b = brute.predict(A, B, 4, 8, 2, 2, 1, median)
        assert np.array_equal(a, b)


def test_grid_counts_for_configs():
    # one vector per step^2 pixels: nx*ny = W*H/step^2 for every workload
    for W, H, step in [(256, 256, 16), (1024, 1024, 8), (3840, 2160, 12), (512, 512, 8),
                       (2048, 2048, 8)]:
        X, Y = synth.node_centres(W, H, step)
        assert X.size == W * H // step ** 2
