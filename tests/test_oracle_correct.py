"""Pins of the oracle's deformation and correlation stage (displacement
interpolation, bilinear warp, Pearson coefficient, argmax and Gaussian
sub-pixel fit) against closed forms, library routines and brute force."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2504_17987_amd import synth


def test_interp_exact_at_nodes_and_linear():
    rng = np.random.default_rng(11)
    step, nx, ny = 8, 5, 4
    U = rng.normal(0, 3, (2, ny, nx))
    for a in range(ny):
        for b in range(nx):
            x, y = b * step + (step - 1) / 2, a * step + (step - 1) / 2
            u, v = oracle.interp(U, step, x, y)
            assert u == U[0, a, b] and v == U[1, a, b]
    # a linear field is reproduced inside the node hull
    X, Y = synth.node_centres(nx * step, ny * step, step)
    L = np.stack([0.3 * X - 0.2 * Y + 1.0, -0.1 * X + 0.05 * Y])
    for x, y in rng.uniform([3.5, 3.5], [(nx - 1) * step + 3.5, (ny - 1) * step + 3.5], (50, 2)):
        u, v = oracle.interp(L, step, x, y)
        assert abs(u - (0.3 * x - 0.2 * y + 1.0)) < 1e-12
        assert abs(v - (-0.1 * x + 0.05 * y)) < 1e-12
    # outside the hull the value is held at the edge
    assert oracle.interp(L, step, -50.0, 3.5)[0] == L[0, 0, 0]
    assert oracle.interp(L, step, 1e4, 1e4)[1] == L[1, -1, -1]


def test_interp_vs_scipy():
    rng = np.random.default_rng(12)
    U = rng.normal(0, 3, (2, 4, 6))
    xs = rng.uniform(-10, 60, 40)
    ys = rng.uniform(-10, 40, 40)
    bu, bv = brute.displacement_at(U, 8, xs, ys)
    for i in range(40):
        u, v = oracle.interp(U, 8, xs[i], ys[i])
        assert abs(u - bu[i]) < 1e-12 and abs(v - bv[i]) < 1e-12


def test_warp_closed_forms_and_scipy():
    rng = np.random.default_rng(13)
    B = rng.integers(0, 256, (32, 40)).astype(float)
    Z = np.zeros((2, 4, 5))
    assert np.array_equal(oracle.warp_image(B, 1, 0, Z, 8), B)
    # integer uniform displacement: an exact shift with zeros entering
    Ui = np.zeros((2, 4, 5))
    Ui[0], Ui[1] = 3, -2
    W = oracle.warp_image(B, 1, 0, Ui, 8)
    ref = np.zeros_like(B)
    ref[2:, :-3] = B[:-2, 3:]
    assert np.array_equal(W, ref)
    # central mode: A'(p) = A(p - u/2), B'(p) = B(p + u/2); with u = (2, -4):
    Uc = np.zeros((2, 4, 5))
    Uc[0], Uc[1] = 2, -4
    Wa = oracle.warp_image(B, 0, 1, Uc, 8)
    refa = np.zeros_like(B)
    refa[:-2, 1:] = B[2:, :-1]
    assert np.array_equal(Wa, refa)
    # random field vs scipy map_coordinates (grid-constant zero padding)
    U = rng.normal(0, 2.5, (2, 4, 5))
    for which, mode in [(1, 0), (0, 1), (1, 1)]:
        W = oracle.warp_image(B, which, mode, U, 8)
        R = brute.warped_region(B, which, mode, U, 8, 0, 0, 32, 40)
        assert np.abs(W - R).max() < 1e-9


def test_gauss3_recovers_gaussian_peak():
    for (a, w) in [(0.3, 0.9), (-0.45, 1.4), (0.0, 0.7), (0.12, 2.0)]:
        c = [math.exp(-((s - a) ** 2) / (2 * w * w)) for s in (-1, 0, 1)]
        d, nc = oracle.gauss3(*c)
        assert not nc and abs(d - a) < 1e-12
    # a flat or convex triple has no curvature
    assert oracle.gauss3(0.5, 0.5, 0.5) == (0.0, True)
    assert oracle.gauss3(-0.2, -0.4, 0.0)[1]       # floored to 1e-3: equal logs
    assert oracle.gauss3(0.9, 0.1, 0.9)[1]


def test_gaussian_plane_through_correct():
    """An image pair whose windows correlate as a sampled Gaussian: a single
    smooth Gaussian blob shifted by a sub-pixel amount.  The peak index is
    the rounded shift and the sub-pixel estimate is close to the truth."""
    H = W = 48
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    A = 200 * np.exp(-((xs - 23.5) ** 2 + (ys - 23.5) ** 2) / (2 * 2.0 ** 2))
    B = 200 * np.exp(-((xs - 25.2) ** 2 + (ys - 22.9) ** 2) / (2 * 2.0 ** 2))
    disp, peak, flags = oracle.correct(A, B, 16, 8, 4, None)
    a = b = 2  # window centred on the blob
    assert abs(disp[0, a, b] - 1.7) < 0.05 and abs(disp[1, a, b] + 0.6) < 0.05
    assert flags[a, b] == 0


def test_rho_bounds_and_exact_match():
    rng = np.random.default_rng(14)
    A = rng.integers(0, 256, (48, 48)).astype(float)
    B = np.zeros_like(A)
    B[2:, :-3] = A[:-2, 3:]   # B(p) = A(p + (3, -2)) : content moved by (-3, +2)
    rho = oracle.corr_plane(A, B, 16, 8, 4, 0, None, 2, 2)
    assert (np.abs(rho) <= 1 + 1e-12).all()
    assert abs(rho[2 + 4, -3 + 4] - 1.0) < 1e-12
    assert np.unravel_index(np.argmax(rho), rho.shape) == (6, 1)


def test_corr_plane_vs_numpy_corrcoef():
    rng = np.random.default_rng(15)
    A, B = synth.make_pair(40, 40, synth.Uniform(1.3, -0.7), 0.08, seed=3)
    pred = rng.normal(0, 1.5, (2, 5, 5))
    for mode in (0, 1):
        for (a, b) in [(0, 0), (2, 3), (4, 4)]:
            r1 = oracle.corr_plane(A, B, 16, 8, 3, mode, pred, a, b)
            r2 = brute.corr_plane(A, B, 16, 8, 3, mode, pred, a, b)
            assert np.abs(r1 - r2).max() < 1e-10


def test_argmax_order_and_fit_vs_brute():
    """The corrected vector equals pred + argmax (python tuple ordering of
    (-rho, L1, sy, sx)) + Gaussian fits computed here from the brute plane."""
    rng = np.random.default_rng(16)
    A, B = synth.make_pair(48, 48, synth.Uniform(2.6, -1.2), 0.05, seed=5)
    pred = np.zeros((2, 6, 6))
    pred[0] = 1
    disp, peak, flags = oracle.correct(A, B, 16, 8, 4, pred)
    for (a, b) in [(1, 1), (2, 4), (3, 3), (0, 5)]:
        rho = brute.corr_plane(A, B, 16, 8, 4, 0, pred, a, b)
        keys = [(-rho[sy + 4, sx + 4], abs(sx) + abs(sy), sy, sx)
                for sy in range(-4, 5) for sx in range(-4, 5)]
        _, _, sy, sx = min(keys)
        assert abs(peak[a, b] - rho[sy + 4, sx + 4]) < 1e-10
        ex = 0.0 if abs(sx) == 4 else oracle.gauss3(rho[sy + 4, sx + 3], rho[sy + 4, sx + 4], rho[sy + 4, sx + 5])[0]
        ey = 0.0 if abs(sy) == 4 else oracle.gauss3(rho[sy + 3, sx + 4], rho[sy + 4, sx + 4], rho[sy + 5, sx + 4])[0]
        assert abs(disp[0, a, b] - (1 + sx + ex)) < 1e-9
        assert abs(disp[1, a, b] - (sy + ey)) < 1e-9
        assert bool(flags[a, b] & oracle.BORDER) == (abs(sx) == 4 or abs(sy) == 4)


def test_gain_offset_invariance():
    A, B = synth.make_pair(64, 64, synth.Uniform(1.4, 0.8), 0.05, seed=21)
    A = A.astype(float)
    B = B.astype(float)
    d1, p1, f1 = oracle.correct(A, B, 16, 8, 3, None)
    d2, p2, f2 = oracle.correct(A, 2 * B + 10, 16, 8, 3, None)
    # windows whose search stays inside the image (the zero padding outside is
    # not transformed): nodes 1..6 need pixels -4-3 .. ; take nodes 1..6
    inner = (slice(None), slice(1, 7), slice(1, 7))
    assert np.abs(d1[inner] - d2[inner]).max() < 1e-9
    assert np.abs(p1[1:7, 1:7] - p2[1:7, 1:7]).max() < 1e-12


def test_flat_images():
    Z = np.zeros((32, 32))
    disp, peak, flags = oracle.correct(Z, Z, 16, 8, 2, None)
    assert (flags & oracle.FLAT).all() and (disp == 0).all() and (peak == 0).all()
    C = np.full((32, 32), 9.0)
    disp, peak, flags = oracle.correct(C, C, 16, 8, 2, None)
    # interior windows see a constant: flat.  The two modes agree.
    assert flags[1, 1] & oracle.FLAT
    d2, _, f2 = oracle.correct(Z, Z, 16, 8, 2, None, peak_mode=1)
    assert (f2 & oracle.FLAT).all() and (d2 == 0).all()


def test_fixed_centre_stencil():
    """Paper's a-priori stencil: centre at zero shift, offset from the five
    points, clamped to [-1, 1]."""
    A, B = synth.make_pair(64, 64, synth.Uniform(0.35, -0.25), 0.06, seed=31)
    d, pk, fl = oracle.correct(A, B, 16, 8, 4, None, peak_mode=1)
    rho = brute.corr_plane(A, B, 16, 8, 1, 0, None, 3, 3)
    ex = oracle.gauss3(rho[1, 0], rho[1, 1], rho[1, 2])[0]
    ey = oracle.gauss3(rho[0, 1], rho[1, 1], rho[2, 1])[0]
    assert abs(d[0, 3, 3] - ex) < 1e-10 and abs(d[1, 3, 3] - ey) < 1e-10
    assert abs(pk[3, 3] - rho[1, 1]) < 1e-10
    assert (np.abs(d) <= 1).all() and not (fl & oracle.BORDER).any()
    inner = (slice(None), slice(1, 7), slice(1, 7))
    assert abs(d[inner][0].mean() - 0.35) < 0.05 and abs(d[inner][1].mean() + 0.25) < 0.05


def _interior(ny, nx, m):
    return (slice(m, ny - m), slice(m, nx - m))


@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_config1_uniform_recovery(seed):
    """256x256, 32/16 windows, +-8, zero predictor: the peak index is the
    rounded shift everywhere inside, the sub-pixel error is small.  Bounds
    calibrated on this oracle (see the accuracy table of the design notes)."""
    A, B, flow = synth.cfg1_pair(seed)
    disp, peak, flags = oracle.correct(A, B, 32, 16, 8, None)
    inner = _interior(16, 16, 1)
    eu = disp[0][inner] - 3.4
    ev = disp[1][inner] + 1.7
    assert not (flags[inner] & (oracle.FLAT | oracle.BORDER)).any()
    assert abs(eu.mean()) < 0.01 and abs(ev.mean()) < 0.01
    assert math.sqrt((eu ** 2).mean()) < 0.03 and math.sqrt((ev ** 2).mean()) < 0.03
    assert np.abs(eu).max() < 0.12 and np.abs(ev).max() < 0.12
    # integer peak = nearest integer shift
    assert (np.rint(disp[0][inner]) == 3).all() and (np.rint(disp[1][inner]) == -2).all()


def test_zero_displacement_gives_zero():
    A, _, _ = synth.cfg1_pair(1000)
    disp, peak, flags = oracle.correct(A, A, 32, 16, 8, None)
    inner = _interior(16, 16, 1)
    assert (np.rint(disp[:, 1:15, 1:15]) == 0).all()
    assert (peak[inner] > 1 - 1e-12).all()
    assert abs(disp[0][inner].mean()) < 0.01 and np.abs(disp[:, 1:15, 1:15]).max() < 0.1


def test_composition_is_window_mean_of_predictor():
    """Blank frames give no correlation (FLAT, zero shift, no fit), so the
    result is exactly the base the correction is added to: the mean over the
    window of the interpolated predictor (scipy's bilinear interpolation
    averaged over the window's pixels), which for 50% overlap equals the
    separable (1/4, 1/2, 1/4) node stencil inside and (3/4, 1/4) at edges."""
    rng = np.random.default_rng(17)
    P = rng.integers(-5, 6, (2, 6, 7)).astype(float)
    Z = np.zeros((48, 56))
    d, pk, fl = oracle.correct(Z, Z, 16, 8, 2, P)
    assert (fl & oracle.FLAT).all()
    ys, xs = np.mgrid[-4:12, -4:12].astype(float)
    w = lambda i, n: ({0: [0, .75, .25], n - 1: [.25, .75, 0]}.get(i, [.25, .5, .25]))
    for a in range(6):
        for b in range(7):
            u, v = brute.displacement_at(P, 8, xs + 8 * b, ys + 8 * a)
            assert abs(d[0, a, b] - u.mean()) < 1e-12 and abs(d[1, a, b] - v.mean()) < 1e-12
            st = np.outer(w(a, 6), w(b, 7))
            Pp = np.pad(P, ((0, 0), (1, 1), (1, 1)))
            ref = (st * Pp[0, a:a + 3, b:b + 3]).sum()
            assert abs(d[0, a, b] - ref) < 1e-12


def test_window_mean_composition_beats_node_value_on_solid_body():
    """Why the correction is added to the window mean of the interpolated
    predictor rather than to its node value: with an integer predictor on a
    solid-body rotation (linear field, so the window mean of the truth is the
    node's truth), adding the correlation's residual shift to the node value
    mixes the deformation applied across the window with the node's own
    rounding.  The window-mean reading must be the more accurate one against
    the analytic truth (interior nodes)."""
    W, H = 256, 192
    flow = synth.SolidBody((W - 1) / 2, (H - 1) / 2, 0.04)
    A, B = synth.make_pair(W, H, flow, 0.04, noise=2.0, seed=81)
    pred = oracle.predict(A, B, 8, 16, 3, 6, 2).astype(float)
    pred, _ = oracle.validate(pred, None)
    assert np.mean(pred == np.rint(pred)) > 0.95   # integer but for a few replaced vectors
    disp, _, _ = oracle.correct(A, B, 16, 8, 4, pred)
    Z = np.zeros((H, W))
    base, _, fl = oracle.correct(Z, Z, 16, 8, 4, pred)   # blank frames: the composition base alone
    assert (fl & oracle.FLAT).all()
    node_value = disp - base + pred
    T = synth.truth(flow, W, H, 8)
    inner = (slice(None), slice(2, -2), slice(2, -2))
    rms = lambda d: np.sqrt(((d - T)[inner] ** 2).mean())
    assert rms(disp) < 0.12 and rms(disp) < 0.6 * rms(node_value), (rms(disp), rms(node_value))
