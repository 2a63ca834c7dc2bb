"""Pins of the oracle's gradient refinement (an addition: preconditioned
gradient steps on the total windowed SSD) and of its temporal smoothing
(the paper's exponential smoothing in time, Sec. 2), each against something
other than the oracle itself: finite differences of the scipy brute-force
loss, closed forms, and the geometric weights of an exponential average."""
import numpy as np
import pytest

import oracle
from oracle import brute


def total_loss(A, B, U, win=16, step=8):
    return brute.ssd_forward(A, B, U, win, step).sum()


def fractional_field(rng, ny, nx, spread=0.08):
    """Node field whose bilinear samples keep their fractional parts inside
    (0.2, 0.6): with perturbations below 0.05 px no sample crosses a pixel
    line, so the loss is exactly quadratic along every node component."""
    U = np.empty((2, ny, nx))
    U[0] = 0.37 + rng.uniform(-spread, spread, (ny, nx))
    U[1] = -0.61 + rng.uniform(-spread, spread, (ny, nx))
    return U


def test_refine_one_step_matches_finite_differences():
    """One step U - tau G / (D + lam_rel mean(D)) where G and D are the exact
    first and second derivatives of the total loss (central differences of
    the scipy loss, exact on a quadratic) -- so the step, the Gauss-Newton
    diagonal, the regulariser and the update's sign are all pinned."""
    rng = np.random.default_rng(61)
    H = W = 48
    A = rng.random((H, W))
    B = rng.random((H, W))
    U0 = fractional_field(rng, 6, 6)
    h = 0.05
    L0 = total_loss(A, B, U0)
    G = np.zeros_like(U0)
    D = np.zeros_like(U0)
    for idx in np.ndindex(U0.shape):
        Up = U0.copy(); Up[idx] += h
        Um = U0.copy(); Um[idx] -= h
        Lp, Lm = total_loss(A, B, Up), total_loss(A, B, Um)
        G[idx] = (Lp - Lm) / (2 * h)
        D[idx] = (Lp - 2 * L0 + Lm) / (h * h)
    tau, lam_rel = 0.7, 0.3
    lam = lam_rel * D.mean()
    expect = U0 - tau * G / (D + lam)
    U1, hist = oracle.ssd_refine(A, B, U0, 16, 8, steps=1, tau=tau, lam_rel=lam_rel)
    assert np.abs(U1 - expect).max() < 1e-7 * np.abs(U0 - expect).max() + 1e-12
    assert abs(hist[0] - L0) < 1e-9 * L0
    assert abs(hist[1] - total_loss(A, B, U1)) < 1e-9 * L0


@pytest.mark.parametrize("tau,frac", [(1.0, 0.0), (0.5, 0.5)])
def test_refine_ramp_single_node_lands_on_minimiser(tau, frac):
    """B a linear ramp, A = B deformed by the true field U*, U0 = U* except
    one interior node's u component (off by delta).  The gradient and the
    diagonal at that node are 2 a^2 delta sum(m w^2) and 2 a^2 sum(m w^2), so
    with lambda = 0 the step moves it by tau delta: tau = 1 lands exactly on
    the minimiser, tau = 1/2 half way."""
    H = W = 64
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    B = 0.7 * xs - 0.4 * ys + 5.0
    rng = np.random.default_rng(62)
    Ustar = rng.normal(0, 0.5, (2, 8, 8))
    A = oracle.warp_image(B, 1, 0, Ustar, 8)
    delta = 0.83
    U0 = Ustar.copy()
    U0[0, 3, 4] += delta
    U1, _ = oracle.ssd_refine(A, B, U0, 16, 8, steps=1, tau=tau, lam_rel=0.0)
    assert abs(U1[0, 3, 4] - (Ustar[0, 3, 4] + frac * delta)) < 1e-10


def test_refine_reduces_loss_and_approaches_truth():
    """Ten steps from a perturbed field on a smooth particle-like image: the
    total loss falls monotonically and the field moves toward the truth."""
    rng = np.random.default_rng(63)
    H = W = 64
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    B = np.zeros((H, W))
    for _ in range(120):
        cx, cy = rng.uniform(-4, W + 4), rng.uniform(-4, H + 4)
        B += 200 * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / 2.0)
    B /= 255.0
    Ustar = 0.6 * rng.normal(0, 1, (2, 8, 8))
    A = oracle.warp_image(B, 1, 0, Ustar, 8)
    U0 = Ustar + rng.normal(0, 0.3, Ustar.shape)
    U10, hist = oracle.ssd_refine(A, B, U0, 16, 8, steps=10)
    assert (np.diff(hist) < 0).all()
    inner = (slice(None), slice(1, -1), slice(1, -1))
    assert np.sqrt(((U10 - Ustar)[inner] ** 2).mean()) < 0.5 * np.sqrt(((U0 - Ustar)[inner] ** 2).mean())


def test_refine_leaves_zero_curvature_nodes_unchanged():
    """Blank frames: D = 0 everywhere and lambda = 0, so no node moves."""
    Z = np.zeros((32, 32))
    U0 = np.random.default_rng(64).normal(0, 1, (2, 4, 4))
    U1, hist = oracle.ssd_refine(Z, Z, U0, 16, 8, steps=3)
    assert np.array_equal(U1, U0) and (hist == 0).all()


# --- temporal smoothing -------------------------------------------------------

def test_smooth_constant_field_is_fixed_point():
    c = np.full((2, 3, 4), 1.75)
    f, s = oracle.smooth(c, c, 0.3, False)
    assert np.array_equal(f, c) and np.array_equal(s, c)


def test_smooth_half_is_exact_average_and_one_is_identity():
    rng = np.random.default_rng(65)
    x, st = rng.normal(0, 3, (2, 5, 6)), rng.normal(0, 3, (2, 5, 6))
    f, s = oracle.smooth(x, st, 0.5, False)
    assert np.array_equal(f, (x + st) / 2) and np.array_equal(s, f)
    f, s = oracle.smooth(x, st, 1.0, False)
    assert np.array_equal(f, x)
    f, s = oracle.smooth(x, st, 0.25, True)       # a first frame starts the state
    assert np.array_equal(f, x) and np.array_equal(s, x)


def test_smooth_sequence_has_geometric_weights():
    """s_t = (1 - a)^t x_0 + sum_{j=1..t} a (1 - a)^(t - j) x_j."""
    rng = np.random.default_rng(66)
    xs = rng.normal(0, 2, (7, 2, 3, 3))
    a = 0.35
    s = None
    for t, x in enumerate(xs):
        f, s = oracle.smooth(x, s, a, t == 0)
        w = [(1 - a) ** t] + [a * (1 - a) ** (t - j) for j in range(1, t + 1)]
        closed = sum(wj * xs[j] for j, wj in enumerate(w))
        assert np.abs(f - closed).max() < 1e-12
        assert abs(sum(w) - 1) < 1e-12


def test_smooth_batch_chains_slots_in_order():
    """Frames of one stream in one batch chain in batch order; frames of
    other streams do not interfere; slots outside the table are skipped."""
    rng = np.random.default_rng(67)
    xs = rng.normal(0, 2, (5, 2, 2, 3))
    states = rng.normal(0, 2, (3, 2, 2, 3))
    slots = [-1 - 1, 0, 1, 1, 7]
    out, st = oracle.smooth_batch(xs, states, slots, 0.5)
    # stream 1 starts with frame 0, continues with frames 2 and 3
    s1 = xs[0]
    s1 = 0.5 * xs[2] + 0.5 * s1
    assert np.array_equal(out[2], s1)
    s1 = 0.5 * xs[3] + 0.5 * s1
    assert np.array_equal(out[3], s1) and np.array_equal(st[1], s1)
    assert np.array_equal(out[1], 0.5 * xs[1] + 0.5 * states[0])
    assert np.array_equal(out[4], xs[4]) and np.array_equal(st[2], states[2])
