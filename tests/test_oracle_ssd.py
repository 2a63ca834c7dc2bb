"""Pins of the oracle's windowed-SSD loss and its analytic adjoint."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2504_17987_amd import synth


def fd_grad(A, B, U, g, win, step, h):
    G = np.zeros_like(U)
    for idx in np.ndindex(U.shape):
        Up = U.copy(); Up[idx] += h
        Um = U.copy(); Um[idx] -= h
        G[idx] = ((g * oracle.ssd_forward(A, B, Up, win, step)).sum()
                  - (g * oracle.ssd_forward(A, B, Um, win, step)).sum()) / (2 * h)
    return G


def test_forward_vs_scipy():
    rng = np.random.default_rng(51)
    A = rng.random((40, 48))
    B = rng.random((40, 48))
    U = rng.normal(0, 2, (2, 5, 6))
    assert np.abs(oracle.ssd_forward(A, B, U, 16, 8) - brute.ssd_forward(A, B, U, 16, 8)).max() < 1e-10


def test_linear_ramp_quadratic_loss_fd_exact():
    """B = ax + by + c: B' is linear in U wherever the sample stays inside the
    image, so the loss of the inner windows is quadratic in U and a central
    difference with a large step is exact."""
    H = W = 64
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    B = 0.7 * xs - 0.4 * ys + 5.0
    rng = np.random.default_rng(52)
    A = rng.normal(0, 1, (H, W))
    U = rng.normal(0, 0.8, (2, 8, 8))
    g = np.zeros((8, 8))
    g[2:6, 2:6] = rng.random((4, 4)) + 0.5   # windows far from the image edge
    G, D = oracle.ssd_grad(A, B, U, g, 16, 8)
    Gfd = fd_grad(A, B, U, g, 16, 8, 0.37)
    assert np.abs(G - Gfd).max() < 1e-8 * np.abs(G).max()
    # Gauss-Newton diagonal of a linear model: the exact second derivative
    for idx in [(0, 3, 3), (1, 4, 2), (0, 2, 5)]:
        Up = U.copy(); Up[idx] += 0.5
        Um = U.copy(); Um[idx] -= 0.5
        L = lambda V: (g * oracle.ssd_forward(A, B, V, 16, 8)).sum()
        second = (L(Up) - 2 * L(U) + L(Um)) / 0.25
        assert abs(second - D[idx]) < 1e-8 * abs(D[idx])


def test_exact_solution_has_zero_gradient():
    rng = np.random.default_rng(53)
    B = rng.random((48, 48))
    U = rng.normal(0, 1.5, (2, 6, 6))
    A = oracle.warp_image(B, 1, 0, U, 8)   # A(p) = B(p + u(p)) on the image
    g = np.zeros((6, 6))
    g[1:5, 1:5] = 1.0                      # windows that do not overhang the image
    G, D = oracle.ssd_grad(A, B, U, g, 16, 8)
    assert np.abs(G).max() < 1e-12 and (D >= 0).all() and D.max() > 0
    assert np.abs(oracle.ssd_forward(A, B, U, 16, 8)[1:5, 1:5]).max() < 1e-20


def test_fd_uniform_fractional_field():
    """u(p) + p never within h of an integer: the loss is smooth at U."""
    A, B = synth.make_pair(48, 48, synth.Uniform(0.4, -0.6), 0.08, seed=54)
    A = A / 255.0
    B = B / 255.0
    U = np.zeros((2, 6, 6))
    U[0], U[1] = 0.37, -0.61
    g = np.random.default_rng(54).random((6, 6)) + 0.5
    G, _ = oracle.ssd_grad(A, B, U, g, 16, 8)
    Gfd = fd_grad(A, B, U, g, 16, 8, 1e-3)
    assert np.abs(G - Gfd).max() < 1e-6 * np.abs(G).max()


def test_fd_random_field_excluding_kinks():
    A, B = synth.make_pair(48, 48, synth.Uniform(1.2, 0.7), 0.08, seed=55)
    A = A / 255.0
    B = B / 255.0
    rng = np.random.default_rng(55)
    U = rng.normal(0, 1.0, (2, 6, 6)) + 0.5
    g = rng.random((6, 6)) + 0.5
    h = 1e-3
    G, _ = oracle.ssd_grad(A, B, U, g, 16, 8)
    Gfd = fd_grad(A, B, U, g, 16, 8, h)
    # a node is smooth when none of the samples it moves lies within h of a
    # grid line in the moved coordinate
    smooth = np.ones(U.shape, bool)
    for y in range(-4, 52):
        for x in range(-4, 52):
            u, v = oracle.interp(U, 8, x, y)
            tx = min(max((x - 3.5) / 8, 0), 5)
            ty = min(max((y - 3.5) / 8, 0), 5)
            bx, by = min(int(np.floor(tx)), 4), min(int(np.floor(ty)), 4)
            for c, q in ((0, x + u), (1, y + v)):
                if abs(q - np.rint(q)) < 1.5 * h:
                    smooth[c, by:by + 2, bx:bx + 2] = False
    assert smooth.sum() >= 0.5 * smooth.size
    err = np.abs(G - Gfd)[smooth]
    assert err.max() < 1e-6 * np.abs(G).max()
