"""Pins of the oracle's semi-global-matching predictor level: zero
penalties reduce it to block matching (the brute-force SAD search); the
four-path aggregation against an independent numpy recursion and a
two-node closed form; integer shifts recovered exactly; and the smoothness
penalty overriding a corrupted block."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2504_17987_amd import synth


def agg_brute(C, R, P1, P2):
    """The four path recursions written per path with numpy over the
    candidate axis (8-neighbour minimum by shifted copies of the grid)."""
    ny, nx, nd = C.shape
    n1 = 2 * R + 1
    big = np.iinfo(np.int64).max // 4

    def step(prev, c):
        g = prev.reshape(n1, n1)
        pad = np.full((n1 + 2, n1 + 2), big, np.int64)
        pad[1:-1, 1:-1] = g
        nb = np.full_like(g, big)
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                if oy or ox:
                    nb = np.minimum(nb, pad[1 + oy:1 + oy + n1, 1 + ox:1 + ox + n1])
        m = prev.min()
        best = np.minimum(np.minimum(g, nb + P1), m + P2).ravel()
        return c + best - m

    S = np.zeros_like(C)
    for a in range(ny):                 # along rows, both ways
        for order in (range(nx), range(nx - 1, -1, -1)):
            prev = None
            for b in order:
                cur = C[a, b].copy() if prev is None else step(prev, C[a, b])
                S[a, b] += cur
                prev = cur
    for b in range(nx):                 # along columns, both ways
        for order in (range(ny), range(ny - 1, -1, -1)):
            prev = None
            for a in order:
                cur = C[a, b].copy() if prev is None else step(prev, C[a, b])
                S[a, b] += cur
                prev = cur
    return S


@pytest.mark.parametrize("R,P1,P2", [(1, 3, 20), (2, 10, 40), (3, 0, 0), (2, 7, 7)])
def test_aggregate_vs_numpy_recursion(R, P1, P2):
    rng = np.random.default_rng(21)
    C = rng.integers(0, 200, (5, 7, (2 * R + 1) ** 2)).astype(np.int64)
    assert np.array_equal(oracle.sgm_aggregate(C, R, P1, P2), agg_brute(C, R, P1, P2))


def test_aggregate_two_nodes_closed_form():
    """Two nodes side by side, R = 1: the vertical paths see one node each
    (L = C), the horizontal paths one step of the recursion each way."""
    C0 = np.array([9, 4, 9, 9, 9, 9, 9, 9, 1], np.int64)   # minimum at k = 8 (dy = dx = 1)
    C1 = np.array([5, 0, 5, 5, 5, 5, 5, 5, 5], np.int64)   # minimum at k = 1 (dy = -1, dx = 0)
    P1, P2 = 2, 6
    C = np.stack([C0, C1])[None]
    S = oracle.sgm_aggregate(C, 1, P1, P2)
    # node 1 from node 0 (m0 = 1): k = 1 is 8-adjacent to nothing at cost 1
    # (k = 8 is two away), so min(C0[1] = 4, neighbours + P1, m0 + P2 = 7) = 4
    L1 = C1 + np.array([min(C0[k], min(C0[j] for j in range(9) if j != k and abs(j // 3 - k // 3) <= 1
                                       and abs(j % 3 - k % 3) <= 1) + P1, 1 + P2) for k in range(9)]) - 1
    L0 = C0 + np.array([min(C1[k], min(C1[j] for j in range(9) if j != k and abs(j // 3 - k // 3) <= 1
                                       and abs(j % 3 - k % 3) <= 1) + P1, 0 + P2) for k in range(9)]) - 0
    assert np.array_equal(S[0, 0], 3 * C0 + L0) and np.array_equal(S[0, 1], 3 * C1 + L1)
    assert L1[1] == 0 + 4 - 1 and L1[8] == 5 + 1 - 1


def test_zero_penalties_reduce_to_block_matching():
    A, B = synth.make_pair(96, 80, synth.SolidBody(47.5, 39.5, 0.05), 0.05, noise=2.0, seed=22)
    ny, nx = 80 // 8, 96 // 8
    d_sgm = oracle.sgm_level(A, B, nx, ny, 8, 16, 3, 0, 0)
    d_bm = brute.sad_level(A, B, nx, ny, 8, 16, 3)
    assert np.array_equal(d_sgm, d_bm)


@pytest.mark.parametrize("levels", [1, 3])
def test_integer_shift_recovered(levels):
    A, B = synth.make_pair(128, 96, synth.Uniform(4.0, -3.0), 0.05, noise=1.0, seed=23)
    pred = oracle.predict(A, B, 8, 16, levels, 6 if levels == 1 else 3, 2, sgm=(2, 16))
    inner = (slice(None), slice(2, -2), slice(2, -2))
    assert (pred[0][inner[1:]] == 4).all() and (pred[1][inner[1:]] == -3).all()


def test_smoothness_penalty_overrides_a_corrupted_block():
    """Uniform shift (3, 2); one node's block of A is replaced by noise.
    Block matching there returns some other shift; with a large P2 the
    aggregated costs of its neighbours pull it to (3, 2)."""
    A, B = synth.make_pair(128, 128, synth.Uniform(3.0, 2.0), 0.05, noise=1.0, seed=24)
    A = A.copy()
    rng = np.random.default_rng(25)
    a, b = 8, 8                                   # node (8, 8): block rows/cols 60..75
    A[60:76, 60:76] = rng.integers(0, 256, (16, 16))
    d_bm = oracle.sad_level(A, B, 16, 16, 8, 16, 4)
    assert (d_bm[0, a, b], d_bm[1, a, b]) != (3, 2)
    d = oracle.sgm_level(A, B, 16, 16, 8, 16, 4, 2, 64)
    assert (d[0, a, b], d[1, a, b]) == (3, 2)
    assert (d[0, 2:-2, 2:-2] == 3).all() and (d[1, 2:-2, 2:-2] == 2).all()
