"""Pins of the oracle's normalised-median validation and vorticity."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2504_17987_amd import synth


def test_uniform_field_has_no_outliers():
    f = np.zeros((2, 6, 7))
    f[0], f[1] = 2.5, -1.25
    g, fl = oracle.validate(f, np.zeros((6, 7), np.uint8))
    assert np.array_equal(g, f) and (fl == 0).all()


def test_spike_is_replaced_by_uniform_value():
    f = np.zeros((2, 6, 7))
    f[0], f[1] = 2.5, -1.25
    f[0, 3, 4] += 10.0
    g, fl = oracle.validate(f, np.zeros((6, 7), np.uint8))
    assert g[0, 3, 4] == 2.5 and g[1, 3, 4] == -1.25
    assert fl[3, 4] == oracle.OUTLIER | oracle.REPLACED
    fl[3, 4] = 0
    assert (fl == 0).all()


@pytest.mark.parametrize("dev,flagged", [(0.15, False), (0.25, True), (-0.19, False), (-0.21, True)])
def test_regulariser_closed_form(dev, flagged):
    # neighbours identical -> residual median 0 -> r0 = |dev| / 0.1
    f = np.ones((2, 5, 5))
    f[1, 2, 2] += dev
    g, fl = oracle.validate(f, np.zeros((5, 5), np.uint8))
    assert bool(fl[2, 2] & oracle.OUTLIER) == flagged
    assert g[1, 2, 2] == (1.0 if flagged else 1.0 + dev)


def test_flat_and_border_vectors_are_outliers_and_not_neighbours():
    f = np.zeros((2, 4, 4))
    f[0] = 1.0
    f[0, 1, 1] = 50.0          # bad value, but flagged FLAT: must not pollute
    flags = np.zeros((4, 4), np.uint8)
    flags[1, 1] = oracle.FLAT
    g, fl = oracle.validate(f, flags)
    assert g[0, 1, 1] == 1.0 and fl[1, 1] & oracle.REPLACED
    assert (g[0] == 1.0).all()
    # an isolated vector with every neighbour flagged stays, UNRESOLVED if it is itself bad
    flags = np.full((3, 3), oracle.BORDER, np.uint8)
    g, fl = oracle.validate(np.ones((2, 3, 3)), flags)
    assert (fl & oracle.UNRESOLVED).all()


def test_scan_order_independence():
    rng = np.random.default_rng(41)
    f = rng.normal(0, 0.3, (2, 9, 11))
    f[:, rng.integers(0, 9, 8), rng.integers(0, 11, 8)] += rng.normal(0, 6, (2, 8))
    g, fl = oracle.validate(f, np.zeros((9, 11), np.uint8))
    # transpose the grid (swap the roles of rows and columns, and of u and v)
    ft = np.ascontiguousarray(f[::-1].transpose(0, 2, 1))
    gt, flt = oracle.validate(ft, np.zeros((11, 9), np.uint8))
    assert np.array_equal(gt, g[::-1].transpose(0, 2, 1)) and np.array_equal(flt, fl.T)
    # mirrored scan
    fm = np.ascontiguousarray(f[:, ::-1, ::-1])
    gm, flm = oracle.validate(fm, np.zeros((9, 11), np.uint8))
    assert np.array_equal(gm, g[:, ::-1, ::-1])


def test_validate_vs_brute():
    rng = np.random.default_rng(42)
    for trial in range(4):
        ny, nx = rng.integers(1, 9, 2)
        f = rng.normal(0, 0.5, (2, ny, nx))
        k = max(1, ny * nx // 6)
        f[:, rng.integers(0, ny, k), rng.integers(0, nx, k)] += rng.normal(0, 5, (2, k))
        flags = (rng.random((ny, nx)) < 0.1).astype(np.uint8) * oracle.BORDER
        g, fl = oracle.validate(f, flags)
        gb, flb, _ = brute.validate(f, flags)
        assert np.abs(g - gb).max() < 1e-12 and np.array_equal(fl, flb)
        g, _ = oracle.validate(f, None)
        gb, _, _ = brute.validate(f, None)
        assert np.abs(g - gb).max() < 1e-12


def test_vorticity_uniform_and_solid_body():
    assert (oracle.vorticity(np.full((2, 5, 6), 3.0), 8) == 0).all()
    om = 0.0123
    fl = synth.SolidBody(20.0, 17.0, om)
    U = synth.truth(fl, 64, 48, 8)
    w = oracle.vorticity(U, 8)
    assert np.abs(w - 2 * om).max() < 1e-15


def test_vorticity_vs_numpy_gradient():
    rng = np.random.default_rng(43)
    for ny, nx in [(5, 7), (3, 3), (8, 4)]:
        f = rng.normal(0, 1, (2, ny, nx))
        assert np.abs(oracle.vorticity(f, 12) - brute.vorticity(f, 12)).max() < 1e-12
    # 2-node lines: first-order difference; 1-node lines: zero
    f = rng.normal(0, 1, (2, 2, 1))
    w = oracle.vorticity(f, 4)
    assert np.allclose(w[:, 0], -(f[0, 1, 0] - f[0, 0, 0]) / 4)


def test_vorticity_lamb_oseen_truncation():
    lo = synth.cfg2_flow()
    U = synth.truth(lo, 1024, 1024, 8)
    w = oracle.vorticity(U, 8)
    X, Y = synth.node_centres(1024, 1024, 8)
    exact = lo.vorticity(X, Y)
    # central differences: error O(h^2); bound h^2/6 * (|v_xxx| + |u_yyy|),
    # third derivatives of the vortex ~ |u|max / rc^3 * c with c ~ 10
    bound = 8 ** 2 / 6 * 2 * 10 * 20.0 / 128.0 ** 3
    inner = (slice(1, -1), slice(1, -1))
    err = np.abs(w - exact)[inner]
    assert err.max() < bound
    # second order: halving the node spacing divides the interior error by ~4
    U4 = synth.truth(lo, 1024, 1024, 4)
    X4, Y4 = synth.node_centres(1024, 1024, 4)
    err4 = np.abs(oracle.vorticity(U4, 4) - lo.vorticity(X4, Y4))[inner]
    assert 3.6 < err.max() / err4.max() < 4.4
    # the stencil applied to node samples equals numpy.gradient's within rounding
    assert np.abs(w - brute.vorticity(U, 8)).max() < 1e-12
