"""Shared helpers of the GPU parity tests (comparison rules, tolerances)."""
from __future__ import annotations

import sys

import numpy as np

import oracle

# Tolerances (FP32 kernels against the FP64 oracle)
TOL_DISP_PX = 0.01        # sub-pixel displacement
TOL_REL = 1e-4            # vorticity and gradients, relative to max |value|
TOL_RHO = 2e-5            # correlation coefficient at the chosen shift
NEAR_TIE_RHO = 1e-5       # top-2 coefficient gap under which either peak is correct
NEAR_TIE_UOD = 1e-4       # |r0 - threshold| under which either decision is correct


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def corr_gap(A, B, win, step, r, mode, pred, a, b):
    """Gap between the two largest coefficients of a window (oracle FP64)."""
    rho = oracle.corr_plane(A, B, win, step, r, mode, pred, a, b).ravel()
    top = np.sort(rho)[-2:]
    return top[1] - top[0]


def uod_r0(field, flags, a, b, eps=0.1):
    """Largest normalised residual of vector (a, b) (FP64, numpy median)."""
    _, ny, nx = field.shape
    nb = [(y, x) for y in range(a - 1, a + 2) for x in range(b - 1, b + 2)
          if 0 <= y < ny and 0 <= x < nx and (y, x) != (a, b)
          and (flags is None or not (flags[y, x] & 3))]
    if not nb:
        return 0.0
    worst = 0.0
    for c in range(2):
        v = np.array([field[c, y, x] for y, x in nb], np.float64)
        um = np.median(v)
        rm = np.median(np.abs(v - um))
        worst = max(worst, abs(field[c, a, b] - um) / (rm + eps))
    return worst


def compare_correct(Ag, Bg, Ao, Bo, win, step, r, pred, disp_g, peak_g, flags_g, disp_o, peak_o,
                    flags_o, mode=0, fixed=False, max_ties=None):
    """Element-wise comparison of a correction result with the oracle's.
    Where they differ, the oracle's correlation plane must show a near-tie.
    Returns the number of near-tie exemptions."""
    d = np.abs(disp_g - disp_o).max(axis=0)
    bad = (d > TOL_DISP_PX) | (np.abs(peak_g - peak_o) > TOL_RHO) | (flags_g != flags_o)
    ties = 0
    for a, b in zip(*np.nonzero(bad)):
        R = 1 if fixed else r
        gap = corr_gap(Ao, Bo, win, step, R, mode, pred, int(a), int(b))
        assert gap < NEAR_TIE_RHO, (
            f"node ({a},{b}): gpu {disp_g[:, a, b]} rho {peak_g[a, b]} fl {flags_g[a, b]} vs "
            f"oracle {disp_o[:, a, b]} rho {peak_o[a, b]} fl {flags_o[a, b]}, top-2 gap {gap}")
        ties += 1
    if max_ties is not None:
        assert ties <= max_ties, f"{ties} near-tie exemptions"
    return ties
