"""Brute-force NumPy/SciPy restatement of the oracle for tiny images.

TEST INFRASTRUCTURE ONLY.  It pins the C oracle from the outside: each step
is computed a second way, mostly through a library routine that states the
textbook operation (scipy's bilinear ``map_coordinates``, numpy's Pearson
``corrcoef``, ``median`` and ``gradient``), vectorised over whole images
rather than looped per window, so that a slip in the C loops (a dropped
term, a swapped index, a wrong sign) shows up as a mismatch.  Suitable for
images of a few thousand pixels only.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import map_coordinates


def pad(I, p):
    return np.pad(np.asarray(I), p, mode="constant")


def pyr_down(I):
    I = np.asarray(I, dtype=np.int64)
    H, W = I.shape
    P = np.zeros((H + (H & 1), W + (W & 1)), np.int64)
    P[:H, :W] = I
    s = P.reshape(P.shape[0] // 2, 2, P.shape[1] // 2, 2).sum(axis=(1, 3))
    return (s + 2) // 4


def sad_level(A, B, nx, ny, step, block, R, cand=None):
    """Exhaustive SAD over every candidate of every node, winner chosen by
    Python's tuple ordering of (SAD, |dx|+|dy|, dy, dx)."""
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    M = 256
    Ap, Bp = pad(A, M), pad(B, M)
    off = (step - block) // 2
    d = np.zeros((2, ny, nx), np.int64)
    for a in range(ny):
        for b in range(nx):
            oy, ox = a * step + off + M, b * step + off + M
            cx = 0 if cand is None else int(cand[0, a, b])
            cy = 0 if cand is None else int(cand[1, a, b])
            blk = Ap[oy:oy + block, ox:ox + block]
            keys = []
            for dy in range(cy - R, cy + R + 1):
                for dx in range(cx - R, cx + R + 1):
                    s = np.abs(blk - Bp[oy + dy:oy + dy + block, ox + dx:ox + dx + block]).sum()
                    keys.append((int(s), abs(dx) + abs(dy), dy, dx))
            best = min(keys)
            d[0, a, b], d[1, a, b] = best[3], best[2]
    return d


def median3_int(d):
    import statistics
    d = np.asarray(d)
    out = np.zeros_like(d)
    _, ny, nx = d.shape
    for c in range(2):
        for a in range(ny):
            for b in range(nx):
                vals = d[c, max(a - 1, 0):a + 2, max(b - 1, 0):b + 2].ravel().tolist()
                out[c, a, b] = statistics.median_low(vals)
    return out


def predict(A, B, step, block, levels, Rc, Rf, median=True):
    PA, PB = [np.asarray(A, np.int64)], [np.asarray(B, np.int64)]
    for _ in range(1, levels):
        PA.append(pyr_down(PA[-1]))
        PB.append(pyr_down(PB[-1]))
    H, W = PA[0].shape
    grids = [(W // step, H // step)]
    for _ in range(1, levels):
        nx, ny = grids[-1]
        grids.append(((nx + 1) // 2, (ny + 1) // 2))
    prev = None
    for l in range(levels - 1, -1, -1):
        nx, ny = grids[l]
        cand = None
        if prev is not None:
            # parent (a//2, b//2): repeat each parent twice along both axes
            cand = 2 * np.repeat(np.repeat(prev, 2, axis=1), 2, axis=2)[:, :ny, :nx]
        d = sad_level(PA[l], PB[l], nx, ny, step, block, Rc if l == levels - 1 else Rf, cand)
        if median:
            d = median3_int(d)
        prev = d
    return prev


def displacement_at(U, step, xs, ys):
    """u at pixel positions by bilinear interpolation of the node field with
    the position clamped to the node hull (scipy map_coordinates, order 1,
    edge-held)."""
    U = np.asarray(U, np.float64)
    ty = (np.asarray(ys, np.float64) - (step - 1) / 2.0) / step
    tx = (np.asarray(xs, np.float64) - (step - 1) / 2.0) / step
    c = np.stack([ty.ravel(), tx.ravel()])
    u = map_coordinates(U[0], c, order=1, mode="nearest").reshape(np.shape(xs))
    v = map_coordinates(U[1], c, order=1, mode="nearest").reshape(np.shape(xs))
    return u, v


def sample(I, xs, ys):
    """bilinear sample, zero outside (scipy 'grid-constant')."""
    c = np.stack([np.ravel(ys), np.ravel(xs)])
    return map_coordinates(np.asarray(I, np.float64), c, order=1, mode="grid-constant",
                           cval=0.0).reshape(np.shape(xs))


def warped_region(I, which, mode, U, step, y0, x0, h, w):
    """Warped frame over the pixel rectangle [y0, y0+h) x [x0, x0+w)."""
    ys, xs = np.mgrid[y0:y0 + h, x0:x0 + w].astype(np.float64)
    if which == 0 and mode == 0:
        return sample(I, xs, ys)
    if U is None:
        u = v = np.zeros_like(xs)
    else:
        u, v = displacement_at(U, step, xs, ys)
    s = 0.5 if mode == 1 else 1.0
    if which == 0:
        s = -s
    return sample(I, xs + s * u, ys + s * v)


def corr_plane(A, B, win, step, r, mode, pred, a, b):
    """Pearson coefficient per shift via numpy.corrcoef (0 when a window is
    constant)."""
    h = (win - step) // 2
    oy, ox = a * step - h, b * step - h
    Aw = warped_region(A, 0, mode, pred, step, oy, ox, win, win)
    Breg = warped_region(B, 1, mode, pred, step, oy - r, ox - r, win + 2 * r, win + 2 * r)
    rho = np.zeros((2 * r + 1, 2 * r + 1))
    for sy in range(-r, r + 1):
        for sx in range(-r, r + 1):
            Bw = Breg[sy + r:sy + r + win, sx + r:sx + r + win]
            if np.ptp(Aw) == 0 or np.ptp(Bw) == 0:
                rho[sy + r, sx + r] = 0.0
            else:
                rho[sy + r, sx + r] = np.corrcoef(Aw.ravel(), Bw.ravel())[0, 1]
    return rho


def validate(field, flags=None, thr=2.0, eps=0.1):
    """Normalised median test with numpy.median (even counts average the two
    middle values), replacement from the detection-pass field."""
    f = np.array(field, np.float64)
    _, ny, nx = f.shape
    bad_in = np.zeros((ny, nx), bool) if flags is None else (np.asarray(flags) & 3) != 0
    out = bad_in.copy()
    for a in range(ny):
        for b in range(nx):
            if bad_in[a, b]:
                continue
            nb = [(y, x) for y in range(a - 1, a + 2) for x in range(b - 1, b + 2)
                  if 0 <= y < ny and 0 <= x < nx and (y, x) != (a, b) and not bad_in[y, x]]
            if not nb:
                continue
            worst = 0.0
            for c in range(2):
                vals = np.array([f[c, y, x] for y, x in nb])
                um = np.median(vals)
                rm = np.median(np.abs(vals - um))
                worst = max(worst, abs(f[c, a, b] - um) / (rm + eps))
            out[a, b] = worst > thr
    g = f.copy()
    fl = None if flags is None else np.array(flags, np.uint8)
    for a in range(ny):
        for b in range(nx):
            if not out[a, b]:
                continue
            nb = [(y, x) for y in range(a - 1, a + 2) for x in range(b - 1, b + 2)
                  if 0 <= y < ny and 0 <= x < nx and (y, x) != (a, b) and not out[y, x]]
            if fl is not None:
                fl[a, b] |= 8
            if nb:
                for c in range(2):
                    g[c, a, b] = np.median([f[c, y, x] for y, x in nb])
                if fl is not None:
                    fl[a, b] |= 16
            elif fl is not None:
                fl[a, b] |= 32
    return g, fl, out


def vorticity(field, step):
    """numpy.gradient with second-order edges: central inside, one-sided
    second order on the edges."""
    f = np.asarray(field, np.float64)
    dvdx = np.gradient(f[1], float(step), axis=1, edge_order=2)
    dudy = np.gradient(f[0], float(step), axis=0, edge_order=2)
    return dvdx - dudy


def ssd_forward(A, B, U, win, step):
    """Per-window SSD of B sampled at p + u(p) against A."""
    A = np.asarray(A, np.float64)
    H, W = A.shape
    nx, ny = W // step, H // step
    h = (win - step) // 2
    loss = np.zeros((ny, nx))
    for a in range(ny):
        for b in range(nx):
            ys, xs = np.mgrid[a * step - h:a * step - h + win, b * step - h:b * step - h + win].astype(float)
            u, v = displacement_at(U, step, xs, ys)
            r = sample(B, xs + u, ys + v) - sample(A, xs, ys)
            loss[a, b] = (r * r).sum()
    return loss
