"""FP64 CPU oracle of the PIV hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C reference in ``oracle.c`` (built
with gcc by ``oracle/build.py``) and shares no code with the GPU library.

All arrays are numpy; images are [H][W], fields [2][ny][nx] (u, v),
per-vector arrays [ny][nx].
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _nullable(nd):
    """ndpointer that also accepts None."""
    class _N(nd):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return super().from_param(obj)
    return _N


_Dn = _nullable(_D)
_In = _nullable(_I)
_U8n = _nullable(_U8)
_i = C.c_int
_d = C.c_double


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        L.o_pyr_down.argtypes = [_I, _i, _i, _I]
        L.o_sad_level.argtypes = [_I, _I, _i, _i, _i, _i, _i, _i, _i, _In, _I]
        L.o_median3_int.argtypes = [_I, _i, _i, _I]
        L.o_predict.argtypes = [_I, _I, _i, _i, _i, _i, _i, _i, _i, _i, _I]
        L.o_interp.argtypes = [_D, _i, _i, _i, _d, _d, C.POINTER(_d), C.POINTER(_d)]
        L.o_bilin.argtypes = [_D, _i, _i, _d, _d]
        L.o_bilin.restype = _d
        L.o_warp_image.argtypes = [_D, _i, _i, _Dn, _i, _i, _i, _D]
        L.o_gauss3.argtypes = [_d, _d, _d, C.POINTER(_i)]
        L.o_gauss3.restype = _d
        L.o_corr_plane.argtypes = [_D, _D, _i, _i, _i, _i, _i, _i, _Dn, _i, _i, _D]
        L.o_correct_node.argtypes = [_D, _D, _i, _i, _i, _i, _i, _i, _i, _Dn, _i, _i,
                                     C.POINTER(_d), C.POINTER(_d), C.POINTER(_d), C.POINTER(C.c_uint8)]
        L.o_correct.argtypes = [_D, _D, _i, _i, _i, _i, _i, _i, _i, _Dn, _D, _Dn, _U8]
        L.o_validate.argtypes = [_D, _U8n, _i, _i, _d, _d]
        L.o_vorticity.argtypes = [_D, _i, _i, _i, _D]
        L.o_ssd_forward.argtypes = [_D, _D, _D, _i, _i, _i, _i, _D]
        L.o_ssd_grad.argtypes = [_D, _D, _D, _D, _i, _i, _i, _i, _D, _Dn]
        L.o_ssd_refine.argtypes = [_D, _D, _D, _i, _i, _i, _i, _i, _d, _d, _Dn]
        L.o_smooth.argtypes = [_D, _D, _i, _d, _i]
        L.o_highpass.argtypes = [_I, _i, _i, _i, _I]
        _L = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        L.o_sgm_aggregate.argtypes = [_L, _i, _i, _i, C.c_int64, C.c_int64, _L]
        L.o_sgm_level.argtypes = [_I, _I, _i, _i, _i, _i, _i, _i, _i, _i, _i, _I]
        L.o_predict_sgm.argtypes = [_I, _I, _i, _i, _i, _i, _i, _i, _i, _i, _i, _i, _i, _I]
        L.o_clahe_clip.argtypes = [C.c_int64, _i, _d]
        L.o_clahe_clip.restype = C.c_int64
        L.o_clahe.argtypes = [_I, _i, _i, _i, _i, _i, _d, _I]
        _lib = L
    return _lib


FLAT, BORDER, NOCURV, OUTLIER, REPLACED, UNRESOLVED = 1, 2, 4, 8, 16, 32


def _img_i(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _img_d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def pyr_down(img):
    img = _img_i(img)
    H, W = img.shape
    out = np.zeros(((H + 1) // 2, (W + 1) // 2), np.int32)
    lib().o_pyr_down(img, W, H, out)
    return out


def sad_level(A, B, nx, ny, step, block, R, cand=None):
    A, B = _img_i(A), _img_i(B)
    H, W = A.shape
    d = np.zeros((2, ny, nx), np.int32)
    lib().o_sad_level(A, B, W, H, nx, ny, step, block, R,
                      None if cand is None else _img_i(cand), d)
    return d


def median3_int(d):
    d = _img_i(d)
    out = np.zeros_like(d)
    lib().o_median3_int(d, d.shape[2], d.shape[1], out)
    return out


def predict(A, B, step, block, levels, Rc, Rf, median=True, sgm=None):
    """The predictor; sgm = (p1, p2) searches the coarsest level by
    semi-global matching with those penalties per block pixel."""
    A, B = _img_i(A), _img_i(B)
    H, W = A.shape
    pred = np.zeros((2, H // step, W // step), np.int32)
    if sgm is None:
        lib().o_predict(A, B, W, H, step, block, levels, Rc, Rf, int(bool(median)), pred)
    else:
        lib().o_predict_sgm(A, B, W, H, step, block, levels, Rc, Rf, int(bool(median)), 1, int(sgm[0]),
                            int(sgm[1]), pred)
    return pred


def sgm_aggregate(C, R, P1, P2):
    """C [ny][nx][(2R+1)^2] int64 -> S, the sum of the four path costs."""
    C = np.ascontiguousarray(C, dtype=np.int64)
    ny, nx, nd = C.shape
    S = np.zeros_like(C)
    lib().o_sgm_aggregate(C, nx, ny, int(R), int(P1), int(P2), S)
    return S


def sgm_level(A, B, nx, ny, step, block, R, p1, p2):
    A, B = _img_i(A), _img_i(B)
    H, W = A.shape
    d = np.zeros((2, ny, nx), np.int32)
    lib().o_sgm_level(A, B, W, H, nx, ny, step, block, R, int(p1), int(p2), d)
    return d


def interp(U, step, x, y):
    U = _img_d(U)
    u, v = _d(), _d()
    lib().o_interp(U, U.shape[2], U.shape[1], step, float(x), float(y), C.byref(u), C.byref(v))
    return u.value, v.value


def bilin(I, x, y):
    I = _img_d(I)
    return lib().o_bilin(I, I.shape[1], I.shape[0], float(x), float(y))


def warp_image(I, which, mode, U, step):
    I = _img_d(I)
    H, W = I.shape
    out = np.zeros((H, W))
    lib().o_warp_image(I, int(which), int(mode), None if U is None else _img_d(U), W, H, step, out)
    return out


def gauss3(cm, c0, cp):
    nc = _i()
    d = lib().o_gauss3(float(cm), float(c0), float(cp), C.byref(nc))
    return d, bool(nc.value)


def corr_plane(A, B, win, step, r, mode, pred, a, b):
    A, B = _img_d(A), _img_d(B)
    H, W = A.shape
    rho = np.zeros((2 * r + 1, 2 * r + 1))
    lib().o_corr_plane(A, B, W, H, win, step, r, mode, None if pred is None else _img_d(pred), a, b, rho)
    return rho


def correct_node(A, B, win, step, r, pred, a, b, warp_mode=0, peak_mode=0):
    A, B = _img_d(A), _img_d(B)
    H, W = A.shape
    du, dv, pk, fl = _d(), _d(), _d(), C.c_uint8()
    lib().o_correct_node(A, B, W, H, win, step, r, warp_mode, peak_mode,
                         None if pred is None else _img_d(pred), a, b,
                         C.byref(du), C.byref(dv), C.byref(pk), C.byref(fl))
    return du.value, dv.value, pk.value, fl.value


def correct(A, B, win, step, r, pred=None, warp_mode=0, peak_mode=0):
    A, B = _img_d(A), _img_d(B)
    H, W = A.shape
    nx, ny = W // step, H // step
    disp = np.zeros((2, ny, nx))
    peak = np.zeros((ny, nx))
    flags = np.zeros((ny, nx), np.uint8)
    lib().o_correct(A, B, W, H, win, step, r, warp_mode, peak_mode,
                    None if pred is None else _img_d(pred), disp, peak, flags)
    return disp, peak, flags


def validate(field, flags=None, thr=2.0, eps=0.1):
    f = _img_d(field).copy()
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8).copy()
    lib().o_validate(f, fl, f.shape[2], f.shape[1], thr, eps)
    return f, fl


def vorticity(field, step):
    f = _img_d(field)
    om = np.zeros(f.shape[1:])
    lib().o_vorticity(f, f.shape[2], f.shape[1], step, om)
    return om


def ssd_forward(A, B, U, win, step):
    A, B, U = _img_d(A), _img_d(B), _img_d(U)
    H, W = A.shape
    loss = np.zeros((H // step, W // step))
    lib().o_ssd_forward(A, B, U, W, H, win, step, loss)
    return loss


def ssd_grad(A, B, U, g, win, step, want_diag=True):
    A, B, U, g = _img_d(A), _img_d(B), _img_d(U), _img_d(g)
    H, W = A.shape
    gU = np.zeros_like(U)
    D = np.zeros_like(U) if want_diag else None
    lib().o_ssd_grad(A, B, U, g, W, H, win, step, gU, D)
    return gU, D


def ssd_refine(A, B, U0, win, step, steps=10, tau=4.0 / 9.0, lam_rel=1e-3):
    """Refined field and the total-loss history [steps + 1] (FP64)."""
    A, B = _img_d(A), _img_d(B)
    U = _img_d(U0).copy()
    H, W = A.shape
    hist = np.zeros(steps + 1)
    lib().o_ssd_refine(A, B, U, W, H, win, step, steps, float(tau), float(lam_rel), hist)
    return U, hist


def smooth(field, state, alpha, first):
    """One frame of exponential smoothing; returns (smoothed field, new state)."""
    f = _img_d(field).copy()
    s = np.zeros_like(f) if state is None else _img_d(state).copy()
    lib().o_smooth(f, s, f.size, float(alpha), int(bool(first)))
    return f, s


def smooth_batch(fields, states, slots, alpha):
    """Smoothing of a batch in order: fields [n][2][ny][nx], states
    [nstate][2][ny][nx] (updated copies returned), slot k >= 0 continues
    state k, -1 - k starts it; slots outside [0, nstate) leave their pair
    untouched."""
    out = np.array(fields, dtype=np.float64, copy=True)
    st = np.array(states, dtype=np.float64, copy=True)
    for i, k in enumerate(slots):
        k = int(k)
        first = k < 0
        if first:
            k = -1 - k
        if not 0 <= k < st.shape[0]:
            continue
        out[i], st[k] = smooth(out[i], st[k], alpha, first)
    return out, st


def highpass(img, radius):
    """Background removal: max(0, I - floor(box mean over the image part of
    the (2 radius + 1)^2 box))."""
    I = _img_i(img)
    H, W = I.shape
    out = np.zeros_like(I)
    lib().o_highpass(I, W, H, int(radius), out)
    return out


def clahe_clip(npix, nbins, clip_factor):
    return int(lib().o_clahe_clip(int(npix), int(nbins), float(clip_factor)))


def clahe(img, bits, tiles_x, tiles_y, clip_factor):
    """Contrast-limited adaptive histogram equalisation on a tiles_x x
    tiles_y grid (see oracle.c for the exact reading)."""
    I = _img_i(img)
    H, W = I.shape
    out = np.zeros_like(I)
    lib().o_clahe(I, W, H, int(bits), int(tiles_x), int(tiles_y), float(clip_factor), out)
    return out


def run(A, B, *, win, step, r, levels, block=0, Rc, Rf, median=True, warp_mode=0, peak_mode=0,
        thr=2.0, eps=0.1, sgm=None):
    """The whole plain path: predict, validate the predictor, correct,
    validate, vorticity.  Returns dict of numpy arrays."""
    blk = block or win
    pred = predict(A, B, step, blk, levels, Rc, Rf, median, sgm).astype(np.float64)
    pred, _ = validate(pred, None, thr, eps)
    disp, peak, flags = correct(A, B, win, step, r, pred, warp_mode, peak_mode)
    disp_v, flags_v = validate(disp, flags, thr, eps)
    om = vorticity(disp_v, step)
    return dict(pred=pred, disp_raw=disp, peak=peak, flags_raw=flags, disp=disp_v,
                flags=flags_v, omega=om)


def run_temporal(frames, *, win, step, r, levels, block=0, Rc, Rf, median=True, alpha1=0.5, alpha2=0.5,
                 warp_mode=0, peak_mode=0, thr=2.0, eps=0.1):
    """The path with the paper's temporal smoothing over one stream of
    pairs [(A, B), ...] in time order: predict, validate the predictor,
    smooth it (alpha1), correct about the smoothed predictor, validate,
    smooth the final field (alpha2), vorticity.  alpha None skips that
    smoothing.  Returns one dict per pair."""
    blk = block or win
    sp = sd = None
    outs = []
    for t, (A, B) in enumerate(frames):
        pred = predict(A, B, step, blk, levels, Rc, Rf, median).astype(np.float64)
        pred, _ = validate(pred, None, thr, eps)
        if alpha1 is not None:
            pred, sp = smooth(pred, sp, alpha1, t == 0)
        disp, peak, flags = correct(A, B, win, step, r, pred, warp_mode, peak_mode)
        disp_v, flags_v = validate(disp, flags, thr, eps)
        if alpha2 is not None:
            disp_v, sd = smooth(disp_v, sd, alpha2, t == 0)
        om = vorticity(disp_v, step)
        outs.append(dict(pred=pred, disp_raw=disp, peak=peak, flags_raw=flags, disp=disp_v, flags=flags_v,
                         omega=om))
    return outs
