"""GPU parity of every stage of the hot path with the FP64 oracle, called
through the C ABI (libpiv.so via ctypes).  Integer work (pyramid, SAD
predictor, medians) must be bit-exact; sub-pixel displacements within
0.01 px; correlation-peak indices exact except where the oracle's own plane
shows a near-tie; vorticity within 1e-4 of max |omega|."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import (TOL_DISP_PX, TOL_REL, compare_correct, compare_end_to_end, compare_validate, dilate,
                      say)
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def api():
    from paper_2504_17987_amd import api as A
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def small_vortex_pair(W=256, H=192, seed=7, peak=8.0, dropout=0.1):
    flow = synth.LambOseen.with_peak((W - 1) / 2, (H - 1) / 2, 40.0, peak)
    A, B = synth.make_pair(W, H, flow, 0.04, noise=2.0, dropout=dropout, seed=seed)
    return A, B, flow


PRED_CASES = {
    # name: (image maker, plan kwargs)
    "vortex_L3_16_8": (lambda: small_vortex_pair()[:2],
                       dict(win=16, step=8, levels=3, radius_coarse=6, radius_fine=2)),
    # the cell-shared u8 coarse search with three passes of shift rows (R 7)
    # and one (R 3)
    "coarse_r7_L3": (lambda: small_vortex_pair(seed=19)[:2],
                     dict(win=16, step=8, levels=3, radius_coarse=7, radius_fine=2)),
    "coarse_r3_L3": (lambda: small_vortex_pair(seed=20)[:2],
                     dict(win=16, step=8, levels=3, radius_coarse=3, radius_fine=2)),
    "cfg1_L1_32_16_r8": (lambda: synth.cfg1_pair(1000)[:2],
                         dict(win=32, step=16, levels=1, radius_coarse=8, radius_fine=2, radius=8)),
    # the generic SAD kernel at its widest: 64 px blocks, 33 x 33 candidates
    # (candidate rows in groups of five per thread, one node per workgroup)
    "cfg1_L1_64_32_r16": (lambda: synth.cfg1_pair(1001)[:2],
                          dict(win=64, step=32, levels=1, radius_coarse=16, radius_fine=2, radius=8)),
    "ragged_200x136": (lambda: small_vortex_pair(200, 136, seed=3)[:2],
                       dict(win=16, step=8, levels=3, radius_coarse=5, radius_fine=2)),
    "median_off_L2": (lambda: small_vortex_pair(seed=11)[:2],
                      dict(win=16, step=8, levels=2, radius_coarse=4, radius_fine=1, median=False)),
    "block24_step8": (lambda: small_vortex_pair(seed=12)[:2],
                      dict(win=16, step=8, block=24, levels=3, radius_coarse=3, radius_fine=2)),
    # image rows not a multiple of 4 and a ragged last 32-byte chunk
    "step6_204x138": (lambda: small_vortex_pair(204, 138, seed=13)[:2],
                      dict(win=12, step=6, levels=3, radius_coarse=5, radius_fine=2)),
    # a fine level searched by the lane-per-row kernel (radius above 2, with a parent)
    "fine_r3_L2": (lambda: small_vortex_pair(seed=14)[:2],
                   dict(win=16, step=8, levels=2, radius_coarse=4, radius_fine=3)),
    # 12 px blocks at step 8: the staged quad-SAD coarse level and the
    # one-node-per-lane fine level with unaligned block columns
    "block12_step8": (lambda: small_vortex_pair(seed=15)[:2],
                      dict(win=12, step=8, levels=2, radius_coarse=4, radius_fine=2)),
    # the coarsest level by semi-global matching (three levels, and one level
    # with a wide search), then block matching below
    "sgm_vortex_L3": (lambda: small_vortex_pair(seed=16)[:2],
                      dict(win=16, step=8, levels=3, radius_coarse=6, radius_fine=2, sgm=True)),
    "sgm_cfg1_L1": (lambda: synth.cfg1_pair(1002)[:2],
                    dict(win=32, step=16, levels=1, radius_coarse=8, radius_fine=2, radius=8, sgm=True,
                         sgm_p1=1, sgm_p2=8)),
    "sgm_ragged_L2": (lambda: small_vortex_pair(200, 136, seed=17)[:2],
                      dict(win=16, step=8, levels=2, radius_coarse=5, radius_fine=2, sgm=True, sgm_p1=4,
                           sgm_p2=40)),
    # every candidate count per lane of the path aggregation (1, 4, 8, 12, 18
    # candidates per lane), by the cell kernel's cost volume (R 3 and 7) and
    # by the per-candidate cost kernel (12 px blocks, R above 7)
    "sgm_R3_L2": (lambda: small_vortex_pair(seed=18)[:2],
                  dict(win=16, step=8, levels=2, radius_coarse=3, radius_fine=2, sgm=True)),
    "sgm_R7_L1": (lambda: small_vortex_pair(seed=19)[:2],
                  dict(win=16, step=8, levels=1, radius_coarse=7, radius_fine=2, sgm=True, sgm_p1=3, sgm_p2=24)),
    "sgm_R10_L1_block12": (lambda: small_vortex_pair(seed=20)[:2],
                           dict(win=12, step=8, levels=1, radius_coarse=10, radius_fine=2, sgm=True)),
    "sgm_R13_L2": (lambda: small_vortex_pair(seed=21)[:2],
                   dict(win=16, step=8, levels=2, radius_coarse=13, radius_fine=2, sgm=True)),
    "sgm_R16_L1": (lambda: small_vortex_pair(160, 96, seed=22)[:2],
                   dict(win=16, step=8, levels=1, radius_coarse=16, radius_fine=2, sgm=True, sgm_p1=1, sgm_p2=4)),
}


@pytest.mark.parametrize("case", list(PRED_CASES))
def test_predict_bitexact(case):
    say(f"[predict] {case}")
    make, kw = PRED_CASES[case]
    A, B = make()
    H, W = A.shape
    P = api().Plan(W, H, max_batch=2, **kw)
    Ad, Bd = dev(np.stack([A, B])), dev(np.stack([B, A]))   # two pairs: (A,B) and (B,A)
    pred = P.predict(Ad, Bd).cpu().numpy()
    blk = kw.get("block", 0) or kw["win"]
    sgm = (kw.get("sgm_p1", 2), kw.get("sgm_p2", 16)) if kw.get("sgm") else None
    for i, (a, b) in enumerate([(A, B), (B, A)]):
        ref = oracle.predict(a, b, kw["step"], blk, kw["levels"], kw["radius_coarse"],
                             kw["radius_fine"], kw.get("median", True), sgm)
        assert np.array_equal(pred[i], ref.astype(np.float32)), f"pair {i}"


# every coarse radius of the cell-shared u16 search (its waves take 2, 3, 4,
# 5 and 5 passes of shift rows for R 3..7)
@pytest.mark.parametrize("rc", [3, 4, 5, 6, 7])
def test_predict_u16_bitexact(rc):
    say(f"[predict] u16 step 12, coarse radius {rc}")
    A, B, _ = synth.cfg3_pair(0, W=384, H=216)
    P = api().Plan(384, 216, dtype="u16", win=24, step=12, levels=3, radius_coarse=rc, radius_fine=2)
    pred = P.predict(dev(A[None].view(np.int16)).view(torch.uint16),
                     dev(B[None].view(np.int16)).view(torch.uint16)).cpu().numpy()[0]
    ref = oracle.predict(A, B, 12, 24, 3, rc, 2)
    assert np.array_equal(pred, ref.astype(np.float32))


def test_predict_u16_sgm_bitexact():
    say("[predict] u16 step 12, semi-global coarsest level")
    A, B, _ = synth.cfg3_pair(2, W=384, H=216)
    P = api().Plan(384, 216, dtype="u16", win=24, step=12, levels=3, radius_coarse=6, radius_fine=2, sgm=True)
    pred = P.predict(dev(A[None].view(np.int16)).view(torch.uint16),
                     dev(B[None].view(np.int16)).view(torch.uint16)).cpu().numpy()[0]
    ref = oracle.predict(A, B, 12, 24, 3, 6, 2, sgm=(2, 16))
    assert np.array_equal(pred, ref.astype(np.float32))


def test_run_end_to_end_sgm_predictor():
    """The whole path with the semi-global coarsest level (strong vortex),
    stage by stage against the oracle; accuracy against the truth reported
    beside the block-matching predictor's."""
    say("[run] semi-global predictor, strong vortex")
    flow = synth.LambOseen.with_peak(127.5, 95.5, 40.0, 8.0)
    A, B = synth.make_pair(256, 192, flow, 0.04, noise=2.0, dropout=0.1, seed=7)
    kw = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    g, o = _run_both(A, B, dict(kw, sgm=True), "run[sgm]", sgm=(2, 16))
    T = synth.truth(flow, 256, 192, 8)
    e = lambda d: np.sqrt(((d - T)[:, 2:-2, 2:-2] ** 2).mean())
    ob = oracle.run(A, B, win=16, step=8, r=4, levels=3, Rc=6, Rf=2)
    say(f"  vs truth: rms {e(g['disp']):.3f} px with the semi-global level, {e(ob['disp']):.3f} px with block "
        f"matching")


# u16 coarse searches wider than the lane-per-row kernel takes (2R+1 > 17):
# the general kernel with its candidate rows in groups, with the band staged
@pytest.mark.parametrize("rc", [10, 16])
def test_predict_u16_wide_coarse_bitexact(rc):
    say(f"[predict] u16 16/8, coarse radius {rc}")
    A, B, _ = synth.cfg3_pair(3, W=256, H=192)
    P = api().Plan(256, 192, dtype="u16", win=16, step=8, levels=2, radius_coarse=rc, radius_fine=2)
    pred = P.predict(dev(A[None].view(np.int16)).view(torch.uint16),
                     dev(B[None].view(np.int16)).view(torch.uint16)).cpu().numpy()[0]
    ref = oracle.predict(A, B, 8, 16, 2, rc, 2)
    assert np.array_equal(pred, ref.astype(np.float32))


@pytest.mark.parametrize("W,H,step,win", [(200, 136, 8, 16), (204, 204, 12, 24)])
def test_predict_u16_ragged_bitexact(W, H, step, win):
    """u16 frames with ragged pyramid edges (204 px rows are not a whole
    number of 16-byte chunks; 204 rows give odd level-2 heights): levels 1
    and 2 come from one pass over the frames."""
    say(f"[predict] u16 ragged {W}x{H} step {step}")
    A, B, _ = synth.cfg3_pair(1, W=W, H=H)
    P = api().Plan(W, H, dtype="u16", win=win, step=step, levels=3, radius_coarse=5, radius_fine=2)
    pred = P.predict(dev(A[None].view(np.int16)).view(torch.uint16),
                     dev(B[None].view(np.int16)).view(torch.uint16)).cpu().numpy()[0]
    ref = oracle.predict(A, B, step, win, 3, 5, 2)
    assert np.array_equal(pred, ref.astype(np.float32))


def test_predict_equal_frames_is_zero():
    say("[predict] A = B")
    A, _, _ = small_vortex_pair()
    P = api().Plan(256, 192, win=16, step=8)
    pred = P.predict(dev(A[None]), dev(A[None])).cpu().numpy()
    assert (pred == 0).all()


def _u16(x):
    return dev(np.ascontiguousarray(x).view(np.int16)).view(torch.uint16)


CORR_CASES = {
    # name: (images, plan kwargs, use predictor)
    "tiled_u8_8_r4": ("vortex", dict(win=16, step=8, radius=4), True),
    "generic_u8_8_r3": ("vortex", dict(win=16, step=8, radius=3), True),
    "generic_u8_cfg1_r8": ("cfg1", dict(win=32, step=16, radius=8, levels=1, radius_coarse=8), False),
    "tiled_u8_central": ("vortex", dict(win=16, step=8, radius=4, warp="central"), True),
    "tiled_u8_fixed": ("vortex_small", dict(win=16, step=8, radius=4, peak="fixed"), True),
    "generic_u8_fixed_16": ("cfg1", dict(win=32, step=16, radius=8, levels=1, radius_coarse=8, peak="fixed"), False),
    "generic_u8_win24_8": ("vortex", dict(win=24, step=8, radius=4, block=16), True),
    "tiled_u16_12_r4": ("u16", dict(dtype="u16", win=24, step=12, radius=4), True),
    "tiled_u8_ragged": ("ragged", dict(win=16, step=8, radius=4, radius_coarse=5), True),
    "tiled_u16_8_r4": ("u16", dict(dtype="u16", win=16, step=8, radius=4), True),
    "tiled_u16_8_fixed": ("u16", dict(dtype="u16", win=16, step=8, radius=4, peak="fixed"), True),
    "tiled_u8_8_nopred": ("vortex_small", dict(win=16, step=8, radius=4), False),
    # displacements of 16 px: a tile's predictor range decides the staged box
    "tiled_u8_vortex16_r1": ("vortex16", dict(win=16, step=8, radius=1), True),
    "tiled_u8_vortex16_fixed": ("vortex16", dict(win=16, step=8, radius=4, peak="fixed"), True),
    "tiled_u8_vortex16_r4": ("vortex16", dict(win=16, step=8, radius=4), True),
    # central deformation on the generic kernel, on u16 frames, and the
    # fixed-centre stencil with a predictor on the generic kernel
    "generic_u8_central_r3": ("vortex", dict(win=16, step=8, radius=3, warp="central"), True),
    "generic_u8_cfg1_central": ("cfg1", dict(win=32, step=16, radius=8, levels=1, radius_coarse=8,
                                             warp="central"), True),
    "tiled_u16_12_central": ("u16", dict(dtype="u16", win=24, step=12, radius=4, warp="central"), True),
    "tiled_u16_8_central": ("u16", dict(dtype="u16", win=16, step=8, radius=4, warp="central"), True),
    "generic_u8_fixed_pred": ("vortex", dict(win=24, step=8, radius=4, block=16, peak="fixed"), True),
    # the low-seeding wake (0.002 ppp, 32 x 32 windows at 50% step-over):
    # the a-priori stencil and the argmax search
    "wake_fixed_32_16": ("wake", dict(win=32, step=16, radius=4, levels=2, radius_coarse=6, peak="fixed"), True),
    "wake_argmax_32_16": ("wake", dict(win=32, step=16, radius=4, levels=2, radius_coarse=6), True),
    # the generic kernel at the largest geometries the plan accepts: a window
    # of 64 px with 33 x 33 shifts (one row part per shift, 83 KB of LDS),
    # and 48 px with 25 x 25 shifts (row parts of a 1,024-thread workgroup)
    "generic_u8_win64_r16": ("cfg1", dict(win=64, step=32, radius=16, levels=1, radius_coarse=8), False),
    "generic_u8_win48_r12": ("cfg1", dict(win=48, step=16, radius=12, levels=1, radius_coarse=8), False),
}


def _images(kind):
    if kind == "vortex":
        return small_vortex_pair()[:2]
    if kind == "vortex_small":
        return small_vortex_pair(peak=0.8, seed=5)[:2]
    if kind == "vortex16":
        return small_vortex_pair(peak=16.0, seed=9)[:2]
    if kind == "ragged":
        return small_vortex_pair(200, 136, seed=3)[:2]
    if kind == "cfg1":
        return synth.cfg1_pair(1001)[:2]
    if kind == "u16":
        return synth.cfg3_pair(1, W=384, H=216)[:2]
    if kind == "wake":
        return synth.make_pair(512, 256, synth.cylinder_wake(512, 256), 0.002, noise=2.0, seed=7100)
    raise KeyError(kind)


@pytest.mark.parametrize("case", list(CORR_CASES))
def test_correct_parity(case):
    say(f"[correct] {case}")
    kind, kw, use_pred = CORR_CASES[case]
    A, B = _images(kind)
    H, W = A.shape
    P = api().Plan(W, H, max_batch=1, **kw)
    blk = kw.get("block", 0) or kw["win"]
    pred = None
    if use_pred:
        pred = oracle.predict(A, B, kw["step"], blk, kw.get("levels", 3), kw.get("radius_coarse", 6),
                              kw.get("radius_fine", 2)).astype(np.float64)
        pred, _ = oracle.validate(pred, None)
    mode = 1 if kw.get("warp") == "central" else 0
    fixed = kw.get("peak") == "fixed"
    disp_o, peak_o, flags_o = oracle.correct(A, B, kw["win"], kw["step"], kw["radius"], pred, mode,
                                             1 if fixed else 0)
    if kind == "u16":
        Ad, Bd = _u16(A[None]), _u16(B[None])
    else:
        Ad, Bd = dev(A[None]), dev(B[None])
    pg = None if pred is None else dev(pred[None].astype(np.float32))
    disp, peak, flags = P.correct(Ad, Bd, pg)
    say(f"  impl={P.correct_impl()}")
    compare_correct(Ad, Bd, A.astype(float), B.astype(float), kw["win"], kw["step"], kw["radius"],
                    pred, disp.cpu().numpy()[0], peak.cpu().numpy()[0], flags.cpu().numpy()[0],
                    disp_o, peak_o, flags_o, mode=mode, fixed=fixed, where=f"correct[{case}]")


STRETCH = 0.6


def _stretch(x, y):
    x = np.asarray(x, dtype=np.float64)
    return STRETCH * (x - 128.0), np.zeros_like(x)


def _stretch_pred():
    # the pair renders particles at midpoint -/+ u/2, so in the frame of A the
    # correspondence is s / (1 - s/2) (x - 128)
    X, _ = synth.node_centres(256, 192, 8)
    u = STRETCH / (1.0 - STRETCH / 2.0) * (X - 128.0)
    return np.stack([u, np.zeros_like(u)]).astype(np.float32).astype(np.float64)


# predictors far from zero or steep across a tile: the deformation then reads
# the frame with checked loads instead of a staged box
WILD_CASES = {
    # |d| >= 100 px at every node
    "far_uniform": (synth.Uniform(104.3, -2.6),
                    lambda: np.round(synth.truth(synth.Uniform(104.3, -2.6), 256, 192, 8))),
    # the predictor spans more than 64 px across every tile
    "steep_stretch": (_stretch, _stretch_pred),
}


@pytest.mark.parametrize("case", list(WILD_CASES))
def test_correct_parity_wild_predictor(case):
    say(f"[correct] {case}")
    flow, make_pred = WILD_CASES[case]
    A, B = synth.make_pair(256, 192, flow, 0.04, noise=2.0, seed=31, margin=240)
    kw = dict(win=16, step=8, radius=4)
    pred = make_pred()
    P = api().Plan(256, 192, max_batch=1, **kw)
    disp_o, peak_o, flags_o = oracle.correct(A, B, 16, 8, 4, pred, 0, 0)
    Ad, Bd = dev(A[None]), dev(B[None])
    disp, peak, flags = P.correct(Ad, Bd, dev(pred[None].astype(np.float32)))
    compare_correct(Ad, Bd, A.astype(float), B.astype(float), 16, 8, 4, pred, disp.cpu().numpy()[0],
                    peak.cpu().numpy()[0], flags.cpu().numpy()[0], disp_o, peak_o, flags_o, where=f"wild[{case}]")
    say(f"  flat windows {int((flags_o & 1).sum())}")


def test_correct_impl_selection():
    assert api().Plan(256, 192, win=16, step=8, radius=4).correct_impl() == 1
    assert api().Plan(256, 192, win=16, step=8, radius=3).correct_impl() == 0
    assert api().Plan(384, 216, dtype="u16", win=24, step=12, radius=4).correct_impl() == 1


def test_validate_parity():
    say("[validate]")
    rng = np.random.default_rng(71)
    ny, nx = 37, 53
    f = rng.normal(0, 0.4, (2, ny, nx))
    k = 120
    f[:, rng.integers(0, ny, k), rng.integers(0, nx, k)] += rng.normal(0, 5, (2, k))
    f = f.astype(np.float32).astype(np.float64)
    flags = ((rng.random((ny, nx)) < 0.05) * 2 + (rng.random((ny, nx)) < 0.03) * 1).astype(np.uint8)
    go, flo = oracle.validate(f, flags)
    P = api().Plan(nx * 8, ny * 8, win=16, step=8)
    fg = dev(f[None].astype(np.float32))
    flg = dev(flags[None])
    P.validate(fg, flg)
    g, fl = fg.cpu().numpy()[0], flg.cpu().numpy()[0]
    compare_validate(f, flags, g, fl, go, flo, where="validate[flags]")
    # predictor-style call without flags
    f2 = dev(f[None].astype(np.float32))
    P.validate(f2, None)
    g2, _ = oracle.validate(f, None)
    z = np.zeros((ny, nx), np.uint8)
    compare_validate(f, None, f2.cpu().numpy()[0], z, g2, z, where="validate[no flags]")


def test_validate_parity_tiles():
    """Several pairs on a grid of several ragged 32 x 8 tiles, with outlier
    clusters across tile edges and FLAT/BORDER flags, against the oracle."""
    say("[validate] tiles")
    rng = np.random.default_rng(73)
    n, ny, nx = 3, 29, 70
    f = rng.normal(0, 0.4, (n, 2, ny, nx))
    for p in range(n):
        for (y, x) in [(7, 31), (8, 32), (15, 63), (16, 64), (0, 0), (28, 69), (23, 31), (24, 32)]:
            f[p, :, max(0, y - 1):y + 2, max(0, x - 1):x + 2] += rng.normal(0, 6, (2, 1, 1))
        k = 200
        f[p, :, rng.integers(0, ny, k), rng.integers(0, nx, k)] += rng.normal(0, 5, (k, 2))
    f = f.astype(np.float32).astype(np.float64)
    flags = ((rng.random((n, ny, nx)) < 0.05) * 2 + (rng.random((n, ny, nx)) < 0.03) * 1).astype(np.uint8)
    P = api().Plan(nx * 8, ny * 8, win=16, step=8, max_batch=n)
    fg = dev(f.astype(np.float32))
    flg = dev(flags)
    P.validate(fg, flg)
    for p in range(n):
        go, flo = oracle.validate(f[p], flags[p])
        g, fl = fg.cpu().numpy()[p], flg.cpu().numpy()[p]
        compare_validate(f[p], flags[p], g, fl, go, flo, where=f"validate[tiles, pair {p}]")


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_run_equals_separate_steps(dtype):
    """piv_run (predictor output and its validation in one kernel; the
    correction written to the workspace and validated from there) gives the
    same bits as predict, validate, correct, validate, vorticity called one
    by one."""
    say(f"[run] separate steps {dtype}")
    pairs = [small_vortex_pair(seed=s)[:2] for s in (41, 42)]
    A = np.stack([p[0] for p in pairs])
    B = np.stack([p[1] for p in pairs])
    if dtype == "u16":
        A, B = A.astype(np.uint16) * 181, B.astype(np.uint16) * 181
    P = api().Plan(256, 192, max_batch=2, win=16, step=8, dtype=dtype)
    Ag, Bg = dev(A), dev(B)
    out = P.run(Ag, Bg)
    pred = P.predict(Ag, Bg)
    P.validate(pred, None)
    disp, peak, flags = P.correct(Ag, Bg, pred)
    P.validate(disp, flags)
    omega = P.vorticity(disp)
    for k, v in (("pred", pred), ("disp", disp), ("peak", peak), ("flags", flags), ("omega", omega)):
        assert torch.equal(out[k], v), k


def test_two_plans_on_two_streams_equal_alone():
    """Two plans running the whole path at once on two HIP streams (two
    batches in flight, as the benchmark runs them) give the same bits as
    each batch run alone: the plans share no workspace."""
    say("[run] two plans on two streams")
    pairs = [small_vortex_pair(seed=s)[:2] for s in (43, 44, 45, 46)]
    A = np.stack([p[0] for p in pairs])
    B = np.stack([p[1] for p in pairs])
    P1 = api().Plan(256, 192, max_batch=2, win=16, step=8)
    P2 = api().Plan(256, 192, max_batch=2, win=16, step=8)
    A1, B1, A2, B2 = dev(A[:2]), dev(B[:2]), dev(A[2:]), dev(B[2:])
    ref1 = {k: v.clone() for k, v in P1.run(A1, B1).items()}
    ref2 = {k: v.clone() for k, v in P2.run(A2, B2).items()}
    torch.cuda.synchronize()
    o1 = {k: torch.empty_like(v) for k, v in ref1.items()}
    o2 = {k: torch.empty_like(v) for k, v in ref2.items()}
    main = torch.cuda.current_stream()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(3):
        for o in (o1, o2):
            for v in o.values():
                v.zero_()
        s1.wait_stream(main)
        s2.wait_stream(main)
        for _ in range(4):
            with torch.cuda.stream(s1):
                P1.run(A1, B1, o1)
            with torch.cuda.stream(s2):
                P2.run(A2, B2, o2)
        main.wait_stream(s1)
        main.wait_stream(s2)
        torch.cuda.synchronize()
        for k in ref1:
            assert torch.equal(o1[k], ref1[k]), (it, "first", k)
            assert torch.equal(o2[k], ref2[k]), (it, "second", k)


def test_vorticity_parity():
    say("[vorticity]")
    lo = synth.cfg2_flow()
    U = synth.truth(lo, 1024, 1024, 8)
    rng = np.random.default_rng(72)
    U = (U + rng.normal(0, 0.05, U.shape)).astype(np.float32).astype(np.float64)
    P = api().Plan(1024, 1024, win=16, step=8)
    om = P.vorticity(dev(U[None].astype(np.float32))).cpu().numpy()[0]
    ref = oracle.vorticity(U, 8)
    assert np.abs(om - ref).max() <= TOL_REL * np.abs(ref).max()
    # solid body gives 2 omega
    sb = synth.SolidBody(500.0, 480.0, 0.01)
    S = synth.truth(sb, 1024, 1024, 8)
    om = P.vorticity(dev(S[None].astype(np.float32))).cpu().numpy()[0]
    assert np.abs(om - 0.02).max() < 1e-4 * 0.02 + 1e-6


def _run_both(A, B, kw, where, peak_mode=0, sgm=None):
    """The whole path on the GPU (piv_run) and in the oracle, compared stage
    by stage on identical inputs, every difference explained:
    the predictor bit-exact; the raw correction (piv_correct on the run's
    predictor, the kernel piv_run uses) against the oracle's; validation of
    that raw field against the oracle's validation of the same field; the
    final field against the oracle's only where a raw exemption or a
    near-threshold decision lies in the 3x3 neighbourhood; vorticity of the
    GPU's final field within 1e-4 of its max."""
    H, W = A.shape
    P = api().Plan(W, H, max_batch=1, **kw)
    Ad, Bd = dev(A[None]), dev(B[None])
    out = P.run(Ad, Bd)
    raw, peak, flags = P.correct(Ad, Bd, out["pred"])
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy()[0] for k, v in out.items()}
    raw, peak, flags = raw.cpu().numpy()[0], peak.cpu().numpy()[0], flags.cpu().numpy()[0]
    o = oracle.run(A, B, win=kw["win"], step=kw["step"], r=kw["radius"], levels=kw["levels"],
                   Rc=kw["radius_coarse"], Rf=kw["radius_fine"], peak_mode=peak_mode, sgm=sgm)
    assert np.array_equal(g["pred"], o["pred"].astype(np.float32)), f"{where}: predictor"
    raw_ex = compare_correct(None, None, A.astype(float), B.astype(float), kw["win"], kw["step"], kw["radius"],
                             o["pred"], raw, peak, flags, o["disp_raw"], o["peak"], o["flags_raw"],
                             fixed=peak_mode == 1, where=f"{where} raw")
    vo, flo = oracle.validate(raw.astype(np.float64), flags.copy())
    uod_ex = compare_validate(raw.astype(np.float64), flags, g["disp"], g["flags"], vo, flo,
                              where=f"{where} validate")
    compare_end_to_end(g["disp"], o["disp"], raw_ex, uod_ex, where=f"{where} end-to-end")
    om = oracle.vorticity(g["disp"].astype(np.float64), kw["step"])
    assert np.abs(g["omega"] - om).max() <= TOL_REL * np.abs(om).max(), f"{where}: vorticity"
    return g, o


def test_run_end_to_end_vortex():
    say("[run] vortex 256x192")
    flow = synth.LambOseen.with_peak(127.5, 95.5, 60.0, 6.0)
    A, B = synth.make_pair(256, 192, flow, 0.04, noise=2.0, dropout=0.1, seed=7)
    kw = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    g, o = _run_both(A, B, kw, "run[vortex]")
    d = np.abs(g["disp"] - o["disp"]).max(axis=0)
    say(f"  max |d disp| {d.max():.2e}")
    # accuracy against the analytic truth (reported; loose bound)
    T = synth.truth(flow, 256, 192, 8)
    err = np.abs(g["disp"] - T)[:, 2:-2, 2:-2]
    say(f"  vs truth: rms {np.sqrt((err ** 2).mean()):.3f} px, max {err.max():.3f} px")
    assert np.sqrt((err ** 2).mean()) < 0.25   # the oracle itself: 0.18 px on this pair


def test_run_end_to_end_strong_vortex():
    """The stronger vortex (core 40 px, 8 px peak) the gentler case above
    replaced: the same stage-by-stage comparison; accuracy against the truth
    is reported only."""
    say("[run] strong vortex 256x192")
    flow = synth.LambOseen.with_peak(127.5, 95.5, 40.0, 8.0)
    A, B = synth.make_pair(256, 192, flow, 0.04, noise=2.0, dropout=0.1, seed=7)
    kw = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    g, o = _run_both(A, B, kw, "run[strong vortex]")
    T = synth.truth(flow, 256, 192, 8)
    err = np.abs(g["disp"] - T)[:, 2:-2, 2:-2]
    say(f"  vs truth: rms {np.sqrt((err ** 2).mean()):.3f} px (oracle "
        f"{np.sqrt(((o['disp'] - T)[:, 2:-2, 2:-2] ** 2).mean()):.3f} px)")


@pytest.mark.parametrize("peak", ["fixed", "argmax"])
def test_run_end_to_end_low_seeding_wake(peak):
    """The low-seeding case (0.002 ppp cylinder-like wake, 32 x 32 windows
    at step 16, two-level predictor): the whole path stage by stage against
    the oracle, with the a-priori stencil and with the argmax search."""
    say(f"[run] low-seeding wake, {peak}")
    A, B = synth.make_pair(512, 256, synth.cylinder_wake(512, 256), 0.002, noise=2.0, seed=7101)
    kw = dict(win=32, step=16, radius=4, levels=2, radius_coarse=6, radius_fine=2, peak=peak)
    g, o = _run_both(A, B, kw, f"run[wake {peak}]", peak_mode=1 if peak == "fixed" else 0)
    T = synth.truth(synth.cylinder_wake(512, 256), 512, 256, 16)
    err = np.abs(g["disp"] - T)[:, 2:-2, 2:-2]
    say(f"  vs truth: rms {np.sqrt((err ** 2).mean()):.3f} px")


def test_run_end_to_end_cfg1():
    say("[run] config-1 plain path L=1")
    A, B, flow = synth.cfg1_pair(1000)
    kw = dict(win=32, step=16, radius=8, levels=1, radius_coarse=8, radius_fine=2)
    g, o = _run_both(A, B, kw, "run[cfg1]")
    d = np.abs(g["disp"] - o["disp"]).max(axis=0)
    assert (d <= TOL_DISP_PX).all(), d.max()
    # pred = NULL ("plain" correction only)
    P = api().Plan(256, 256, win=32, step=16, radius=8, levels=1, radius_coarse=8)
    disp, peak, flags = P.correct(dev(A[None]), dev(B[None]), None)
    do, po, fo = oracle.correct(A, B, 32, 16, 8, None)
    compare_correct(None, None, A.astype(float), B.astype(float), 32, 16, 8, None, disp.cpu().numpy()[0],
                    peak.cpu().numpy()[0], flags.cpu().numpy()[0], do, po, fo, where="correct[cfg1 plain]")


def test_blank_images_are_flat():
    say("[correct] blank")
    Z = np.zeros((1, 128, 128), np.uint8)
    P = api().Plan(128, 128, win=16, step=8)
    out = P.run(dev(Z), dev(Z))
    fl = out["flags"].cpu().numpy()
    assert (fl & 1).all() and (out["pred"].cpu().numpy() == 0).all()
    assert np.isfinite(out["disp"].cpu().numpy()).all()


def test_batch_invariance_and_determinism():
    say("[run] batch invariance")
    pairs = [small_vortex_pair(seed=s)[:2] for s in (21, 22, 23)]
    A = np.stack([p[0] for p in pairs])
    B = np.stack([p[1] for p in pairs])
    P = api().Plan(256, 192, max_batch=3, win=16, step=8)
    full = P.run(dev(A), dev(B))
    again = P.run(dev(A), dev(B))
    for k in full:
        assert torch.equal(full[k], again[k]), k
    for i in range(3):
        one = P.run(dev(A[i:i + 1]), dev(B[i:i + 1]))
        for k in ("pred", "disp", "flags", "omega"):
            assert torch.equal(one[k][0], full[k][i]), (i, k)


def test_padded_rows_equal_packed_rows():
    """Frames whose rows are longer than the image (pitch = width + 68 bytes)
    give the same bits as packed frames: the pyramid copy, the in-place
    level-0 search and the correlation all address rows by the pitch."""
    say("[run] padded rows")
    pairs = [small_vortex_pair(seed=s)[:2] for s in (51, 52)]
    A = np.stack([p[0] for p in pairs])
    B = np.stack([p[1] for p in pairs])
    n, H, W = A.shape
    P = api().Plan(W, H, max_batch=2, win=16, step=8)
    ref = P.run(dev(A), dev(B))
    Aw = torch.zeros((n, H, W + 68), dtype=torch.uint8, device="cuda")
    Bw = torch.zeros_like(Aw)
    Aw[:, :, :W] = dev(A)
    Bw[:, :, :W] = dev(B)
    Aw[:, :, W:] = 255   # bytes past the image row must not be read as image
    Bw[:, :, W:] = 255
    out = P.run(Aw[:, :, :W], Bw[:, :, :W])
    for k in ("pred", "disp", "flags", "omega"):
        assert torch.equal(out[k], ref[k]), k


def test_slot_mask_skips_pairs():
    say("[run] slot mask")
    pairs = [small_vortex_pair(seed=s)[:2] for s in (31, 32)]
    A = dev(np.stack([p[0] for p in pairs]))
    B = dev(np.stack([p[1] for p in pairs]))
    P = api().Plan(256, 192, max_batch=2, win=16, step=8)
    ref = P.run(A, B)
    out = {k: torch.full_like(v, 7) for k, v in ref.items()}
    mask = torch.tensor([0, 1], dtype=torch.uint8, device="cuda")
    P.bind_slot_mask(mask)
    P.run(A, B, out)
    P.bind_slot_mask(None)
    for k in ("pred", "disp", "flags", "omega"):
        assert (out[k][0] == 7).all() and torch.equal(out[k][1], ref[k][1]), k
