"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every symbol include/piv.h declares; piv_plan validates parameters;
entry points reject bad arguments before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2504_17987_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2504_17987_amd import build
        build.build(verbose=False)
    return _lib


def test_exports_match_header(L):
    hdr = open(os.path.join(ROOT, "include", "piv.h")).read()
    declared = set(re.findall(r"\b(piv_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name


def plan(L, **kw):
    p = L.Params()
    L.lib().piv_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    s = L.lib().piv_plan(C.byref(p), C.byref(h))
    return s, h


def test_defaults_are_the_papers(L):
    p = L.Params()
    L.lib().piv_params_default(C.byref(p))
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_params.json")))
    assert p.win == g["window_px"] and p.step == g["window_px"] * (1 - g["step_over"])
    assert abs(p.uod_threshold - g["uod_threshold"]) < 1e-7
    assert abs(p.uod_epsilon - g["uod_regulariser_px"]) < 1e-7


@pytest.mark.parametrize("kw,status", [
    (dict(win=15), 1), (dict(win=4), 1), (dict(width=1020), 1), (dict(radius=0), 1),
    (dict(radius=17), 1), (dict(levels=7), 1), (dict(dtype=9), 1), (dict(win=66, step=8), 1),
    (dict(radius_coarse=30, levels=4), 1), (dict(max_batch=0), 1),
    (dict(dtype=2, bit_depth=10), 1), (dict(dtype=3, levels=3), 2), (dict(block=36), 2),
    (dict(), 0), (dict(dtype=2, bit_depth=12, win=24, step=12, width=3840, height=2160), 0),
    (dict(sgm=2), 1), (dict(sgm=1, sgm_p2=256), 1), (dict(sgm=1, radius_coarse=0), 1), (dict(sgm=1), 0),
])
def test_plan_validation(L, kw, status):
    s, h = plan(L, **kw)
    assert s == status, L.lib().piv_last_error()
    if s == 0:
        L.lib().piv_plan_destroy(h)
    else:
        assert not h.value and L.lib().piv_last_error()


def test_workspace_and_argument_errors(L):
    """Argument errors come back before any launch.  Binding a workspace to
    a U8 plan enqueues the zeroing of its margins, so the successful binds
    here use an F32 plan (no pyramid, no device work) and a pointer that is
    never dereferenced."""
    s, h = plan(L, max_batch=4)
    assert s == 0
    lib = L.lib()
    per = lib.piv_plan_workspace_bytes(h, 1)
    assert per > 0 and lib.piv_plan_workspace_bytes(h, 4) == 4 * per
    fake = C.c_void_p(1 << 20)   # never dereferenced: calls fail before any launch
    # no workspace bound
    assert lib.piv_predict(h, fake, fake, 1024, 1, fake, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_run(h, fake, fake, 1024, 1, fake, fake, None, fake, fake, None) == L.PIV_ENOWORKSPACE
    # misaligned workspace and too small workspace (rejected before the margins are touched)
    assert lib.piv_plan_bind_workspace(h, C.c_void_p((1 << 20) + 4), per, None) == L.PIV_EINVAL
    assert lib.piv_plan_bind_workspace(h, fake, per - 1, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_predict(h, fake, fake, 1024, 5, fake, None) == L.PIV_EINVAL      # n > max_batch
    assert lib.piv_correct(h, fake, fake, 1022, 1, None, fake, None, fake, None) == L.PIV_EINVAL  # pitch
    assert lib.piv_correct(h, None, fake, 1024, 1, None, fake, None, fake, None) == L.PIV_EINVAL
    assert lib.piv_correct(h, fake, fake, 1024, 1, None, None, None, fake, None) == L.PIV_EINVAL
    assert lib.piv_ssd_forward(h, fake, fake, fake, 1, fake, None) == L.PIV_EINVAL  # not an F32 plan
    assert lib.piv_ssd_refine(h, fake, fake, fake, 1, 10, 0.5, 1e-3, None, None) == L.PIV_EINVAL
    # smoothing: NULL state/slot, nstate, alpha out of (0, 1]
    assert lib.piv_smooth(h, fake, None, fake, 1, 0.5, 1, None) == L.PIV_EINVAL
    assert lib.piv_smooth(h, fake, fake, fake, 0, 0.5, 1, None) == L.PIV_EINVAL
    assert lib.piv_smooth(h, fake, fake, fake, 1, 0.0, 1, None) == L.PIV_EINVAL
    assert lib.piv_smooth(h, fake, fake, fake, 1, 1.5, 1, None) == L.PIV_EINVAL
    assert lib.piv_smooth(h, fake, fake, fake, 1, 0.5, 0, None) == 0                 # n = 0: no-op
    assert lib.piv_run_temporal(h, fake, fake, 1024, 1, None, 1, fake, fake, 0.5, 0.5, fake, fake, None,
                                fake, fake, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_status_string(3) == b"PIV_ENOWORKSPACE"
    # n = 0 is a no-op that succeeds
    assert lib.piv_vorticity(h, fake, fake, 0, None) == 0
    lib.piv_plan_destroy(h)
    # F32 plan: binding does no device work
    s, f = plan(L, max_batch=4, dtype=3, levels=1, width=64, height=64)
    assert s == 0
    perf = lib.piv_plan_workspace_bytes(f, 1)
    assert lib.piv_ssd_refine(f, fake, fake, fake, 1, 10, 0.5, 1e-3, None, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_plan_bind_workspace(f, fake, 2 * perf, None) == 0
    assert lib.piv_ssd_refine(f, fake, fake, fake, 3, 10, 0.5, 1e-3, None, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_ssd_refine(f, fake, fake, fake, 5, 10, 0.5, 1e-3, None, None) == L.PIV_EINVAL
    assert lib.piv_ssd_refine(f, fake, fake, fake, 1, 10, 0.0, 1e-3, None, None) == L.PIV_EINVAL   # tau
    assert lib.piv_ssd_refine(f, fake, fake, fake, 1, 10, 0.5, -1.0, None, None) == L.PIV_EINVAL   # lam_rel
    assert lib.piv_ssd_refine(f, fake, fake, fake, 1, -1, 0.5, 1e-3, None, None) == L.PIV_EINVAL   # steps
    assert lib.piv_ssd_refine(f, fake, fake, fake, 0, 10, 0.5, 1e-3, None, None) == 0              # n = 0
    assert lib.piv_predict(f, fake, fake, 256, 1, fake, None) == L.PIV_EUNSUPPORTED
    lib.piv_plan_destroy(f)


def test_f32_workspace_holds_refinement_fields(L):
    """F32 plans size their workspace for the refinement's gradient and
    diagonal ([2][ny][nx] each) and window losses ([ny][nx]) per pair."""
    lib = L.lib()
    s, f = plan(L, dtype=3, levels=1, width=512, height=512)
    s2, u = plan(L, dtype=1, levels=1, width=512, height=512)
    assert s == 0 and s2 == 0
    np_ = 64 * 64
    assert lib.piv_plan_workspace_bytes(f, 1) >= 5 * 4 * np_ + 2 * 4 * np_
    lib.piv_plan_destroy(f)
    lib.piv_plan_destroy(u)


def _levels(L, **kw):
    s, h = plan(L, **kw)
    assert s == 0, L.lib().piv_last_error()
    lib = L.lib()
    lib.piv_debug_level.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    out = []
    l = 0
    while True:
        buf = (C.c_int32 * 11)()
        if lib.piv_debug_level(h, l, buf) != 0:
            break
        out.append(dict(zip("W H margin pitch rows R nx ny es step block".split(), list(buf))))
        l += 1
    lib.piv_plan_destroy(h)
    return out


PLANS = [
    dict(),                                                                   # 1 MP, 16/8, L3, 6/2
    dict(width=256, height=256, win=32, step=16, radius=8, levels=1, radius_coarse=8),
    dict(width=3840, height=2160, dtype=2, bit_depth=12, win=24, step=12, levels=3),
    dict(width=200, height=136, levels=3, radius_coarse=5),
    dict(width=2048, height=2048),
    dict(width=1000, height=504, levels=4, radius_coarse=4, radius_fine=3),
    dict(width=96, height=40, win=24, step=8, block=16, levels=2, radius_coarse=16, radius_fine=16),
    dict(width=512, height=512, levels=6, radius_coarse=3, radius_fine=1),
    dict(width=64, height=64, win=8, step=8, block=8, levels=1, radius_coarse=0),
    dict(width=640, height=480, dtype=2, bit_depth=16, win=16, step=8, levels=3, radius_coarse=8, radius_fine=1),
    dict(width=512, height=512, dtype=2, bit_depth=12, win=32, step=16, levels=2, radius_coarse=4, radius_fine=2),
]


@pytest.mark.parametrize("kw", PLANS)
def test_padded_pyramid_holds_every_sad_read(L, kw):
    """Every byte the SAD kernels and the pyramid read lies inside the padded
    level buffer, for the largest candidate centre the level can see."""
    lv = _levels(L, **kw)
    maxd_parent = 0
    for l in range(len(lv) - 1, -1, -1):
        v = lv[l]
        es, step, blk, R, M = v["es"], v["step"], v["block"], v["R"], v["margin"]
        cand = 0 if l == len(lv) - 1 else 2 * maxd_parent
        maxd_parent = cand + R
        off = (step - blk) // 2
        NW = blk * es // 4
        # rows: A block rows and B search rows over all nodes and candidates
        rmin = off - cand - R
        rmax = (v["ny"] - 1) * step + off + blk - 1 + cand + R
        assert rmin + M >= 0 and rmax + M < v["rows"], (l, v)
        # columns in bytes; word loads start at the floor multiple of 4
        xmin = (off - cand - R) * es
        assert (xmin + M * es) - 3 >= 0, (l, v)
        if es == 1 and R <= 2 and NW in (2, 3, 4):
            # one node per lane: from the floor word of the leftmost shift,
            # RW + 1 words with RW = NW + (2R+3)//4 + 1
            start = ((v["nx"] - 1) * step + off + cand - R) * es
            span = 4 * (NW + (2 * R + 3) // 4 + 2)
        elif es == 2 and 1 <= R <= 2 and NW in (6, 8, 12):
            # u16, one node per lane with streamed A rows: from the floor word
            # of the leftmost shift, NW + ceil(2R es / 4) + 1 words
            start = ((v["nx"] - 1) * step + off + cand - R) * es
            span = 4 * (NW + (2 * R * es + 3) // 4 + 1)
        elif es == 2 and 2 * R + 1 <= 17:
            # u16, a lane per candidate row: from the floor word of the
            # leftmost shift, RWR + 1 words, RWR = NW + ceil((KMAX-1) es / 4)
            kmax = next(k for k in (5, 9, 13, 17) if k >= 2 * R + 1)
            start = ((v["nx"] - 1) * step + off + cand - R) * es
            span = 4 * (NW + ((kmax - 1) * es + 3) // 4 + 1)
        elif es == 1 and NW <= 4 and 2 * R + 1 <= 32:
            # a lane per candidate row (quad SAD): from the floor word of the
            # leftmost shift, RW + 1 words with RW = NW + ceil((2R+1)/4)
            start = ((v["nx"] - 1) * step + off + cand - R) * es
            span = 4 * (NW + (2 * R + 4) // 4 + 1)
        else:
            # the general kernel (a thread per candidate column and group of
            # candidate rows; without a parent, the band those threads read,
            # staged once): each from the floor word of its own shift, NW + 1 words
            start = ((v["nx"] - 1) * step + off + cand + R) * es
            span = 4 * (NW + 1)
        assert ((start + M * es) & ~3) + span <= v["pitch"], (l, v)
        # the A block itself (k_sad word_at reads 8 bytes from its floor word)
        assert ((((v["nx"] - 1) * step + off) * es + 4 * (NW - 1) + M * es) & ~3) + 8 <= v["pitch"]
        # pyramid: level l reads rows/cols up to 2*size - 1 of level l-1 (one into the margin)
        if l > 0:
            u = lv[l - 1]
            assert 2 * v["H"] - 1 < u["H"] + u["margin"] and 2 * v["W"] - 1 < u["W"] + u["margin"]
        assert v["pitch"] % 64 == 0 and M % 16 == 0


FRAME = 32   # px of the level-0 copy written along each edge when level 0 is read in place


@pytest.mark.parametrize("kw", [dict(), dict(width=200, height=136, levels=3, radius_coarse=5),
                                dict(width=204, height=138, win=12, step=6, levels=3, radius_coarse=5),
                                dict(width=256, height=192, levels=2, radius_coarse=4, radius_fine=1),
                                dict(width=384, height=216, dtype=2, bit_depth=12, win=24, step=12, levels=3),
                                dict(width=200, height=136, dtype=2, bit_depth=12, levels=3, radius_coarse=5)])
def test_level0_in_place_reads_stay_in_written_bytes(L, kw):
    """When level 0 is searched in place (u8 one node per lane or cell
    columns, u16 streamed), an A block or B span wholly inside the image
    reads the caller's frame and any other reads the padded copy, of which
    only FRAME px along the edges (plus the zero margins) are written.  For
    every node and every candidate centre the level can see, a padded read
    must touch only margin or frame bytes (columns in bytes below)."""
    import numpy as np
    lv = _levels(L, **kw)
    v = lv[0]
    es, step, blk, R, W, H = v["es"], v["step"], v["block"], v["R"], v["W"], v["H"]
    NW = blk * es // 4
    assert (es == 1 and R <= 2 and NW in (2, 3, 4)) or (es == 2 and 1 <= R <= 2 and NW in (6, 8, 12))
    maxd = 0
    for u in lv[:0:-1]:
        maxd = (0 if maxd == 0 and u is lv[-1] else 2 * maxd) + u["R"]
    cand = 2 * maxd if len(lv) > 1 else 0
    RW = NW + (2 * R + 3) // 4 + 1
    off = (step - blk) // 2
    aal = step % 4 == 0 and off % 4 == 0
    WB = W * es   # row bytes
    written_col = np.zeros(WB, bool)
    for q in range((WB + 15) // 16):
        if 16 * q < FRAME * es or 16 * q + 16 > (W - FRAME) * es:
            written_col[16 * q:16 * q + 16] = True
    written_row = np.zeros(H, bool)
    written_row[:FRAME] = True
    written_row[max(H - FRAME, 0):] = True

    def check(r0, nr, c0, nc):
        inside = r0 >= 0 and r0 + nr <= H and c0 >= 0 and c0 + nc <= WB
        if inside:
            return
        rows = np.arange(max(r0, 0), min(r0 + nr, H))
        cols = np.arange(max(c0, 0), min(c0 + nc, WB))
        if len(rows) and len(cols):
            ok = written_row[rows][:, None] | written_col[cols][None, :]
            assert ok.all(), (r0, nr, c0, nc)

    cs = range(-cand, cand + 1, 2)
    if es == 2 and step == 12 and blk == 24 and len(lv) > 1:
        # the u16 cell-shared form: 12x12 cells (24-byte A rows), B spans of
        # the cell plus 2R rows and CWD + R + 1 = 7 + R words
        for ci in range(v["ny"] + 1):
            y = ci * 12 - 6
            for cj in range(v["nx"] + 1):
                check(y, 12, (cj * 12 - 6) * 2, 24)
            for cy in cs:
                for cj in range(v["nx"] + 1):
                    x = cj * 12 - 6
                    for cx in (cs if cj in (0, 1, v["nx"] - 1, v["nx"]) else (-cand, 0, cand)):
                        xs = (x + cx - R) * 2
                        check(y + cy - R, 12 + 2 * R, xs & ~3, 4 * (7 + R))
        return
    if es == 2:
        # the streamed u16 kernel: A rows from the floor word of the block,
        # NW + 1 words; B rows from the floor word of the leftmost shift,
        # NW + ceil(2R es / 4) + 1 words
        rws = NW + (2 * R * es + 3) // 4
        for a in range(v["ny"]):
            oy = a * step + off
            for b in range(v["nx"]):
                check(oy, blk, ((b * step + off) * es) & ~3, 4 * (NW + 1))
            for cy in cs:
                for b in range(v["nx"]):
                    for cx in (cs if b in (0, 1, v["nx"] - 2, v["nx"] - 1) else (-cand, 0, cand)):
                        xs = (b * step + off + cx - R) * es
                        check(oy + cy - R, blk + 2 * R, xs & ~3, 4 * (rws + 1))
        return
    if step == 8 and blk == 16 and len(lv) > 1:
        # the cell-shared form: a column of three stacked 8x8 cells per lane
        # (24 A rows, 24 + 2R B rows) from cell row 2 pa
        rwc = 2 + (2 * R + 4) // 4
        for pa in range((v["ny"] + 1) // 2):
            y = 2 * pa * 8 - 4
            for cj in range(v["nx"] + 1):
                check(y, 24, cj * 8 - 4, 8)
            for cy in cs:
                for cj in range(v["nx"] + 1):
                    x = cj * 8 - 4
                    for cx in (cs if cj in (0, 1, v["nx"] - 1, v["nx"]) else (-cand, 0, cand)):
                        xs = x + cx - R
                        check(y + cy - R, 24 + 2 * R, xs & ~3, 4 * (rwc + 1))
    for a in range(v["ny"]):
        oy = a * step + off
        for b in range(v["nx"]):
            ox = b * step + off
            check(oy, blk, ox & ~3, 4 * (NW if aal else NW + 1))
        for cy in cs:
            y0 = oy + cy - R
            for b in range(v["nx"]):
                for cx in (cs if b in (0, 1, v["nx"] - 2, v["nx"] - 1) else (-cand, 0, cand)):
                    xs = b * step + off + cx - R
                    check(y0, blk + 2 * R, xs & ~3, 4 * (RW + 1))


def test_noalloc_rejects_before_any_device_call(L):
    """piv_run_noalloc checks its arguments and the size of its fixed scratch
    array on the host: work beyond the array, bad arguments and n = 0 return
    without touching a device (this runs without one)."""
    lib = L.lib()
    s, h = plan(L, width=2048, height=2048, max_batch=16)
    assert s == 0
    per = lib.piv_plan_workspace_bytes(h, 1)
    n = L.NOALLOC_SCRATCH_BYTES // per + 1
    assert n <= 16
    fake = C.c_void_p(1 << 20)
    assert lib.piv_run_noalloc(h, fake, fake, 2048, n, fake, fake, None, fake, fake, None) == L.PIV_ENOWORKSPACE
    assert b"scratch" in lib.piv_last_error()
    assert lib.piv_run_noalloc(h, fake, fake, 2048, 0, fake, fake, None, fake, fake, None) == 0
    assert lib.piv_run_noalloc(h, fake, fake, 2046, 1, fake, fake, None, fake, fake, None) == L.PIV_EINVAL
    assert lib.piv_run_noalloc(h, fake, fake, 2048, 1, None, fake, None, fake, fake, None) == L.PIV_EINVAL
    assert lib.piv_run_noalloc(None, fake, fake, 2048, 1, fake, fake, None, fake, fake, None) == L.PIV_EINVAL
    lib.piv_plan_destroy(h)


def test_preprocess_argument_errors(L):
    """Pre-processing rejects bad arguments on the host, before any launch."""
    lib = L.lib()
    s, h = plan(L, max_batch=2)
    assert s == 0
    fake, fake2 = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    assert lib.piv_highpass(h, fake, fake, 1024, 1, 7, None) == L.PIV_EINVAL          # in place
    assert lib.piv_highpass(h, fake, fake2, 1024, 1, 0, None) == L.PIV_EINVAL         # radius
    assert lib.piv_highpass(h, fake, fake2, 1024, 1, 17, None) == L.PIV_EINVAL
    assert lib.piv_highpass(h, fake, fake2, 1023, 1, 7, None) == L.PIV_EINVAL         # pitch
    assert lib.piv_highpass(h, fake, fake2, 1024, 3, 7, None) == L.PIV_EINVAL         # n > max_batch
    assert lib.piv_highpass(h, fake, fake2, 1024, 0, 7, None) == 0
    need = lib.piv_clahe_lut_bytes(h, 2, 8, 8)
    assert need == 2 * 64 * 256 * 2
    assert lib.piv_clahe(h, fake, fake, 1024, 2, 8, 8, 2.0, fake2, need - 1, None) == L.PIV_EINVAL
    assert lib.piv_clahe(h, fake, fake, 1024, 2, 0, 8, 2.0, fake2, need, None) == L.PIV_EINVAL
    assert lib.piv_clahe(h, fake, fake, 1024, 2, 65, 8, 2.0, fake2, 1 << 30, None) == L.PIV_EINVAL
    assert lib.piv_clahe(h, fake, fake, 1024, 2, 8, 8, 0.0, fake2, need, None) == L.PIV_EINVAL
    assert lib.piv_clahe(h, fake, fake, 1024, 2, 8, 8, 2.0, None, need, None) == L.PIV_EINVAL
    assert lib.piv_clahe(h, fake, fake, 1024, 0, 8, 8, 2.0, fake2, need, None) == 0
    lib.piv_plan_destroy(h)
    s, u = plan(L, dtype=2, bit_depth=12, win=24, step=12, width=3840, height=2160)
    assert s == 0 and lib.piv_clahe_lut_bytes(u, 1, 8, 8) == 64 * 4096 * 2
    lib.piv_plan_destroy(u)
    s, f = plan(L, dtype=3, levels=1, width=64, height=64)
    assert lib.piv_highpass(f, fake, fake2, 256, 1, 7, None) == L.PIV_EUNSUPPORTED
    lib.piv_plan_destroy(f)
