"""Parity at the benchmark's full size and launch configuration: one batch of
64 pairs of 1024 x 1024 u8 (eight distinct rendered pairs, each eight times,
exactly as bench.py runs them) through one piv_run.  Against the FP64 oracle:

* the predictor at every node of every distinct pair (bit-exact);
* the correction at sampled nodes (edges, corners and random interior nodes),
  called again with the same kernel and launch configuration on the run's own
  predictor: displacement within 0.01 px, coefficient within 2e-5, flags
  exact, unless the oracle's plane shows a near-tie; and at every node of two
  of the pairs;
* validation and vorticity on the whole grid, from the GPU's correction;
* all eight copies of a pair give bitwise identical results;
* the largest image the paper runs, 8192 x 4096, one pair, checked the same
  way;
* the 4K u16 stream form (3840 x 2160, 12-bit, 24/12 windows) as the bench
  runs it: a captured HIP graph over 8 slots, two distinct rendered pairs.
"""
import numpy as np
import pytest
import torch

import oracle
from _helpers import (MAX_TIES, NEAR_TIE_RHO, TOL_DISP_PX, TOL_REL, TOL_RHO, compare_correct, compare_validate,
                      corr_gap, record, say)
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

KW = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)
ND, NB, W, H = 8, 64, 1024, 1024


@pytest.fixture(scope="module")
def fullsize():
    from paper_2504_17987_amd import api
    say("[fullsize] rendering 8 distinct 1024x1024 pairs")
    pairs = [synth.cfg2_pair(2000 + i) for i in range(ND)]
    A = torch.empty((NB, H, W), dtype=torch.uint8, device="cuda")
    B = torch.empty_like(A)
    for k in range(NB):
        A[k].copy_(torch.from_numpy(pairs[k % ND][0]))
        B[k].copy_(torch.from_numpy(pairs[k % ND][1]))
    P = api.Plan(W, H, max_batch=NB, **KW)
    say("[fullsize] piv_run, batch 64")
    out = P.run(A, B)
    disp = torch.empty_like(out["disp"])
    peak = torch.empty_like(out["peak"])
    flags = torch.empty_like(out["flags"])
    say("[fullsize] piv_correct on the run's predictor")
    P.correct(A, B, out["pred"], disp, peak, flags)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    corr = dict(disp=disp.cpu().numpy(), peak=peak.cpu().numpy(), flags=flags.cpu().numpy())
    return pairs, host, corr


def test_fullsize_copies_identical(fullsize):
    _, g, c = fullsize
    for k in range(ND, NB):
        for name in ("pred", "disp", "peak", "flags", "omega"):
            assert np.array_equal(g[name][k], g[name][k % ND]), (name, k)
        for name in ("disp", "peak", "flags"):
            assert np.array_equal(c[name][k], c[name][k % ND]), (name, k)


def test_fullsize_predictor_bitexact(fullsize):
    pairs, g, _ = fullsize
    for i in range(ND):
        A, B, _ = pairs[i]
        po = oracle.predict(A, B, 8, 16, 3, 6, 2).astype(np.float64)
        po, _ = oracle.validate(po, None)
        say(f"  pair {i}: predictor range {po.min():.0f}..{po.max():.0f}")
        assert np.array_equal(g["pred"][i], po.astype(np.float32)), i


def _sample_nodes(rng, ny, nx, k):
    edge = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (0, nx // 2), (ny // 2, 0),
            (ny - 1, nx // 3), (ny // 3, nx - 1), (7, 8), (8, 7), (63, 64), (64, 63)]
    inner = [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, k), rng.integers(0, nx, k))]
    return edge + inner


def test_fullsize_correction_sampled(fullsize):
    pairs, g, c = fullsize
    rng = np.random.default_rng(2504)
    ny, nx = g["pred"].shape[2:]
    ties = 0
    worst = 0.0
    for i in range(ND):
        A, B, _ = pairs[i]
        Ad, Bd = A.astype(np.float64), B.astype(np.float64)
        pred = g["pred"][i].astype(np.float64)   # bit-exact with the oracle's (checked above)
        for a, b in _sample_nodes(rng, ny, nx, 48):
            du, dv, pk, fl = oracle.correct_node(Ad, Bd, 16, 8, 4, pred, a, b)
            d = max(abs(c["disp"][i, 0, a, b] - du), abs(c["disp"][i, 1, a, b] - dv))
            ok = d <= TOL_DISP_PX and abs(c["peak"][i, a, b] - pk) <= TOL_RHO and c["flags"][i, a, b] == fl
            if not ok:
                gap = corr_gap(Ad, Bd, 16, 8, 4, 0, pred, a, b)
                assert gap < NEAR_TIE_RHO, (i, a, b, c["disp"][i, :, a, b], (du, dv), gap)
                ties += 1
            else:
                worst = max(worst, d)
    say(f"  max |d disp| {worst:.2e} px, near-tie exemptions {ties}")
    record("fullsize sampled correction", "near-tie", ties)
    assert ties <= MAX_TIES


def test_fullsize_correction_full_grid(fullsize):
    """Every node of two of the distinct pairs (all 256 tiles of each, edges
    included) against the oracle's full correction on the run's predictor."""
    pairs, g, c = fullsize
    for i in (0, 5):
        A, B, _ = pairs[i]
        pred = g["pred"][i].astype(np.float64)
        disp_o, peak_o, flags_o = oracle.correct(A, B, 16, 8, 4, pred)
        ex = compare_correct(None, None, A.astype(np.float64), B.astype(np.float64), 16, 8, 4, pred,
                             c["disp"][i], c["peak"][i], c["flags"][i], disp_o, peak_o, flags_o,
                             where=f"fullsize full grid, pair {i}")
        d = np.abs(c["disp"][i] - disp_o)[:, ~ex].max()
        say(f"  pair {i}: max |d disp| {d:.2e} px over {pred.shape[1] * pred.shape[2]} nodes, "
            f"exempted {int(ex.sum())}")


def test_fullsize_validation_and_vorticity(fullsize):
    _, g, c = fullsize
    for i in range(ND):
        f = c["disp"][i].astype(np.float64)
        fl = c["flags"][i].copy()
        vo, flo = oracle.validate(f, fl)
        compare_validate(f, c["flags"][i], g["disp"][i], g["flags"][i], vo, flo,
                         where=f"fullsize validation, pair {i}")
        om = oracle.vorticity(g["disp"][i].astype(np.float64), 8)
        assert np.abs(g["omega"][i] - om).max() <= TOL_REL * np.abs(om).max(), i


def test_largest_image_8192x4096():
    """The largest image the paper runs (Sec. 4.1: 8192 x 4096, 33.6 MP), one
    pair through piv_run: predictor bit-exact on every node, correction at
    sampled nodes, validation and vorticity on the whole grid.  The frames
    tile one rendered 1 MP pair 8 x 4 times."""
    from paper_2504_17987_amd import api
    A1, B1, _ = synth.cfg2_pair(2600)
    A, B = np.tile(A1, (4, 8)), np.tile(B1, (4, 8))
    H, W = A.shape
    P = api.Plan(W, H, max_batch=1, **KW)
    say(f"[largest] {W}x{H}")
    out = P.run(torch.from_numpy(A[None]).cuda(), torch.from_numpy(B[None]).cuda())
    disp = torch.empty_like(out["disp"])
    peak = torch.empty_like(out["peak"])
    flags = torch.empty_like(out["flags"])
    P.correct(torch.from_numpy(A[None]).cuda(), torch.from_numpy(B[None]).cuda(), out["pred"], disp, peak, flags)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy()[0] for k, v in out.items()}
    c = dict(disp=disp.cpu().numpy()[0], peak=peak.cpu().numpy()[0], flags=flags.cpu().numpy()[0])
    po = oracle.predict(A, B, 8, 16, 3, 6, 2).astype(np.float64)
    po, _ = oracle.validate(po, None)
    assert np.array_equal(g["pred"], po.astype(np.float32))
    ny, nx = po.shape[1:]
    Ad, Bd = A.astype(np.float64), B.astype(np.float64)
    rng = np.random.default_rng(2601)
    ties = 0
    for a, b in _sample_nodes(rng, ny, nx, 40):
        du, dv, pk, fl = oracle.correct_node(Ad, Bd, 16, 8, 4, g["pred"].astype(np.float64), a, b)
        d = max(abs(c["disp"][0, a, b] - du), abs(c["disp"][1, a, b] - dv))
        if not (d <= TOL_DISP_PX and abs(c["peak"][a, b] - pk) <= TOL_RHO and c["flags"][a, b] == fl):
            assert corr_gap(Ad, Bd, 16, 8, 4, 0, g["pred"].astype(np.float64), a, b) < NEAR_TIE_RHO, (a, b)
            ties += 1
    record("largest sampled correction", "near-tie", ties)
    assert ties <= MAX_TIES
    vo, flo = oracle.validate(c["disp"].astype(np.float64), c["flags"].copy())
    compare_validate(c["disp"].astype(np.float64), c["flags"], g["disp"], g["flags"], vo, flo,
                     where="largest validation")
    om = oracle.vorticity(g["disp"].astype(np.float64), 8)
    assert np.abs(g["omega"] - om).max() <= TOL_REL * np.abs(om).max()


def test_cfg3_4k_u16_graph_slots():
    """The 4K u16 stream configuration through the bench's graph runner
    (8 slots, one replay): predictor bit-exact on every node, correction on
    sampled nodes (re-run eagerly on the replay's predictor), validation and
    vorticity on the whole grid, and slots holding the same pair identical."""
    from paper_2504_17987_amd import api
    from paper_2504_17987_amd.serve import GraphRunner
    kw3 = dict(dtype="u16", win=24, step=12, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    say("[cfg3] rendering 2 distinct 3840x2160 u16 pairs")
    prs = [synth.cfg3_pair(k)[:2] for k in (0, 1)]
    run = GraphRunner(api.Plan(3840, 2160, max_batch=8, **kw3), 8)
    run.capture()
    for i in range(8):
        run.A[i].copy_(torch.from_numpy(prs[i % 2][0].view(np.int16)).view(torch.uint16))
        run.B[i].copy_(torch.from_numpy(prs[i % 2][1].view(np.int16)).view(torch.uint16))
    say("[cfg3] graph replay, 8 slots")
    run.replay(8)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in run.out.items()}
    for k in range(2, 8):
        for name in ("pred", "disp", "flags", "omega"):
            assert np.array_equal(g[name][k], g[name][k % 2]), (name, k)
    P = run.plan
    for i in range(2):
        A, B = prs[i]
        po = oracle.predict(A, B, 12, 24, 3, 6, 2).astype(np.float64)
        po, _ = oracle.validate(po, None)
        assert np.array_equal(g["pred"][i], po.astype(np.float32)), i
        disp, peak, flags = P.correct(run.A[i:i + 1], run.B[i:i + 1], run.out["pred"][i:i + 1])
        c = dict(disp=disp.cpu().numpy()[0], peak=peak.cpu().numpy()[0], flags=flags.cpu().numpy()[0])
        Ad, Bd = A.astype(np.float64), B.astype(np.float64)
        ny, nx = po.shape[1:]
        rng = np.random.default_rng(3000 + i)
        ties = 0
        for a, b in _sample_nodes(rng, ny, nx, 40):
            du, dv, pk, fl = oracle.correct_node(Ad, Bd, 24, 12, 4, po, a, b)
            d = max(abs(c["disp"][0, a, b] - du), abs(c["disp"][1, a, b] - dv))
            if not (d <= TOL_DISP_PX and abs(c["peak"][a, b] - pk) <= TOL_RHO and c["flags"][a, b] == fl):
                assert corr_gap(Ad, Bd, 24, 12, 4, 0, po, a, b) < NEAR_TIE_RHO, (i, a, b)
                ties += 1
        record(f"cfg3 sampled correction, pair {i}", "near-tie", ties)
        assert ties <= MAX_TIES
        vo, flo = oracle.validate(c["disp"].astype(np.float64), c["flags"].copy())
        compare_validate(c["disp"].astype(np.float64), c["flags"], g["disp"][i], g["flags"][i], vo, flo,
                         where=f"cfg3 validation, pair {i}")
        om = oracle.vorticity(g["disp"][i].astype(np.float64), 12)
        assert np.abs(g["omega"][i] - om).max() <= TOL_REL * np.abs(om).max()
        say(f"  pair {i}: predictor bit-exact, {ny * nx} vectors, near-ties {ties}")
