"""Exponential smoothing in time (the paper's alpha1 on the validated
predictor and alpha2 on the validated final field, Sec. 2) on the GPU:
the smoothing kernel against the FP64 oracle; piv_run_temporal against the
same steps called one by one, and against the oracle's pipeline over a
stream of frames with every difference explained; and the server's
per-stream smoothing against each stream run alone in order."""
import time

import numpy as np
import pytest
import torch

import oracle
from _helpers import (TOL_REL, compare_correct, compare_validate, dilate, record, say)
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

KW = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)


def api():
    from paper_2504_17987_amd import api as A
    return A


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def stream_frames(n, W=256, H=192, seed=300):
    """A vortex advected 0.5 px per frame in x (a stream of pairs)."""
    frames = []
    for t in range(n):
        flow = synth.LambOseen.with_peak(100.0 + 0.5 * t, 95.5, 50.0, 6.0)
        A, B = synth.make_pair(W, H, flow, 0.04, noise=2.0, dropout=0.05, seed=seed + t)
        frames.append((A, B))
    return frames


def test_smooth_kernel_parity():
    say("[temporal] smoothing kernel")
    rng = np.random.default_rng(90)
    P = api().Plan(80, 64, max_batch=6, win=16, step=8)
    n, nst = 6, 3
    f = rng.normal(0, 4, (n, 2, P.ny, P.nx)).astype(np.float32)
    st = rng.normal(0, 4, (nst, 2, P.ny, P.nx)).astype(np.float32)
    slots = np.array([-1 - 2, 0, 2, 2, 9, -1 - 0], np.int32)   # start, continue, chain, out of range, restart
    for alpha in (0.5, 0.3, 1.0):
        fg, sg = dev(f), dev(st)
        P.smooth(fg, sg, dev(slots), alpha)
        fo, so = oracle.smooth_batch(f.astype(np.float64), st.astype(np.float64), slots, alpha)
        ef = np.abs(fg.cpu().numpy() - fo).max()
        es = np.abs(sg.cpu().numpy() - so).max()
        say(f"  alpha {alpha}: max |gpu - oracle| field {ef:.2e}, state {es:.2e}")
        assert ef <= 1e-6 * np.abs(fo).max() and es <= 1e-6 * np.abs(so).max()
        assert np.array_equal(fg.cpu().numpy()[4], f[4])            # slot out of range: untouched
    # alpha = 0.5 on integers is exact in FP32
    fi = rng.integers(-20, 21, (n, 2, P.ny, P.nx)).astype(np.float32)
    si = rng.integers(-20, 21, (nst, 2, P.ny, P.nx)).astype(np.float32)
    fg, sg = dev(fi), dev(si)
    P.smooth(fg, sg, dev(slots), 0.5)
    fo, so = oracle.smooth_batch(fi.astype(np.float64), si.astype(np.float64), slots, 0.5)
    assert np.array_equal(fg.cpu().numpy(), fo.astype(np.float32))


def test_run_temporal_equals_separate_steps():
    """piv_run_temporal gives the same bits as predict, validate, smooth,
    correct, validate, smooth, vorticity called one by one; with both states
    absent it gives piv_run's bits."""
    say("[temporal] run_temporal vs separate steps")
    frames = stream_frames(4)
    A = dev(np.stack([a for a, _ in frames]))
    B = dev(np.stack([b for _, b in frames]))
    P = api().Plan(256, 192, max_batch=4, **KW)
    slot = dev(np.array([-1, 0, 0, 0], np.int32))   # one stream: frame 0 starts it, the rest chain
    sp, sd = P.new_state(1), P.new_state(1)
    out = P.run_temporal(A, B, slot, sp, sd, 0.5, 0.5)
    sp2, sd2 = P.new_state(1), P.new_state(1)
    pred = P.predict(A, B)
    P.validate(pred, None)
    P.smooth(pred, sp2, slot, 0.5)
    disp, peak, flags = P.correct(A, B, pred)
    P.validate(disp, flags)
    P.smooth(disp, sd2, slot, 0.5)
    omega = P.vorticity(disp)
    for k, v in (("pred", pred), ("disp", disp), ("peak", peak), ("flags", flags), ("omega", omega)):
        assert torch.equal(out[k], v), k
    assert torch.equal(sp, sp2) and torch.equal(sd, sd2)
    plain = P.run(A, B)
    none = P.run_temporal(A, B, slot, None, None)
    for k in plain:
        assert torch.equal(plain[k], none[k]), k


def test_run_temporal_stream_vs_oracle():
    """A stream of 6 frames in two batches of 3 (the state carries across
    batches) against the oracle's pipeline with smoothing, stage by stage:
    the smoothed predictor bit-exact every frame (integer predictors and
    alpha = 1/2 are exact in FP32); the raw correction on it and its
    validation with explained exemptions; the smoothed final field within
    0.01 px except at nodes where an exemption at this or an earlier frame
    lies in the 3x3 neighbourhood (the state carries a node's history)."""
    say("[temporal] stream of 6 frames vs oracle")
    frames = stream_frames(6, seed=310)
    P = api().Plan(256, 192, max_batch=3, **KW)
    sp, sd = P.new_state(1), P.new_state(1)
    outs = []
    for lo in (0, 3):
        A = dev(np.stack([a for a, _ in frames[lo:lo + 3]]))
        B = dev(np.stack([b for _, b in frames[lo:lo + 3]]))
        slot = dev(np.array([-1 if lo == 0 else 0, 0, 0], np.int32))
        out = P.run_temporal(A, B, slot, sp, sd, 0.5, 0.5)
        raw, peak, flags = P.correct(A, B, out["pred"])
        val = raw.clone()
        vfl = flags.clone()
        P.validate(val, vfl)
        torch.cuda.synchronize()
        for i in range(3):
            outs.append({k: v[i].cpu().numpy() for k, v in dict(out, raw=raw, rpeak=peak, rflags=flags,
                                                                 val=val, vflags=vfl).items()})
    ref = oracle.run_temporal(frames, win=16, step=8, r=4, levels=3, Rc=6, Rf=2, alpha1=0.5, alpha2=0.5)
    allowed = np.zeros((P.ny, P.nx), bool)
    worst = 0.0
    for t, (g, o) in enumerate(zip(outs, ref)):
        A, B = frames[t]
        assert np.array_equal(g["pred"], o["pred"].astype(np.float32)), f"frame {t}: smoothed predictor"
        raw_ex = compare_correct(None, None, A.astype(float), B.astype(float), 16, 8, 4, o["pred"], g["raw"],
                                 g["rpeak"], g["rflags"], o["disp_raw"], o["peak"], o["flags_raw"],
                                 where=f"temporal frame {t} raw")
        vo, flo = oracle.validate(g["raw"].astype(np.float64), g["rflags"].copy())
        uod_ex = compare_validate(g["raw"].astype(np.float64), g["rflags"], g["val"], g["vflags"], vo, flo,
                                  where=f"temporal frame {t} validate")
        allowed |= dilate(raw_ex) | dilate(uod_ex)
        d = np.abs(g["disp"] - o["disp"]).max(axis=0)
        bad = d > 0.01
        assert not (bad & ~allowed).any(), f"frame {t}: {int((bad & ~allowed).sum())} unexplained"
        record(f"temporal frame {t}", "propagated", int(bad.sum()))
        worst = max(worst, float(d[~allowed].max()))
        om = oracle.vorticity(g["disp"].astype(np.float64), 8)
        assert np.abs(g["omega"] - om).max() <= TOL_REL * np.abs(om).max()
    say(f"  max |gpu - oracle| over 6 frames: {worst:.2e} px")


def test_served_stream_smoothing_equals_stream_alone():
    """The server with temporal smoothing: every stream's results equal that
    stream's frames run alone, in order, through piv_run_temporal with its
    own state (bitwise), although requests of several streams share
    batches."""
    from paper_2504_17987_amd.serve import make_gpu_server, poisson_trace, serve_trace
    say("[temporal] served smoothing")
    sizes = {"s": (128, 128, 4), "m": (256, 192, 2)}
    stream_class = {0: "s", 1: "s", 2: "s", 3: "m", 4: "m"}
    pairs = {}
    for s, c in stream_class.items():
        W, H, _ = sizes[c]
        fr = [synth.make_pair(W, H, synth.SolidBody((W - 1) / 2, (H - 1) / 2, (3 + s) / W), 0.04, noise=2.0,
                              seed=400 + 10 * s + k) for k in range(4)]
        pairs[s] = (dev(np.stack([a for a, _ in fr])), dev(np.stack([b for _, b in fr])))
    sched, ex = make_gpu_server(sizes, pairs, stream_class, budget=8 << 30, keep_results=True,
                                temporal=dict(alpha1=0.5, alpha2=0.5))
    trace = poisson_trace(list(stream_class.items()), 300.0, 0.05, 4, seed=9)
    # every stream's requests in order: item k is frame k (cycled)
    serve_trace(sched, trace, time.perf_counter, poll=0, deadline=60.0)
    torch.cuda.synchronize()
    assert len(sched.finished) == len(trace)
    plans = {c: api().Plan(W, H, **KW) for c, (W, H, _) in sizes.items()}
    states = {s: (plans[c].new_state(1), plans[c].new_state(1)) for s, c in stream_class.items()}
    seen = set()
    for r in trace:
        a, b = pairs[r.stream]
        P = plans[r.cls]
        slot = torch.tensor([0 if r.stream in seen else -1], dtype=torch.int32, device="cuda")
        seen.add(r.stream)
        e = P.run_temporal(a[r.item:r.item + 1], b[r.item:r.item + 1], slot, *states[r.stream])
        got = ex.results[r.rid]
        for k in ("pred", "disp", "flags", "omega"):
            assert torch.equal(got[k], e[k][0]), (r.rid, r.stream, k)
    say(f"  {len(trace)} requests in {sched.batches} batches, all equal to their streams run alone")
