"""Batched HIP-graph launches and the continuous-batching server on the GPU:
graph replays equal eager runs (several replays, eager work in between,
partial batches through the slot mask), and every served result equals the
same pair run alone."""
import time

import numpy as np
import pytest
import torch

from _helpers import say
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def pairs_u8(W, H, n, seed, flow=None):
    A, B = [], []
    for k in range(n):
        f = flow or synth.SolidBody((W - 1) / 2, (H - 1) / 2, 6.0 / max(W, H))
        a, b = synth.make_pair(W, H, f, 0.03, noise=2.0, seed=seed + k)
        A.append(a)
        B.append(b)
    return dev(np.stack(A)), dev(np.stack(B))


def test_graph_replay_equals_eager_and_partial_batches():
    from paper_2504_17987_amd import api
    from paper_2504_17987_amd.serve import GraphRunner
    say("[graph] replay vs eager")
    A, B = pairs_u8(256, 256, 12, 100)
    ref = api.Plan(256, 256, max_batch=12)
    eager = ref.run(A, B)
    run = GraphRunner(api.Plan(256, 256, max_batch=8), 8)
    run.capture()
    for rep, (lo, n) in enumerate([(0, 8), (4, 8), (8, 4), (0, 8)]):
        run.A[:n].copy_(A[lo:lo + n])
        run.B[:n].copy_(B[lo:lo + n])
        for k in run.out:
            run.out[k].fill_(0)
        run.replay(n)
        run.stream.synchronize()
        # eager work between replays on the default stream
        ref.run(A, B)
        torch.cuda.synchronize()
        for k in ("pred", "disp", "flags", "omega", "peak"):
            assert torch.equal(run.out[k][:n], eager[k][lo:lo + n]), (rep, k)
            if n < 8:
                assert (run.out[k][n:] == 0).all(), (rep, k, "inactive slots must be untouched")


def test_u16_stream_through_graph():
    """Config-3 style: u16 12-bit pairs, 24/12 windows, 8 slots per replay,
    20 pairs -> replays of 8, 8 and 4 (shrunk image for the test)."""
    from paper_2504_17987_amd import api
    from paper_2504_17987_amd.serve import GraphRunner
    say("[graph] u16 stream")
    W, H = 768, 432
    A, B = [], []
    for k in range(5):
        a, b, _ = synth.cfg3_pair(k, W=W, H=H)
        A.append(a.view(np.int16))
        B.append(b.view(np.int16))
    A = dev(np.stack(A)).view(torch.uint16)
    B = dev(np.stack(B)).view(torch.uint16)
    kw = dict(dtype="u16", win=24, step=12, radius=4, levels=3, radius_coarse=6, radius_fine=2)
    ref = api.Plan(W, H, max_batch=1, **kw)
    run = GraphRunner(api.Plan(W, H, max_batch=8, **kw), 8)
    run.capture()
    idx = [k % 5 for k in range(20)]
    for lo in range(0, 20, 8):
        n = min(8, 20 - lo)
        for i in range(n):
            run.A[i].copy_(A[idx[lo + i]])
            run.B[i].copy_(B[idx[lo + i]])
        run.replay(n)
        run.stream.synchronize()
        for i in range(n):
            e = ref.run(A[idx[lo + i]:idx[lo + i] + 1], B[idx[lo + i]:idx[lo + i] + 1])
            torch.cuda.synchronize()
            assert torch.equal(run.out["disp"][i], e["disp"][0]) and torch.equal(run.out["flags"][i], e["flags"][0])


@pytest.mark.parametrize("eager_single", [True, False])
def test_served_results_equal_pair_alone(eager_single):
    """Every served result equals the pair run alone, bitwise; with lone
    requests run eagerly from their own buffers, and with every batch going
    through slot copies and a graph replay."""
    from paper_2504_17987_amd import api
    from paper_2504_17987_amd.serve import latency_stats, make_gpu_server, poisson_trace, serve_trace
    say(f"[serve] invariance, eager single {eager_single}")
    sizes = {"s": (128, 128, 8), "m": (256, 256, 4), "l": (512, 512, 2)}
    stream_class = {s: "sml"[s % 3] for s in range(6)}
    pairs = {}
    for s, c in stream_class.items():
        W, H, _ = sizes[c]
        pairs[s] = pairs_u8(W, H, 4, 1000 + 10 * s)
    sched, ex = make_gpu_server(sizes, pairs, stream_class, budget=8 << 30, keep_results=True,
                                eager_single=eager_single)
    trace = poisson_trace(list(stream_class.items()), 400.0, 0.25, 4, seed=7)
    serve_trace(sched, trace, time.perf_counter, poll=0, deadline=60.0)
    torch.cuda.synchronize()
    assert len(sched.finished) == len(trace)
    st = latency_stats(trace)
    say(f"  {st['n']} requests, p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms, batches {sched.batches}")
    plans = {c: api.Plan(W, H) for c, (W, H, _) in sizes.items()}
    worst = 0.0
    for r in trace:
        a, b = pairs[r.stream]
        e = plans[r.cls].run(a[r.item:r.item + 1], b[r.item:r.item + 1])
        got = ex.results[r.rid]
        d = (got["disp"] - e["disp"][0]).abs().max().item()
        worst = max(worst, d)
        assert d <= 0.01
        assert torch.equal(got["flags"], e["flags"][0])
    say(f"  max |served - alone| = {worst:.3e} px")
    assert worst == 0.0   # no cross-pair arithmetic: bit-identical


def test_admission_budget_refuses_a_class():
    """An HBM budget that holds class s (its runners and streams) but not
    class l: the l stream waits unadmitted, its requests are refused and
    counted apart, no runner of l is built, and every served s result still
    equals the pair run alone."""
    from paper_2504_17987_amd import api
    from paper_2504_17987_amd.serve import latency_stats, make_gpu_server, poisson_trace, serve_trace
    say("[serve] admission refusal")
    sizes = {"s": (128, 128, 4), "l": (512, 512, 2)}
    stream_class = {0: "s", 1: "s", 2: "l"}
    pairs = {s: pairs_u8(*sizes[c][:2], 2, 2000 + 10 * s) for s, c in stream_class.items()}
    probe_sched, probe_ex = make_gpu_server({"s": sizes["s"]}, {0: pairs[0], 1: pairs[1]}, {0: "s", 1: "s"},
                                            budget=0)
    assert not probe_sched.admitted and not probe_ex.runners   # nothing admitted at budget 0
    spec = probe_sched.classes["s"]
    need_s = 2 * spec.stream_bytes + probe_sched.inflight * spec.slot_bytes   # two s streams and their runners
    sched, ex = make_gpu_server(sizes, pairs, stream_class, budget=need_s, keep_results=True)
    assert set(sched.admitted) == {0, 1} and 2 not in sched.admitted and "l" not in ex.runners
    trace = poisson_trace(list(stream_class.items()), 300.0, 0.1, 2, seed=11)
    refused = serve_trace(sched, trace, time.perf_counter, poll=0, deadline=60.0)
    torch.cuda.synchronize()
    assert refused and all(r.stream == 2 for r in refused)
    st = latency_stats(trace)
    say(f"  served {st['n']}, refused {st['refused']}, p99 {st['p99_ms']:.3f} ms")
    assert st["refused"] == len(refused) and st["n"] == len(trace) - len(refused)
    P = api.Plan(128, 128)
    for r in trace:
        if r.stream == 2:
            continue
        a, b = pairs[r.stream]
        e = P.run(a[r.item:r.item + 1], b[r.item:r.item + 1])
        assert torch.equal(ex.results[r.rid]["disp"], e["disp"][0])
