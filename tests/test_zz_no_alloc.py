"""piv_run_noalloc (the entry point that allocates nothing: its workspace is
the library's fixed per-GPU device array) gives the same bits as piv_run on
a plan with its own workspace, on two calls in a row, the second with a
smaller input (another geometry, fewer pairs), and rejects work that does
not fit the array before any device call."""
import numpy as np
import pytest
import torch

from _helpers import say
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

KW = dict(win=16, step=8, radius=4, levels=3, radius_coarse=6, radius_fine=2)


def batch(W, H, n, seed):
    A, B = [], []
    for k in range(n):
        flow = synth.LambOseen.with_peak((W - 1) / 2, (H - 1) / 2, 50.0, 7.0)
        a, b = synth.make_pair(W, H, flow, 0.04, noise=2.0, dropout=0.1, seed=seed + k)
        A.append(a)
        B.append(b)
    return torch.from_numpy(np.stack(A)).cuda(), torch.from_numpy(np.stack(B)).cuda()


def outputs(P, n):
    return dict(pred=torch.full((n, 2, P.ny, P.nx), 7.0, device="cuda"),
                disp=torch.full((n, 2, P.ny, P.nx), 7.0, device="cuda"),
                peak=torch.full((n, P.ny, P.nx), 7.0, device="cuda"),
                flags=torch.full((n, P.ny, P.nx), 7, dtype=torch.uint8, device="cuda"),
                omega=torch.full((n, P.ny, P.nx), 7.0, device="cuda"))


def test_noalloc_equals_run_on_two_calls():
    from paper_2504_17987_amd import api
    for (W, H, n, seed) in [(512, 384, 3, 700), (256, 192, 2, 710)]:
        say(f"[noalloc] {W}x{H}, {n} pairs")
        A, B = batch(W, H, n, seed)
        ref = api.Plan(W, H, max_batch=n, **KW).run(A, B)
        P = api.Plan(W, H, max_batch=n, workspace=False, **KW)
        assert P.workspace_bytes(n) <= 64 << 20
        out = P.run_noalloc(A, B, outputs(P, n))
        torch.cuda.synchronize()
        for k in ("pred", "disp", "peak", "flags", "omega"):
            assert torch.equal(out[k], ref[k]), (W, H, k)


def test_noalloc_rejects_work_beyond_the_array():
    from paper_2504_17987_amd import _lib, api
    P = api.Plan(2048, 2048, max_batch=8, workspace=False, **KW)
    n = 1
    while P.workspace_bytes(n) <= _lib.NOALLOC_SCRATCH_BYTES:
        n += 1
    assert n <= 8
    A = torch.zeros((n, 2048, 2048), dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.PivError, match="ENOWORKSPACE"):
        P.run_noalloc(A, A, outputs(P, n))
