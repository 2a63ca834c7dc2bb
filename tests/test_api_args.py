"""The Python binding checks every tensor it hands to the C ABI (dtype,
shape, batch, contiguity, then device) and raises before any call, so a
wrong tensor can never make a kernel read or write out of bounds.  Runs on
the CPU: plans are created without workspace (host-only), and the tensors
are CPU tensors, which pass the shape checks and fail only the final device
check."""
import os

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def api():
    from paper_2504_17987_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2504_17987_amd import build
        build.build(verbose=False)
    from paper_2504_17987_amd import api as A
    return A


@pytest.fixture
def P(api):
    return api.Plan(64, 48, max_batch=2, win=16, step=8, workspace=False)   # grid 8 x 6


@pytest.fixture
def F(api):
    return api.Plan(64, 48, max_batch=2, dtype="f32", levels=1, workspace=False)


def imgs(n=2, dtype=torch.uint8, H=48, W=64):
    return torch.zeros((n, H, W), dtype=dtype), torch.zeros((n, H, W), dtype=dtype)


def outs(n=2, ny=6, nx=8):
    return dict(pred=torch.zeros((n, 2, ny, nx)), disp=torch.zeros((n, 2, ny, nx)), peak=torch.zeros((n, ny, nx)),
                flags=torch.zeros((n, ny, nx), dtype=torch.uint8), omega=torch.zeros((n, ny, nx)))


def test_good_shapes_fail_only_on_device(P):
    A, B = imgs()
    with pytest.raises(TypeError, match="device"):
        P.run(A, B, outs())


@pytest.mark.parametrize("key,bad,exc", [
    ("disp", torch.zeros((2, 2, 6, 7)), ValueError),                    # wrong grid
    ("disp", torch.zeros((1, 2, 6, 8)), ValueError),                    # too few pairs
    ("pred", torch.zeros((2, 2, 6, 8), dtype=torch.float64), TypeError),
    ("flags", torch.zeros((2, 6, 8)), TypeError),                       # float flags
    ("omega", torch.zeros((2, 8, 6)), ValueError),                      # transposed
    ("peak", torch.zeros((2, 6, 16))[:, :, ::2], ValueError),           # not contiguous
    ("omega", None, ValueError),                                       # missing
])
def test_run_rejects_bad_outputs(P, key, bad, exc):
    A, B = imgs()
    o = outs()
    o[key] = bad
    with pytest.raises(exc):
        P.run(A, B, o)


def test_images_checked(P):
    A, B = imgs()
    with pytest.raises(TypeError):
        P.run(A.float(), B.float(), outs())
    with pytest.raises(ValueError):
        P.run(*imgs(H=40), outs())
    with pytest.raises(ValueError, match="max_batch"):
        P.run(*imgs(n=3), outs(n=3))


def test_correct_validate_vorticity_checked(P):
    A, B = imgs()
    with pytest.raises(ValueError):
        P.correct(A, B, pred=torch.zeros((2, 2, 5, 8)), disp=torch.zeros((2, 2, 6, 8)),
                  peak=torch.zeros((2, 6, 8)), flags=torch.zeros((2, 6, 8), dtype=torch.uint8))
    with pytest.raises(ValueError):
        P.validate(torch.zeros((2, 2, 6, 8)), torch.zeros((1, 6, 8), dtype=torch.uint8))
    with pytest.raises(ValueError):
        P.vorticity(torch.zeros((2, 2, 6, 8)), torch.zeros((2, 6, 9)))
    with pytest.raises(TypeError, match="device"):
        P.vorticity(torch.zeros((2, 2, 6, 8)), torch.zeros((2, 6, 8)))


def test_temporal_arguments_checked(P):
    A, B = imgs()
    st = torch.zeros((3, 2, 6, 8))
    with pytest.raises(TypeError):                                   # int64 slots
        P.run_temporal(A, B, torch.zeros(2, dtype=torch.int64), st, st, out=outs())
    with pytest.raises(ValueError):                                  # too few slots
        P.run_temporal(A, B, torch.zeros(1, dtype=torch.int32), st, st, out=outs())
    with pytest.raises(ValueError):                                  # state grid
        P.run_temporal(A, B, torch.zeros(2, dtype=torch.int32), torch.zeros((3, 2, 5, 8)), None, out=outs())
    with pytest.raises(ValueError):                                  # different stream counts
        P.run_temporal(A, B, torch.zeros(2, dtype=torch.int32), st, torch.zeros((2, 2, 6, 8)), out=outs())
    with pytest.raises(ValueError):
        P.smooth(torch.zeros((2, 2, 6, 8)), None, torch.zeros(2, dtype=torch.int32))
    with pytest.raises(TypeError, match="device"):
        P.smooth(torch.zeros((2, 2, 6, 8)), st, torch.zeros(2, dtype=torch.int32))


def test_ssd_arguments_checked(F):
    A = torch.zeros((2, 48, 64))
    U = torch.zeros((2, 2, 6, 8))
    with pytest.raises(ValueError):                                  # U grid of another plan
        F.ssd_forward(A, A, torch.zeros((2, 2, 12, 16)), torch.zeros((2, 6, 8)))
    with pytest.raises(ValueError):                                  # B holds fewer pairs
        F.ssd_forward(A, A[:1], U, torch.zeros((2, 6, 8)))
    with pytest.raises(ValueError):
        F.ssd_backward(A, A, U, torch.zeros((2, 6, 7)), torch.zeros((2, 2, 6, 8)), torch.zeros((2, 2, 6, 8)))
    with pytest.raises(TypeError):
        F.ssd_backward(A, A, U, torch.zeros((2, 6, 8)), torch.zeros((2, 2, 6, 8), dtype=torch.float16), None,
                       want_diag=False)
    with pytest.raises(ValueError):                                  # history length
        F.ssd_refine(A, A, U, steps=4, hist=torch.zeros((2, 4)))
    with pytest.raises(TypeError, match="device"):
        F.ssd_refine(A, A, U, steps=4, hist=torch.zeros((2, 5)))
    with pytest.raises(ValueError):                                  # non-contiguous
        F.ssd_forward(A, A, torch.zeros((2, 2, 8, 6)).transpose(2, 3), torch.zeros((2, 6, 8)))
