"""Pre-processing on the GPU (high-pass background removal and CLAHE, the
paper's Sec. 2 pre-processing) against the integer oracle: bit-exact, on u8
and u16 frames (12 and 16 bits), ragged sizes and tile grids, several
radii, batches, in place (CLAHE), and on full-size 1 MP frames."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import say
from paper_2504_17987_amd import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def api():
    from paper_2504_17987_amd import api as A
    return A


def dev(x, dtype, pad=0):
    """Device frames [n][H][W] whose rows are padded by `pad` elements (the
    padding holds the largest value, so a read past a row would show)."""
    n, H, W = x.shape
    full = np.full((n, H, W + pad), np.iinfo(x.dtype).max, dtype=x.dtype)
    full[:, :, :W] = x
    t = torch.from_numpy(full.view(np.int16 if dtype == "u16" else np.uint8)).cuda()
    t = t.view(torch.uint16) if dtype == "u16" else t
    return t[:, :, :W]


def host(t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def out_like(t, pad):
    n, H, W = t.shape
    o = torch.zeros((n, H, W + pad), dtype=t.dtype, device=t.device)
    return o[:, :, :W]


def plan_for(W, H, n, dtype, bits):
    """A plan of the frames' size and dtype (pre-processing uses no vector
    grid; any step the library accepts will do)."""
    from paper_2504_17987_amd import _lib
    for s in (8, 6, 4, 2, 10, 12, 14):
        if W % s or H % s:
            continue
        try:
            return api().Plan(W, H, max_batch=n, dtype=dtype, bit_depth=bits if dtype == "u16" else None,
                              levels=1, win=2 * s, step=s, radius=1, workspace=False, block=2 * s)
        except _lib.PivError:
            continue
    raise AssertionError(f"no plan for {W}x{H} {dtype}")


def frames(W, H, n, dtype, bits, seed):
    """Particle images on a sloping, uneven background (what the high-pass
    removes)."""
    out = []
    ys, xs = np.mgrid[0:H, 0:W]
    for k in range(n):
        if dtype == "u8":
            a, _ = synth.make_pair(W, H, synth.Uniform(1.0, 0.5), 0.04, noise=2.0, seed=seed + k)
            bg = (30 + 20 * np.sin(xs / 37.0) + 0.05 * ys).astype(np.int64)
            out.append(np.clip(a.astype(np.int64) + bg, 0, 255).astype(np.uint8))
        else:
            a, _, _ = synth.cfg3_pair(k, seed=seed, W=W, H=H)
            m = (1 << bits) - 1
            bg = (300 + 200 * np.sin(xs / 41.0)).astype(np.int64)
            v = a.astype(np.int64) * (m // 4095) + bg
            out.append(np.clip(v, 0, m).astype(np.uint16))
    return np.stack(out)


# (dtype, bits, W, H, n, row padding in elements): ragged tiles and rows
# (198 px u8 rows end inside a 4-pixel group)
CASES = [("u8", 8, 256, 192, 3, 0), ("u8", 8, 198, 138, 2, 6), ("u16", 12, 384, 216, 2, 2),
         ("u16", 16, 250, 130, 2, 4)]


@pytest.mark.parametrize("dtype,bits,W,H,n,pad", CASES)
@pytest.mark.parametrize("radius", [1, 7, 16])
def test_highpass_bitexact(dtype, bits, W, H, n, pad, radius):
    say(f"[highpass] {dtype}/{bits} {W}x{H} r={radius}")
    I = frames(W, H, n, dtype, bits, 800)
    P = plan_for(W, H, n, dtype, bits)
    Id = dev(I, dtype, pad)
    out = host(P.highpass(Id, out_like(Id, pad), radius=radius))
    for i in range(n):
        ref = oracle.highpass(I[i], radius)
        assert np.array_equal(out[i].astype(np.int64), ref), i


@pytest.mark.parametrize("dtype,bits,W,H,n,pad", CASES)
@pytest.mark.parametrize("tiles,clip", [((8, 8), 2.0), ((5, 3), 1.3), ((1, 1), 1e9), ((16, 9), 4.0)])
def test_clahe_bitexact(dtype, bits, W, H, n, pad, tiles, clip):
    say(f"[clahe] {dtype}/{bits} {W}x{H} tiles {tiles} clip {clip}")
    I = frames(W, H, n, dtype, bits, 820)
    P = plan_for(W, H, n, dtype, bits)
    Id = dev(I, dtype, pad)
    out = host(P.clahe(Id, out_like(Id, pad), tiles=tiles, clip_factor=clip))
    for i in range(n):
        ref = oracle.clahe(I[i], bits, tiles[0], tiles[1], clip)
        assert np.array_equal(out[i].astype(np.int64), ref), i
    # in place gives the same
    P.clahe(Id, Id, tiles=tiles, clip_factor=clip)
    assert np.array_equal(host(Id), out)


def test_preprocess_fullsize_1mp():
    """Eight 1024 x 1024 u8 frames of the headline workload, both filters in
    sequence (high-pass, then CLAHE on its output), every pixel against the
    oracle."""
    say("[preprocess] 8 x 1 MP")
    I = np.stack([synth.cfg2_pair(2000 + i)[0] for i in range(8)])
    P = api().Plan(1024, 1024, max_batch=8, workspace=False)
    hp = P.highpass(dev(I, "u8"), radius=7)
    cl = host(P.clahe(hp, tiles=(8, 8), clip_factor=2.0))
    hp = host(hp)
    for i in range(8):
        r1 = oracle.highpass(I[i], 7)
        assert np.array_equal(hp[i].astype(np.int64), r1), i
        assert np.array_equal(cl[i].astype(np.int64), oracle.clahe(r1, 8, 8, 8, 2.0)), i
