"""int32 output (XCORR_FLAG_OUT_I32) of the int8 path against the CPU oracle:
bit-exact for every window of at most fold_bound (65535) samples, for both
formats, including the largest sums the 8-bit format can make; windows past
the bound are refused and change nothing."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1401_8288_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def xc():
    from paper_1401_8288_amd import xcorr
    return xcorr


SHAPES = [(4, 3, 1), (36, 5, 100), (64, 9, 129), (100, 2, 129), (192, 2, 65), (256, 2, 200), (516, 1, 70)]


@pytest.mark.parametrize("tile", [0, 1, 3])
@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_int32_output_matches_the_oracle(shape, fmt, tile):
    n_in, n_ch, n_t = shape
    if tile == 1 and (fmt != "ci4" or n_in % 16):
        pytest.skip("LDS-DMA tile needs 4-bit samples and n_inputs % 16 == 0")
    X = xc()
    say("int32 out", shape, fmt, tile)
    x = synth.random_input(n_ch, n_t, n_in, fmt, seed=n_in + n_t, device=DEV)
    p = X.Plan(n_in, n_ch, fmt, "i8", flags=X.FLAG_OUT_I32, tile=tile)
    out, info = p.accumulate_dump(x)
    torch.cuda.synchronize()
    assert out.dtype == torch.int32
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy(), fmt))
    p.close()


def test_largest_8bit_sums_at_the_window_bound():
    # (-128, -128) and (127, -128) for 65535 samples: Re of the first auto is
    # 65535 * 2 * 128^2 = 2147450880 and Im of their cross product
    # 65535 * (128^2 + 127 * 128) = 2139062400, both just inside int32
    X = xc()
    n_t = 65535
    re = torch.tensor([-128, 127, -128, 127], dtype=torch.int32)
    im = torch.tensor([-128, -128, 127, 127], dtype=torch.int32)
    x = torch.stack([re, im], dim=-1).to(torch.int8)[None, None].expand(1, n_t, 4, 2).contiguous().to(DEV)
    p = X.Plan(4, 1, "ci8", "i8", flags=X.FLAG_OUT_I32)
    out, info = p.accumulate_dump(x)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.int64)
    ref = oracle.correlate(x.cpu().numpy(), "ci8")
    np.testing.assert_array_equal(got, ref)
    assert ref.max() == 2147450880 and abs(ref[0, 1, 1]) == 2139062400
    p.close()


def test_windows_past_the_bound_are_refused():
    X = xc()
    x = synth.random_input(2, 40000, 32, "ci4", seed=1, device=DEV)
    p = X.Plan(32, 2, "ci4", "i8", flags=X.FLAG_OUT_I32)
    p.accumulate(x)
    with pytest.raises(X.XcorrError):
        p.accumulate(x)                       # 80000 samples in one window
    out, info = p.dump(reset=True)
    torch.cuda.synchronize()
    assert info.samples_accumulated == 40000
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy(), "ci4"))
    out2, info2 = p.accumulate_dump(x)        # a new window is fine
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out2.cpu().numpy(), out.cpu().numpy())
    p.close()


def test_mixed_output_widths_in_one_batch():
    X = xc()
    subs = [(32, 3, 1000), (96, 2, 777), (64, 4, 1500)]
    xs = [synth.random_input(c, t, n, "ci4", seed=n, device=DEV) for n, c, t in subs]
    plans = [X.Plan(n, c, "ci4", "i8", flags=X.FLAG_OUT_I32 if k % 2 == 0 else 0) for k, (n, c, t) in enumerate(subs)]
    b = X.Batch(plans)
    outs = [p.new_output() for p in plans]
    b.run(xs, outs)
    torch.cuda.synchronize()
    for k, (x, o) in enumerate(zip(xs, outs)):
        assert o.dtype == (torch.int32 if k % 2 == 0 else torch.int64)
        np.testing.assert_array_equal(o.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy(), "ci4"))
    b.close()
    for p in plans:
        p.close()


def test_int32_tile_dump_and_gating():
    X = xc()
    n_in, n_ch = 160, 3
    xa = synth.random_input(n_ch, 500, n_in, "ci4", seed=3, device=DEV)
    p = X.Plan(n_in, n_ch, "ci4", "i8", flags=X.FLAG_OUT_I32)
    p.accumulate(xa)
    sel = [1, 0, 1, 0, 0, 1]
    out = torch.zeros(p.out_shape(), dtype=torch.int32, device=DEV)
    p.dump_tiles(out, sel, reset=True)
    full, _ = p.dump()
    torch.cuda.synchronize()
    ref = oracle.correlate(xa.cpu().numpy(), "ci4")
    rows, cols = np.tril_indices(n_in)
    tile = (rows // 64) * (rows // 64 + 1) // 2 + cols // 64
    on = np.isin(tile, np.nonzero(sel)[0])
    np.testing.assert_array_equal(out.cpu().numpy()[:, on].astype(np.int64), ref[:, on])
    assert (out.cpu().numpy()[:, ~on] == 0).all()
    np.testing.assert_array_equal(full.cpu().numpy()[:, ~on].astype(np.int64), ref[:, ~on])
    assert (full.cpu().numpy()[:, on] == 0).all()
    p.close()
    g = np.array([t % 3 for t in range(900)], dtype=np.uint8)
    x = synth.random_input(2, 900, 64, "ci4", seed=4, device=DEV)
    plans = [X.Plan(64, 2, "ci4", "i8", flags=X.FLAG_OUT_I32) for _ in range(3)]
    X.accumulate_gated(plans, x, g)
    a = x.cpu().numpy()
    for k, q in enumerate(plans):
        o, _ = q.dump()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o.cpu().numpy().astype(np.int64), oracle.correlate(a[:, g == k], "ci4"))
        q.close()
