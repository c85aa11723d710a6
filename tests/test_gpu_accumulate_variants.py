"""Pulsar gating and baseline-dependent integration (the paper's planned
accumulate variants) against the CPU oracle: each gate's result is the
visibility of exactly its samples; a tile dump returns exactly the selected
baselines and restarts only them."""
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


def pulsar_gates(n_t, period, phase=0):
    """Gate of each sample: 1 on the pulse (first 9 % of the period), 2 on its
    trailing edge, 255 (discarded) just after it, 0 elsewhere."""
    g = np.zeros(n_t, dtype=np.uint8)
    for t in range(n_t):
        ph = (t + phase) % period
        if ph < 0.09 * period:
            g[t] = 1
        elif ph < 0.15 * period:
            g[t] = 2
        elif ph < 0.20 * period:
            g[t] = 255
    return g


@pytest.mark.parametrize("n_in,fmt", [(96, "ci4"), (36, "ci4"), (64, "ci8"), (6, "ci4"), (171, "ci4"),
                                      (7, "ci8")])
def test_gated_accumulation_matches_oracle(n_in, fmt):
    say("gating", n_in, fmt)
    X = xc()
    n_ch, n_t = 5, 3000
    x1 = synth.random_input(n_ch, n_t, n_in, fmt, seed=n_in + 1, device=DEV)
    x2 = synth.random_input(n_ch, n_t, n_in, fmt, seed=n_in + 2, device=DEV)
    g1 = pulsar_gates(n_t, 700)
    g2 = pulsar_gates(n_t, 700, phase=n_t)
    plans = [X.Plan(n_in, n_ch, fmt, "i8") for _ in range(3)]
    X.accumulate_gated(plans, x1, g1)
    X.accumulate_gated(plans, x2, g2)
    a1, a2 = x1.cpu().numpy(), x2.cpu().numpy()
    for k, p in enumerate(plans):
        out, info = p.dump()
        torch.cuda.synchronize()
        ref = oracle.correlate(a1[:, g1 == k], fmt) + oracle.correlate(a2[:, g2 == k], fmt)
        np.testing.assert_array_equal(out.cpu().numpy(), ref, err_msg="gate %d" % k)
        assert info.samples_accumulated == int((g1 == k).sum() + (g2 == k).sum())
        p.close()


@pytest.mark.parametrize("fmt,flags,tile", [("ci4", 0, 0), ("ci8", 0, 0), ("ci4", "np", 0), ("ci4", 0, 3),
                                             ("ci4", "i32", 0)])
def test_gates_read_listed_rows_or_a_packed_copy(fmt, flags, tile):
    # persistent depth-4 LDS-DMA plans copy each gate's rows straight from
    # the window through the gate's row list, in launches of at most 8192
    # (4-bit) or 4096 (8-bit) rows; other plans (no persistent launch, the
    # register tile) read a packed copy.  A 20000-sample window whose first
    # gate takes most samples makes several row-list launches.  The results
    # are the oracle's either way.
    X = xc()
    fl = {0: 0, "np": X.FLAG_NO_PERSIST, "i32": X.FLAG_OUT_I32}[flags]
    say("gating: listed rows", fmt, flags, tile)
    n_in, n_ch, n_t = 64, 3, 20000
    x = synth.random_input(n_ch, n_t, n_in, fmt, seed=41, lo=-128 if fmt == "ci8" else -8,
                           hi=127 if fmt == "ci8" else 7, device=DEV)
    g = np.where(np.arange(n_t) % 7 == 3, 1, 0).astype(np.uint8)
    g[np.arange(n_t) % 11 == 5] = 255
    plans = [X.Plan(n_in, n_ch, fmt, "i8", flags=fl, tile=tile) for _ in range(2)]
    X.accumulate_gated(plans, x, g)
    a = x.cpu().numpy()
    for k, p in enumerate(plans):
        out, info = p.dump()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), oracle.correlate(a[:, g == k], fmt),
                                      err_msg="gate %d" % k)
        assert info.samples_accumulated == int((g == k).sum())
        p.close()


def test_gates_may_run_different_paths():
    # CI4 products summed over 3000 samples stay below 2^24: the float paths
    # are exact here
    say("gating across paths")
    X = xc()
    n_ch, n_t, n_in = 3, 3000, 40
    x = synth.random_input(n_ch, n_t, n_in, "ci4", seed=8, device=DEV)
    g = pulsar_gates(n_t, 256)
    plans = [X.Plan(n_in, n_ch, "ci4", path) for path in ("f32", "i8", "f16")]
    X.accumulate_gated(plans, x, g)
    a = x.cpu().numpy()
    for k, p in enumerate(plans):
        out, _ = p.dump()
        torch.cuda.synchronize()
        ref = oracle.correlate(a[:, g == k], "ci4")
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref.astype(got.dtype), err_msg="gate %d" % k)
        p.close()


def test_gating_with_every_sample_in_one_gate_equals_plain_accumulation():
    X = xc()
    x = synth.random_input(3, 1000, 128, "ci4", seed=5, device=DEV)
    p0, p1 = X.Plan(128, 3, "ci4", "i8"), X.Plan(128, 3, "ci4", "i8")
    X.accumulate_gated([p0, p1], x, np.ones(1000, dtype=np.uint8))
    out1, _ = p1.dump()
    out0, _ = p0.dump()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out1.cpu().numpy(), oracle.correlate(x.cpu().numpy(), "ci4"))
    assert int(out0.abs().sum()) == 0
    with pytest.raises(X.XcorrError):
        X.accumulate_gated([p0, p1], x, np.full(1000, 2, dtype=np.uint8))   # gate out of range


def test_gating_that_discards_every_sample_leaves_the_gates_empty():
    X = xc()
    x = synth.random_input(2, 400, 64, "ci4", seed=6, device=DEV)
    plans = [X.Plan(64, 2, "ci4", "i8") for _ in range(2)]
    X.accumulate_gated(plans, x, np.full(400, 255, dtype=np.uint8))
    for p in plans:
        out, info = p.dump()
        torch.cuda.synchronize()
        assert int(out.abs().sum()) == 0 and info.samples_accumulated == 0
        p.close()


def tile_of(n_in):
    nr = (n_in + 63) // 64
    rows, cols = np.tril_indices(n_in)
    return (rows // 64) * (rows // 64 + 1) // 2 + cols // 64, nr * (nr + 1) // 2


def test_tile_dump_restarts_only_the_selected_tiles():
    say("baseline-dependent integration")
    X = xc()
    n_in, n_ch = 160, 4                                     # 3 row blocks: 6 tiles
    xa = synth.random_input(n_ch, 500, n_in, "ci4", seed=21, device=DEV)
    xb = synth.random_input(n_ch, 300, n_in, "ci4", seed=22, device=DEV)
    va = oracle.correlate(xa.cpu().numpy(), "ci4")
    vb = oracle.correlate(xb.cpu().numpy(), "ci4")
    tri_tile, n_tiles = tile_of(n_in)
    sel = np.zeros(n_tiles, dtype=np.uint8)
    sel[[1, 5]] = 1                                         # tiles (1,0) and (2,2)
    chosen = np.isin(tri_tile, np.nonzero(sel)[0])
    p = X.Plan(n_in, n_ch, "ci4", "i8")
    p.accumulate(xa)
    out = torch.full(p.out_shape(), -1, dtype=torch.int64, device=DEV)
    p.dump_tiles(out, sel, reset=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    np.testing.assert_array_equal(o[:, chosen], va[:, chosen])
    assert (o[:, ~chosen] == -1).all()                     # untouched
    p.accumulate(xb)
    full, _ = p.dump(reset=True)
    torch.cuda.synchronize()
    f = full.cpu().numpy()
    np.testing.assert_array_equal(f[:, chosen], vb[:, chosen])
    np.testing.assert_array_equal(f[:, ~chosen], (va + vb)[:, ~chosen])
    # without reset the selected tiles keep integrating
    p.accumulate(xa)
    out2 = torch.zeros(p.out_shape(), dtype=torch.int64, device=DEV)
    p.dump_tiles(out2, np.ones(n_tiles, dtype=np.uint8), reset=False)
    p.accumulate(xb)
    full2, _ = p.dump()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out2.cpu().numpy(), va)
    np.testing.assert_array_equal(full2.cpu().numpy(), va + vb)
    p.close()
