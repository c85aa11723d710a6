"""Batches: several subarrays of uneven size in one persistent launch per step,
the autotuner and hipGraph-captured steps, checked against the CPU oracle
through the C ABI (int8 path: bit-exact).

Subarray sizes follow the batched-streaming workload (32/96/192/400/704
inputs, 4+4-bit) with channel counts cut down so that the oracle finishes in
seconds; window lengths differ per subarray and are not multiples of 64.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1401_8288_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

SUBS = [(32, 6, 1024), (96, 4, 1999), (192, 3, 3072), (400, 2, 1100), (704, 1, 4095)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def xc():
    from paper_1401_8288_amd import xcorr
    return xcorr


def inputs(subs, fmt="ci4", seed=0):
    return [synth.random_input(c, t, n, fmt, seed=seed + 13 * k + n, device=DEV)
            for k, (n, c, t) in enumerate(subs)]


def oracle_of(xs, fmt="ci4"):
    return [oracle.correlate(x.cpu().numpy(), fmt) for x in xs]


def make(subs, fmt="ci4"):
    X = xc()
    plans = [X.Plan(n, c, fmt, "i8") for (n, c, _) in subs]
    return plans, X.Batch(plans)


def close(plans, batch):
    batch.close()
    for p in plans:
        p.close()


def test_batch_subarrays_match_oracle():
    say("batch: five uneven subarrays")
    xs = inputs(SUBS)
    refs = oracle_of(xs)
    plans, b = make(SUBS)
    outs = [p.new_output() for p in plans]
    infos = b.run(xs, outs)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="subarray %d" % k)
        assert infos[k].samples_accumulated == SUBS[k][2]
    close(plans, b)


def test_batch_equals_single_plans_and_accumulates():
    say("batch: accumulate-only step, then dump without samples")
    xs = inputs(SUBS, seed=5)
    ys = inputs(SUBS, seed=9)
    refs = [a + c for a, c in zip(oracle_of(xs), oracle_of(ys))]
    plans, b = make(SUBS)
    b.run(xs)                                   # accumulate only
    outs = [p.new_output() for p in plans]
    infos = b.run(ys, outs, reset=False)        # accumulate + dump, keep
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="subarray %d" % k)
        assert infos[k].samples_accumulated == SUBS[k][2] * 2
    # a step with no samples for any plan and a dump with reset returns the same
    outs2 = [p.new_output() for p in plans]
    b.run([None] * len(plans), outs2, reset=True)
    torch.cuda.synchronize()
    for o, r in zip(outs2, refs):
        np.testing.assert_array_equal(o.cpu().numpy(), r)
    # after the reset the next dump is zero
    outs3 = [p.new_output() for p in plans]
    b.run([None] * len(plans), outs3, reset=True)
    torch.cuda.synchronize()
    for o in outs3:
        assert int(o.abs().sum()) == 0
    close(plans, b)


def test_batch_mixed_presence():
    say("batch: some plans idle in a step")
    xs = inputs(SUBS, seed=21)
    refs = oracle_of(xs)
    plans, b = make(SUBS)
    step = [x if k % 2 == 0 else None for k, x in enumerate(xs)]
    outs = [p.new_output() if k % 2 == 0 else None for k, p in enumerate(plans)]
    b.run(step, outs)
    torch.cuda.synchronize()
    for k in range(0, len(SUBS), 2):
        np.testing.assert_array_equal(outs[k].cpu().numpy(), refs[k])
    # the idle plans were not touched: their own single run still matches
    for k in range(1, len(SUBS), 2):
        o, _ = plans[k].accumulate_dump(xs[k])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o.cpu().numpy(), refs[k])
    close(plans, b)


def test_every_config_gives_the_same_result_and_autotune_picks_one():
    say("batch: every tile / grid / balance configuration")
    xs = inputs(SUBS, seed=33)
    refs = oracle_of(xs)
    plans, b = make(SUBS)
    for tile in (1, 2, 3):
        for grid in (256, 512, 64):
            for bal in (0, 1):
                b.set_config(tile=tile, grid=grid, balance=bal)
                outs = [p.new_output() for p in plans]
                b.run(xs, outs)
                torch.cuda.synchronize()
                for k, (o, r) in enumerate(zip(outs, refs)):
                    np.testing.assert_array_equal(o.cpu().numpy(), r,
                                                  err_msg="tile %d grid %d balance %d sub %d"
                                                  % (tile, grid, bal, k))
    cfg, ms = b.autotune(xs, reps=2)
    say("autotune chose", cfg, "%.3f ms" % ms)
    assert cfg["tile"] in (1, 2, 3) and cfg["grid"] % 8 == 0 and ms > 0
    assert b.config() == cfg
    outs = [p.new_output() for p in plans]
    b.run(xs, outs)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        np.testing.assert_array_equal(o.cpu().numpy(), r)
    close(plans, b)


def test_graph_replays_match_eager():
    say("batch: captured step replayed with eager work between replays")
    X = xc()
    xs = inputs(SUBS, seed=41)
    refs = oracle_of(xs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plans = [X.Plan(n, c, "ci4", "i8", stream=s) for (n, c, _) in SUBS]
        b = X.Batch(plans, stream=s)
        outs = [p.new_output() for p in plans]
    torch.cuda.synchronize()
    g = b.capture(xs, outs)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="replay %d sub %d" % (rep, k))
        # eager work on the same plans' data between replays
        junk = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device=DEV).sum()
        torch.cuda.synchronize()
        assert int(junk) >= 0
    g.close()
    close(plans, b)


def test_batch_register_staged_and_ci8():
    say("batch: n_inputs not a multiple of 16 (register staging), rows zero padded, and 8-bit samples")
    for subs, fmt in (([(36, 3, 300), (100, 2, 129), (16, 5, 64)], "ci4"),
                      ([(36, 3, 300), (100, 2, 129), (16, 5, 64)], "ci8"),
                      ([(6, 3, 300), (66, 2, 129), (514, 1, 64)], "ci4"),
                      ([(5, 3, 300), (33, 2, 129)], "ci8")):
        xs = inputs(subs, fmt=fmt, seed=51)
        refs = oracle_of(xs, fmt)
        plans, b = make(subs, fmt)
        outs = [p.new_output() for p in plans]
        b.run(xs, outs)
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="%s sub %d" % (fmt, k))
        close(plans, b)


@pytest.mark.parametrize("tile", [0, 2])
def test_batch_8bit_lds_dma(tile):
    # 8-bit plans whose rows are a multiple of 16 inputs (200 inputs are
    # staged zero padded to 208) run the LDS-DMA kernel together, full value
    # range, one of them over two chunks (70000 samples)
    say("batch: 8-bit LDS-DMA, tile", tile)
    subs = [(64, 3, 300), (256, 2, 129), (16, 5, 64), (200, 1, 77), (32, 2, 70000)]
    xs = [synth.random_input(c, t, n, "ci8", seed=81 + k, lo=-128, hi=127, device=DEV)
          for k, (n, c, t) in enumerate(subs)]
    refs = oracle_of(xs, "ci8")
    plans, b = make(subs, "ci8")
    if tile:
        b.set_config(tile=tile, grid=b.config()["grid"], balance=0)
    outs = [p.new_output() for p in plans]
    b.run(xs, outs)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="sub %d" % k)
    close(plans, b)


def test_batch_more_entries_than_one_launch_holds():
    say("batch: 60 plans (two launches per step; a batch holds up to 64)")
    subs = [(4 * (1 + k % 5), 1 + k % 3, 64 + 7 * k) for k in range(60)]
    xs = inputs(subs, seed=61)
    refs = oracle_of(xs)
    plans, b = make(subs)
    outs = [p.new_output() for p in plans]
    b.run(xs, outs)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="sub %d" % k)
    close(plans, b)


def test_batch_window_longer_than_fold_bound():
    say("batch: 70000-sample window (two chunks) next to a short one")
    subs = [(16, 2, 70000), (32, 1, 500)]
    xs = [synth.constant_input(2, 70000, 16, "ci4", -8, -8, device=DEV),
          synth.random_input(1, 500, 32, "ci4", seed=71, device=DEV)]
    refs = oracle_of(xs)
    plans, b = make(subs)
    outs = [p.new_output() for p in plans]
    b.run(xs, outs)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        np.testing.assert_array_equal(o.cpu().numpy(), r)
    assert int(refs[0][0, 0, 0]) == 70000 * 128
    close(plans, b)


def test_batch_errors():
    X = xc()
    p1 = X.Plan(32, 2, "ci4", "i8")
    p2 = X.Plan(32, 2, "ci8", "i8")
    p3 = X.Plan(32, 2, "ci4", "f32")
    with pytest.raises(X.XcorrError):
        X.Batch([p1, p2])            # mixed formats
    with pytest.raises(X.XcorrError):
        X.Batch([p3])                # not the int8 path
    with pytest.raises(X.XcorrError):
        X.Batch([p1, p1])            # same plan twice
    b = X.Batch([p1])
    with pytest.raises(X.XcorrError):
        b.set_config(tile=1, grid=12, balance=0)   # grid not a multiple of 8
    x = synth.random_input(2, 64, 32, "ci4", seed=1, device=DEV)
    b.run([x])
    with pytest.raises(X.XcorrError):
        b.autotune([x])             # plan not freshly reset
    b.close()
    for p in (p1, p2, p3):
        p.close()


def test_graph_launch_after_a_plan_was_destroyed_is_refused():
    # a replay writes every plan's bookkeeping; once a plan is gone the
    # launch must fail before anything is enqueued
    say("batch: graph launch after destroying one of its plans")
    X = xc()
    subs = [(32, 2, 128), (64, 1, 200)]
    xs = inputs(subs, seed=81)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plans = [X.Plan(n, c, "ci4", "i8", stream=s) for (n, c, _) in subs]
        b = X.Batch(plans, stream=s)
        outs = [p.new_output() for p in plans]
    torch.cuda.synchronize()
    g = b.capture(xs, outs)
    g.launch()
    s.synchronize()
    plans[1].close()
    with pytest.raises(X.XcorrError) as ei:
        g.launch()
    assert ei.value.status == -4
    g.close()
    b.close()
    plans[0].close()


def test_work_queue_counters_survive_changes_of_launch_configuration():
    # every persistent launch takes items from the same per-XCD counters and
    # the last workgroup of each launch zeroes them: launches of different
    # grids, slice balances and XCD maps on one counter set, back to back,
    # must each cover all of their items
    say("batch: alternating persistent launch configurations on one counter set")
    X = xc()
    xs = inputs(SUBS[:3], seed=91)
    refs = oracle_of(xs)
    plans, b = make(SUBS[:3])
    outs = [p.new_output() for p in plans]
    configs = [(0, 512, 1), (2, 256, 0), (1, 256, 1), (0, 1024, 0), (3, 512, 1), (0, 256, 1)]
    for cfg in configs:
        b.set_config(*cfg)
        for o in outs:
            o.fill_(-1)
        b.run(xs, outs)
        for (n, c, t), x, r in zip(SUBS[:3], xs, refs):
            # a single plan on the same stream between the batch steps
            p = X.Plan(n, c, "ci4", "i8")
            got, _ = p.accumulate_dump(x)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy(), r, err_msg="single plan after config %s" % (cfg,))
            p.close()
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg="config %s sub %d" % (cfg, k))
    close(plans, b)
    # the same counters of one plan: persistent launches with and without the
    # XCD map, one workgroup per item, then persistent again
    x = xs[2]
    n, c, t = SUBS[2]
    for flags in (0, X.FLAG_NO_XCD_MAP, X.FLAG_NO_PERSIST, X.FLAG_NO_XCD_MAP | X.FLAG_OUT_I32, 0):
        p = X.Plan(n, c, "ci4", "i8", flags=flags)
        for rep in range(2):
            got, _ = p.accumulate_dump(x)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy().astype(np.int64), refs[2],
                                          err_msg="flags %#x rep %d" % (flags, rep))
        p.close()
