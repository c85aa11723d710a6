"""The streaming server: admission by device memory, continuous batching, and
each window's result the same alone and in the mix (int8 path: bit-exact, so
"the same" means identical), checked against the CPU oracle."""
import sys
import threading
import time

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


def windows(n_in, n_ch, lens, fmt="ci4", seed=0):
    xs = [synth.random_input(n_ch, t, n_in, fmt, seed=seed + 17 * k + n_in, device=DEV)
          for k, t in enumerate(lens)]
    torch.cuda.synchronize()
    return xs


A = (96, 8, [1024, 1999, 4096])      # the stream whose results must not depend on the mix


def run_alone(xs):
    X = xc()
    with X.Server(device_budget=1 << 30, max_streams=4) as srv:
        sid = srv.open(A[0], A[1])
        outs = [srv.new_output(sid) for _ in xs]
        ts = [srv.submit(sid, x, o) for x, o in zip(xs, outs)]
        for t in ts:
            srv.wait(t)
        st = srv.stats()
    return [o.cpu().numpy() for o in outs], st


def test_server_alone_matches_oracle():
    say("server: one stream alone")
    xs = windows(A[0], A[1], A[2], seed=1)
    got, st = run_alone(xs)
    for g, x in zip(got, xs):
        np.testing.assert_array_equal(g, oracle.correlate(x.cpu().numpy(), "ci4"))
    assert st["windows_done"] == 3
    assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]


def test_server_same_alone_and_in_the_mix():
    say("server: the same stream alone and among others submitted from two threads")
    X = xc()
    xs = windows(A[0], A[1], A[2], seed=1)
    alone, _ = run_alone(xs)
    others = [(32, 16, [777, 2048, 1500], "ci4"), (400, 2, [1024, 640], "ci4"),
              (36, 5, [300, 1000], "ci4"), (64, 4, [512, 900], "ci8")]
    other_x = [windows(n, c, lens, fmt, seed=100 + i) for i, (n, c, lens, fmt) in enumerate(others)]
    with X.Server(device_budget=1 << 31, max_streams=8, max_inflight=2) as srv:
        sa = srv.open(A[0], A[1])
        sids = [srv.open(n, c, fmt) for (n, c, _, fmt) in others]
        outs_a = [srv.new_output(sa) for _ in xs]
        outs_o = [[srv.new_output(s) for _ in w] for s, w in zip(sids, other_x)]
        tickets = []
        lock = threading.Lock()

        def feed_others():
            for k in range(3):
                for s, w, o in zip(sids, other_x, outs_o):
                    if k < len(w):
                        t = srv.submit(s, w[k], o[k])
                        with lock:
                            tickets.append(t)
                time.sleep(0.001)

        th = threading.Thread(target=feed_others)
        th.start()
        for x, o in zip(xs, outs_a):
            t = srv.submit(sa, x, o)
            with lock:
                tickets.append(t)
            time.sleep(0.002)
        th.join()
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
        say("mixed stats", st)
        for g, o in zip(alone, outs_a):
            np.testing.assert_array_equal(o.cpu().numpy(), g)
        for (n, c, lens, fmt), w, o in zip(others, other_x, outs_o):
            for xk, ok in zip(w, o):
                np.testing.assert_array_equal(ok.cpu().numpy(), oracle.correlate(xk.cpu().numpy(), fmt))
        assert st["windows_done"] == len(tickets)
        assert st["launches"] <= len(tickets)


def test_server_admits_by_memory():
    say("server: admission by device memory")
    X = xc()
    need = X.plan_bytes(64, 32, "ci4", "i8")
    xs = [windows(64, 32, [256, 256], seed=200 + k) for k in range(3)]
    with X.Server(device_budget=2 * need + need // 2, max_streams=8) as srv:
        sids = [srv.open(64, 32) for _ in range(3)]
        deadline = time.time() + 10
        while srv.stats()["streams_admitted"] < 2 and time.time() < deadline:
            time.sleep(0.01)
        st = srv.stats()
        assert st["streams_admitted"] == 2 and st["streams_waiting"] == 1
        assert st["device_bytes"] <= 2 * need + need // 2
        outs = [[srv.new_output(s) for _ in range(2)] for s in sids]
        ts = [[srv.submit(s, x, o) for x, o in zip(w, ow)] for s, w, ow in zip(sids, xs, outs)]
        for t in ts[0] + ts[1]:
            srv.wait(t)
        time.sleep(0.2)
        assert not any(srv.poll(t)[0] for t in ts[2])     # third stream still waiting
        srv.close_stream(sids[0])
        for t in ts[2]:
            srv.wait(t)
        st = srv.stats()
        assert st["device_bytes"] <= 2 * need + need // 2
        for w, ow in zip(xs, outs):
            for x, o in zip(w, ow):
                np.testing.assert_array_equal(o.cpu().numpy(), oracle.correlate(x.cpu().numpy(), "ci4"))


def test_server_errors():
    X = xc()
    with pytest.raises(X.XcorrError):
        X.Server(device_budget=0)
    with X.Server(device_budget=1 << 20, max_streams=2) as srv:
        with pytest.raises(X.XcorrError):
            srv.open(512, 4096)                 # can never fit the budget
        with pytest.raises(KeyError):
            srv.open(64, 4, "ci9")              # unknown format
        sid = srv.open(16, 2)
        x = windows(16, 2, [64])[0]
        o = srv.new_output(sid)
        t = srv.submit(sid, x, o)
        srv.wait(t)
        srv.close_stream(sid)
        with pytest.raises(X.XcorrError):
            srv.submit(sid, x, o)               # closed stream
        with pytest.raises(X.XcorrError):
            srv.poll(10 ** 9)                   # unknown ticket


def test_server_batches_several_windows_of_a_stream_and_tunes(tmp_path):
    # windows submitted in bursts: one launch takes several windows of the
    # same stream (each its own fused window); the online tuner times every
    # candidate configuration on those launches, settles, and writes the
    # settled configuration to its cache file, which a second server reads
    # back (it starts with the mix tuned); every result is the oracle's
    say("server: bursts of windows, online tuning, tuning cache")
    X = xc()
    path = str(tmp_path / "tune.txt")
    shapes = [(32, 6, 1024), (66, 3, 700), (128, 2, 1500)]
    data = [windows(n, c, [t] * 4, seed=90 + n) for (n, c, t) in shapes]
    refs = [[oracle.correlate(x.cpu().numpy(), "ci4") for x in xs] for xs in data]
    with X.Server(device_budget=1 << 30, max_streams=8, max_inflight=1, tune_path=path) as srv:
        sids = [srv.open(n, c) for (n, c, _) in shapes]
        for rep in range(20):
            outs, tks = [], []
            for sid, xs in zip(sids, data):
                for x in xs:
                    o = srv.new_output(sid)
                    outs.append(o)
                    tks.append(srv.submit(sid, x, o))
            for t in tks:
                srv.wait(t)
            k = 0
            for si, xs in enumerate(data):
                for j in range(len(xs)):
                    np.testing.assert_array_equal(outs[k].cpu().numpy(), refs[si][j],
                                                  err_msg="rep %d stream %d window %d" % (rep, si, j))
                    k += 1
        st = srv.stats()
    assert st["mean_batch"] > 1.5, st
    assert st["mixes_tuned"] >= 1, st
    lines = open(path).read().split("\n")
    assert any(l.strip() for l in lines)
    with X.Server(device_budget=1 << 30, max_streams=8, tune_path=path) as srv:
        assert srv.stats()["mixes_tuned"] >= 1


def test_server_deadlines_order_and_count():
    # earliest deadline first: a stream with tight deadlines beside one
    # without; results stay the oracle's, and misses are counted against the
    # deadlines (none are possible at a generous period, every window misses
    # an impossible one)
    say("server: deadlines")
    X = xc()
    big = windows(256, 16, [4096] * 3, seed=71)
    small = windows(32, 4, [1024] * 6, seed=72)
    rb = [oracle.correlate(x.cpu().numpy(), "ci4") for x in big]
    rs = [oracle.correlate(x.cpu().numpy(), "ci4") for x in small]
    for period, expect in ((10.0, "none"), (1e-12, "all")):
        with X.Server(device_budget=1 << 32, max_streams=4, max_inflight=1) as srv:
            sb, ss = srv.open(256, 16), srv.open(32, 4)
            srv.set_deadline(ss, period)
            ob = [srv.new_output(sb) for _ in big]
            os_ = [srv.new_output(ss) for _ in small]
            tks = [srv.submit(sb, x, o) for x, o in zip(big, ob)] + [srv.submit(ss, x, o) for x, o in zip(small, os_)]
            for t in tks:
                srv.wait(t)
            st = srv.stats()
        for o, r in zip(ob, rb):
            np.testing.assert_array_equal(o.cpu().numpy(), r)
        for o, r in zip(os_, rs):
            np.testing.assert_array_equal(o.cpu().numpy(), r)
        if expect == "none":
            assert st["deadline_misses"] == 0, st
        else:
            assert st["deadline_misses"] == len(small), st
