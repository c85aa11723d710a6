"""GPU corner turn (F-engine packets -> X-stage input) against the oracle,
bit-exact, and the X-stage fed by it."""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def xc():
    from paper_1401_8288_amd import xcorr
    return xcorr


CASES = [  # (B, F, J, C, S): tiles of many channels, ragged channel tiles, one-channel tiles
    (3, 4, 4, 5, 2), (5, 8, 16, 67, 4), (2, 16, 32, 9, 16), (4, 64, 64, 3, 16), (7, 2, 8, 130, 1)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
@pytest.mark.parametrize("fmt", ["ci4", "ci8"])
def test_corner_turn_matches_oracle(case, fmt):
    B, F, J, C, S = case
    say("corner turn", case, fmt)
    g = np.random.default_rng(sum(case))
    packets = g.integers(0, 256, size=(B, F, S, C, J), dtype=np.uint8)
    valid = (g.random((B, F)) > 0.2).astype(np.uint8)
    valid[0, 0] = 1
    ref = oracle.corner_turn(packets, F, J, C, S, valid=valid, out_fmt=fmt)
    got = xc().corner_turn(torch.from_numpy(packets).to(DEV), F, J, C, S,
                           valid=torch.from_numpy(valid).to(DEV), out_fmt=fmt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), ref)
    # all packets received
    ref2 = oracle.corner_turn(packets, F, J, C, S, out_fmt=fmt)
    got2 = xc().corner_turn(torch.from_numpy(packets).to(DEV), F, J, C, S, out_fmt=fmt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got2.cpu().numpy(), ref2)


def test_corner_turn_feeds_the_x_stage():
    say("corner turn -> X-stage")
    X = xc()
    B, F, J, C, S = 16, 8, 16, 6, 8           # 128 inputs, 128 samples
    g = np.random.default_rng(7)
    packets = g.integers(0, 256, size=(B, F, S, C, J), dtype=np.uint8)
    valid = np.ones((B, F), dtype=np.uint8)
    valid[3, 5] = 0
    ref = oracle.correlate(oracle.corner_turn(packets, F, J, C, S, valid=valid), "ci4")
    dp, dv = torch.from_numpy(packets).to(DEV), torch.from_numpy(valid).to(DEV)
    for fmt in ("ci4", "ci8"):
        x = X.corner_turn(dp, F, J, C, S, valid=dv, out_fmt=fmt)
        got = X.correlate(x, fmt, "i8")
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref)


def test_corner_turn_errors():
    X = xc()
    p = torch.zeros(64, dtype=torch.uint8, device=DEV)
    with pytest.raises(X.XcorrError):
        X.corner_turn(p, 2, 2, 4, 4)       # inputs_per_feng not a multiple of 4
    with pytest.raises(ValueError):
        X.corner_turn(p, 3, 4, 5, 1)       # not a whole number of blocks
