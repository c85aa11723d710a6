"""The no-allocation entry point (xcorr_correlate_noalloc) against the
entry point it is a variant of (xcorr_accumulate_dump on a fresh plan), and
against the oracle, through the C ABI.  Two calls in a row share the
library's scratch array; the second has a smaller input and must not see
what the first left there."""
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


def plan_result(x, fmt, flags):
    X = xc()
    n_in = x.shape[2]
    p = X.Plan(n_in, x.shape[0], fmt, "i8", flags=flags)
    out, _ = p.accumulate_dump(x)
    torch.cuda.synchronize()
    p.close()
    return out.cpu().numpy()


CASES = [  # (fmt, first (n_in, n_ch, n_t), second, smaller)
    ("ci4", (512, 40, 700), (192, 9, 130)),
    ("ci4", (256, 33, 4096), (64, 5, 65)),
    ("ci4", (100, 7, 300), (36, 3, 64)),
    ("ci8", (256, 10, 300), (32, 4, 100)),
    ("ci8", (130, 5, 129), (2, 3, 7)),
]


@pytest.mark.parametrize("flags", [0, 0x8, 0x2, 0x4])
@pytest.mark.parametrize("fmt,first,second", CASES, ids=lambda v: str(v))
def test_noalloc_matches_the_plan_entry_point(fmt, first, second, flags):
    X = xc()
    for k, (n_in, n_ch, n_t) in enumerate((first, second)):
        say("noalloc", fmt, (n_in, n_ch, n_t), "flags %#x" % flags, "call", k)
        x = synth.random_input(n_ch, n_t, n_in, fmt, seed=1000 * k + n_in + n_t, device=DEV)
        got = X.correlate_noalloc(x, fmt, flags=flags)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        ref = plan_result(x, fmt, flags)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(got.astype(np.int64), oracle.correlate(x.cpu().numpy(), fmt))


def test_noalloc_refuses_what_it_cannot_run_without_allocating():
    X = xc()
    x = synth.random_input(2, 64, 32, "ci4", seed=1, device=DEV)
    with pytest.raises(X.XcorrError):           # past the int32 fold bound: two launches
        X.correlate_noalloc(torch.zeros((1, 65536, 16), dtype=torch.uint8, device=DEV), "ci4")
    with pytest.raises(X.XcorrError):           # ragged 4-bit row
        X.correlate_noalloc(torch.zeros((1, 8, 6), dtype=torch.uint8, device=DEV), "ci4")
    out = X.correlate_noalloc(x, "ci4")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.correlate(x.cpu().numpy(), "ci4"))
