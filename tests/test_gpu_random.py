"""Randomised parity sweep: seeded random shapes, formats, tiles, launch
flags and output widths through the C ABI, each against the CPU oracle
(int8 path bit-exact).  Shapes are small so that the whole sweep takes
seconds; the case list is fixed by the seed, so a failure names a case that
can be run again on its own."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1401_8288_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def cases(n=48, seed=2024):
    g = np.random.default_rng(seed)
    out = []
    for k in range(n):
        fmt = "ci4" if g.random() < 0.5 else "ci8"
        step = 4 if fmt == "ci4" else 2
        n_in = int(g.integers(1, 80)) * step
        if g.random() < 0.4:
            n_in = int(g.integers(1, 20)) * 16          # LDS-DMA shapes
        n_ch = int(g.integers(1, 7))
        n_t = int(g.integers(1, 300))
        tile = int(g.choice([0, 2, 3]))
        flags = int(g.choice([0, 0x4, 0x8, 0xC, 0x2]))  # NO_PERSIST, OUT_I32, both, NO_XCD_MAP
        out.append((k, fmt, n_in, n_ch, n_t, tile, flags))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: "c%d-%s-%dx%dx%d-t%d-f%x" % c)
def test_random_case(case):
    from paper_1401_8288_amd import xcorr
    k, fmt, n_in, n_ch, n_t, tile, flags = case
    print("random case", case, file=sys.stderr, flush=True)
    if tile == 2 and n_in % 16:
        tile = 0                                        # LDS-DMA needs n_inputs % 16 == 0
    lo, hi = (-8, 7) if fmt == "ci4" else (-128, 127)
    x = synth.random_input(n_ch, n_t, n_in, fmt, seed=1000 + k, lo=lo, hi=hi, device=DEV)
    p = xcorr.Plan(n_in, n_ch, fmt, "i8", flags=flags, tile=tile)
    out, info = p.accumulate_dump(x)
    torch.cuda.synchronize()
    p.close()
    assert info.samples_accumulated == n_t
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), oracle.correlate(x.cpu().numpy(), fmt))
